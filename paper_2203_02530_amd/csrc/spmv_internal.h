// Internal declarations of the SpMV library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "spmv.h"

namespace spmv {

// ----------------------------------------------------------------- errors
// Thread-local message behind spmv_last_error(); set_error returns `code` so
// call sites can `return set_error(...)`.
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
void clear_error();

#define SPMV_HIP(call)                                                    \
    do {                                                                  \
        hipError_t e__ = (call);                                          \
        if (e__ != hipSuccess) return ::spmv::hip_error(e__, #call);      \
    } while (0)

// ----------------------------------------------------------------- share
// One rank's share of the global matrix (Sec. III-A), host side.
struct Share {
    int64_t n_global = 0, lo = 0, n_loc = 0;
    int32_t nranks = 1, rank = 0;
    // A_L: local columns renumbered to col - lo
    std::vector<int32_t> L_ptr, L_col;
    std::vector<double> L_val;
    // A_R over the rows that have remote entries; columns index the halo
    std::vector<int32_t> R_rows, R_ptr, R_col;
    std::vector<double> R_val;
    // halo: ascending global columns; recv_off[q] .. recv_off[q+1] owned by q
    std::vector<int32_t> halo, recv_off;
    // send lists: local indices each destination needs, dest ascending
    std::vector<int32_t> send_idx, send_off;
    // x_halo[p] = recv[perm[p]]; identity under the layout above
    std::vector<int32_t> unpack_perm;
};

int validate_csr(const spmv_csr_t *csr);
int64_t block_lo(int64_t n, int32_t P, int32_t q);
int build_share(const spmv_csr_t *csr, int32_t nranks, int32_t rank, Share &out);
// From the rank's own rows (global columns) and its send lists.
int build_share_local(const spmv_csr_t *local, int64_t n_global, int32_t nranks, int32_t rank,
                      const int32_t *send_idx, const int32_t *send_off, Share &out);

// ----------------------------------------------------------------- DAG
enum class VType : uint8_t { CPU, GPU };
VType vertex_type(int32_t v);
bool is_vertex(int32_t tok);
bool is_sync(int32_t tok);
inline int32_t sync_kind(int32_t tok) { return tok & 0x30; }
inline int32_t sync_operand(int32_t tok) { return tok & 0x0f; }

// A validated, canonical plan: order of tokens, canonical stream per vertex
// (-1 for CPU vertices), explicit or implied Unpack.
struct Schedule {
    std::vector<int32_t> order;            // as given (Unpack inserted if implied)
    int32_t stream[SPMV_N_VERTICES];        // canonical stream of GPU vertices
    int32_t n_streams_used = 0;
    bool unpack_implied = false;
    bool multi = false;                     // nranks > 1
};

int validate_schedule(int32_t nranks, const int32_t *ops, int32_t n_ops,
                      const int32_t *stream_map, int32_t n_streams, Schedule &out);
void default_order(int32_t nranks, std::vector<int32_t> &ops, int32_t *stream_map);
int op_name(int32_t tok, std::string &out);

// Plan-space enumeration (cached per (multi, n_streams)).
struct PlanEntry {
    std::vector<int32_t> order;
    int32_t stream[SPMV_N_VERTICES];
};
const std::vector<PlanEntry> &plan_space(bool multi, int32_t n_streams);
// Index of a complete plan in plan_space(multi, n_streams), -1 if absent.
int64_t plan_index(bool multi, int32_t n_streams, const std::vector<int32_t> &order,
                   const int32_t *stream);

// A program prefix P_k built one token at a time (Sec. III-B): next() lists
// the tokens that may follow -- DAG vertices whose predecessors are placed
// and Table III tokens whose operands are placed, GPU vertices once per
// canonical stream -- in ascending token code, then stream.
struct Prefix {
    struct Step {
        int32_t token, stream;   // stream -1 for CPU vertices and sync tokens
    };
    bool multi = true;
    int32_t n_streams = 1;
    std::vector<int32_t> tokens;            // the token universe, ascending
    std::vector<int32_t> order;             // placed tokens
    int32_t stream[SPMV_N_VERTICES];
    int32_t used = 0;                       // canonical streams in use
    uint64_t placed = 0;

    void init(bool multi, int32_t n_streams);
    void clear();
    void next(std::vector<Step> &out) const;
    void push(Step s);
    void pop();
    bool complete() const { return order.size() == tokens.size(); }

  private:
    static uint64_t bit(int32_t t) { return uint64_t(1) << t; }
    bool preds_done(int32_t v) const;
    bool ready(int32_t t) const;
};

// ----------------------------------------------------------------- fine DAG
// Token fields: op (low 4 bits), synchronisation kind (bits 4-5), peer rank
// + 1 (bits 8-15, 0 for tokens without a peer).
int32_t tok_op(int32_t t);
int32_t tok_kind(int32_t t);
int32_t tok_peer(int32_t t);
std::string tok_name(int32_t t);   // printable name, "token N" if unknown

// The fine-grained program DAG of one share (see spmv_fine.cpp).
struct FineDag {
    std::vector<int32_t> dests, srcs;          // peer ranks, ascending
    std::vector<int32_t> tokens;               // every token of an order, ascending
    std::map<int32_t, int32_t> index;          // token -> position in tokens
    std::vector<std::vector<int32_t>> need;    // positions that must come first
    std::vector<bool> gpu;                     // token is a GPU vertex
    void build(const Share &S);
    int find(int32_t t) const;
};

// A prefix of a fine-grained order (same interface as Prefix).
struct FinePrefix {
    const FineDag *dag = nullptr;
    int32_t n_streams = 1;
    std::vector<int32_t> order, ostream;       // tokens and their streams (-1: none)
    std::vector<bool> placed;
    int32_t used = 0;
    void init(const FineDag *d, int32_t n_streams);
    void clear();
    bool ready(int32_t i) const;
    void next(std::vector<Prefix::Step> &out) const;
    void push(Prefix::Step s);
    bool complete() const { return order.size() == dag->tokens.size(); }
};

struct FineSchedule {
    std::vector<int32_t> order, ostream;       // canonical streams per position
    int32_t n_streams_used = 0;
};

int validate_fine(const FineDag &dag, const int32_t *ops, const int32_t *op_stream,
                  int32_t n_ops, int32_t n_streams, FineSchedule &out);
void fine_default(const FineDag &dag, std::vector<int32_t> &ops, std::vector<int32_t> &streams);
// Number of fine-grained programs: orders times canonical stream maps.
int fine_count(const FineDag &dag, int32_t n_streams, double &count);

// ----------------------------------------------------------------- kernels
// Launchers (spmv_kernels.hip).  All are asynchronous on `s` and launch
// nothing for empty inputs.
struct CsrDev {
    int32_t n_rows = 0;            // rows computed by the kernel
    const int32_t *rp = nullptr;   // [n_rows + 1]
    const int32_t *col = nullptr;
    const double *val = nullptr;
    const int32_t *rows = nullptr; // compressed-row ids (remote), else null
    int64_t nnz_alloc = 0;         // entries allocated (rp[n_rows] + padding)
    int64_t n_x = 0;               // length of the x vector the columns index
    // CSR-stream tiles: [tile_row[t], tile_row[t+1]) rows, entries from tile_k[t]
    const int32_t *tile_row = nullptr, *tile_k = nullptr;
    int32_t n_tiles = 0;
    // sliced ELL (form 2): col/val hold the sliced layout, sell_ptr[s] is
    // the first entry of slice s (64 rows), n_slices slices, U entries per
    // batch of loads
    const int32_t *sell_ptr = nullptr;
    int32_t n_slices = 0, sell_u = 0;
    int32_t sell_width = 0;        // > 0: every slice this wide (sell_ptr unused)
    // form 3: `col` holds 16-bit column offsets from the row (grouped 8 per
    // lane, see build_sell16) in off_bytes bytes
    uint32_t off_bytes = 0;
    // form 4: `col` holds int16 offsets of each column from the first row of
    // the entry's tile (see build_tile16)
    bool col16 = false;
};

// Entries of padding after col/val on the device (vector loads of the
// CSR-stream kernel never straddle the end of a buffer).
constexpr int kEntryPad = 16;

hipError_t launch_pack(const double *x, const int32_t *idx, double *out, int64_t n,
                       hipStream_t s);
hipError_t launch_unpack(const double *recv, const int32_t *perm, double *xh, int64_t n,
                         hipStream_t s);
// y[row] = sum (store) or y[rows[j]] += sum (accumulate) when acc_into != null
hipError_t launch_csr(const CsrDev &A, const double *x, double *out, double *acc_into,
                      int lanes, int rows, int xcd_remap, bool allow_buffer, hipStream_t s);
hipError_t launch_combine(const int32_t *rows, const double *part, double *y, int64_t n,
                          hipStream_t s);
// Pack run by extra blocks of a product's launch (the resident step): the
// blocks after the product's own each gather kPackPerThread entries per
// thread of dst[k] = x[idx[k]], k < n.  A default PackTail adds nothing.
struct PackTail {
    const double *x = nullptr;
    const int32_t *idx = nullptr;
    double *dst = nullptr;
    int32_t n = 0;
};
// The remote part of a row added where the row's local sum is stored (the
// resident step with y_R in y_L's launch).  Local rows come in groups of
// 64: mask[g] marks the rows of group g that have remote entries, j0[g] is
// the compressed index of the first of them; A_R is a CSR over the
// compressed rows (rp, col into xh = x_halo, val).  The remote sum repeats
// the arithmetic of the plan's y_R kernel: an fma chain over the row's
// entries in order (sliced form, fma_chain = 1), or each product rounded
// and the products added left to right from zero (packed tiles with one
// summing lane), so that local + remote has the bits of spmv_exec.
// mask == nullptr: no remote part.
// tj, te (packed-tile y_L with rounded products): tile t's rows hold the
// compressed rows [tj[t], tj[t + 1]) and their entries [te[t], te[t + 1]),
// at most one window's worth (kTileRemoteCap and the tile's window); its
// block loads them beside its own entries instead of each row's storing
// lane walking them after the local sum.
struct RemoteFuse {
    const uint64_t *mask = nullptr;
    const int32_t *j0 = nullptr, *rp = nullptr, *col = nullptr;
    const double *val = nullptr, *xh = nullptr;
    int32_t fma_chain = 0;
    const int32_t *tj = nullptr, *te = nullptr;
    int32_t tile_cap = 0;   // the bound the plan checked te[t + 1] - te[t] against
    // With n_grid > 0 the tiles go to the XCDs in contiguous ranges of
    // equal cost: XCD x runs tiles [xr[x], xr[x + 1]) (the last XCD from
    // the end of its range) in the first n_grid = 8 * (longest range)
    // blocks; a block past its XCD's range exits.
    int32_t n_grid = 0;
    int32_t xr[9] = {};
};
constexpr int kTileRemoteCap = 1024;   // remote entries per tile, 4 per thread
constexpr int kPackPerThread = 4;
// Longest send list a PackTail takes (its block and entry indices are int;
// a longer one runs Pack as a kernel of its own).
constexpr int64_t kPackTailMax = int64_t(1) << 30;
hipError_t launch_csr_stream(const CsrDev &A, const double *x, double *out, double *acc,
                             int npt, int vw, int sum_lanes, int xcd_remap, hipStream_t s,
                             const PackTail &tail = PackTail(),
                             const RemoteFuse &rem = RemoteFuse());
// Sliced-ELL product (CsrDev.sell_ptr set): one wave per slice of 64 rows.
hipError_t launch_sell(const CsrDev &A, const double *x, double *out, double *acc,
                       int xcd_remap, hipStream_t s);
int stream_cap(int npt);
int stream_maxr(int sum_lanes);

// Form 5 (y_R): the halo's columns cut into kSlabs equal ranges, one per
// XCD.  Slab k is a CSR over all compressed remote rows holding the entries
// whose halo index lies in range k, cut into packed stream tiles; the blocks
// of slab k run on XCD k (blocks are dealt to the XCDs round-robin), so the
// x values slab k gathers stay in that XCD's L2.  Each slab writes one
// partial sum per row; a second kernel adds the kSlabs partial sums of a row
// in slab order and stores the result (out[i]) or adds it (acc[rows[i]]).
constexpr int kSlabs = 8;
struct SlabDev {
    const int32_t *rp;          // [kSlabs * (n_rows + 1)], slab k at k * (n_rows + 1)
    const int32_t *col;         // slab k's entries from nnz_off[k]
    const double *val;
    const int32_t *tile_row, *tile_k;   // slab k's tiles from tile_off[k]
    const int32_t *rows;
    const double *x;
    double *part;               // [kSlabs * n_rows]
    double *out, *acc;
    int32_t n_rows, chunk, width, lanes;
    int32_t rpt;                // rows per thread: 1 = tiles of kBlock / lanes rows;
                                // 2, 4, 8 = wide tiles (lanes 1)
    int64_t nnz_off[kSlabs + 1], tile_off[kSlabs + 1];   // tile_off: n_tiles + 1 each
    int64_t nnz_alloc, n_x;
};
hipError_t launch_slabs(const SlabDev &A, hipStream_t s);
// Builds the slabs from a CSR over n_rows rows whose columns index an
// n_x-entry vector; each slab's entries start at a multiple of 4.
void build_slabs(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                 const std::vector<double> &val, int64_t n_rows, int64_t n_x, int cap, int maxr,
                 int vw, std::vector<int32_t> &s_rp, std::vector<int32_t> &s_col,
                 std::vector<double> &s_val, std::vector<int32_t> &tile_row,
                 std::vector<int32_t> &tile_k, int64_t *nnz_off, int64_t *tile_off);
// Sliced ELL with slices of 64 rows (one wave): entry v of row 64 s + l is
// stored at ptr[s] + 64 v + l, a slice as wide as its longest row (or every
// slice as wide as the longest row, `uniform`, when that padding fits too),
// padding entries column -1 and value 0.  Returns false, leaving the
// outputs empty, when the padded size exceeds max_ratio times the entries
// or 32-bit offsets would overflow.
bool build_sell(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                const std::vector<double> &val, int64_t n_rows, double max_ratio,
                std::vector<int32_t> &ptr, std::vector<int32_t> &scol, std::vector<double> &sval,
                int32_t &max_width, bool &uniform);
// Sliced-ELL product with 16-bit row-relative columns (form 3, one width
// for every slice, values in pairs: see pair_values): entries in groups of
// 8 per lane, 8 * `sell_u` entries per batch of loads.
hipError_t launch_sell16(const CsrDev &A, const double *x, double *out, int xcd_remap,
                         hipStream_t s, const PackTail &tail = PackTail(),
                         const RemoteFuse &rem = RemoteFuse());
// Padding marker of the 16-bit column offsets (never a valid offset).
constexpr int16_t kPad16 = -32768;
// The columns of a uniform-width sliced layout as offsets from the row:
// entry v of row r = 64 s + l (column c) is stored as int16 (c - r) at
// ((s * G + v / 8) * 64 + l) * 8 + v % 8, G = ceil(width / 8), so that a
// lane reads 8 entries of its row with one 16-byte load and a wave's load
// is 1 KiB contiguous; padding holds kPad16.  Returns false, leaving `off`
// empty, when some |c - r| exceeds 32767 or 32-bit byte offsets overflow.
bool build_sell16(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                  int64_t n_rows, int32_t width, std::vector<int16_t> &off);
// The columns of a product cut into stream tiles as int16 offsets from the
// first row of each entry's tile: off[k] = col[k] - tile_row[t] for k in
// [tile_k[t], tile_k[t+1]).  Returns false, leaving `off` empty, when an
// offset does not fit 16 bits.
bool build_tile16(const std::vector<int32_t> &col, const std::vector<int32_t> &tile_row,
                  const std::vector<int32_t> &tile_k, std::vector<int16_t> &off);
// Reorder the values of a uniform-width sliced layout (entry v of row
// 64 s + l at 64 w s + 64 v + l) into pairs: entries 2p and 2p + 1 of row l
// at 64 w s + 128 p + 2 l (+ 1), and the last entry of an odd width at
// 64 w s + 64 (w - 1) + l, so that a lane reads two entries with one
// 16-byte load.
void pair_values(std::vector<double> &val, int64_t n_slices, int32_t width);
// Cut [0, n_rows) into CSR-stream tiles (host).
void build_tiles(const std::vector<int32_t> &rp, int64_t n_rows, int cap, int maxr, int vw,
                 std::vector<int32_t> &tile_row, std::vector<int32_t> &tile_k);
int auto_lanes(int64_t nnz, int64_t rows);
int auto_rows(int lanes, int64_t rows);

// Serving: one request's product (y = A x over a resident single-rank plan).
struct ServeDev {
    const int32_t *tile_row, *tile_k, *rp, *col;
    const double *val;
    const double *x;
    double *y;
    uint32_t nnz_alloc, n;
    int32_t lanes, n_tiles;
};
// One grouped launch over the tiles of n_req requests; pref[s] = first global
// tile of request s (pref[n_req] = total).  Grid-stride over tiles.
hipError_t launch_serve(int npt, int vw, const ServeDev *d_desc, const int32_t *d_pref,
                        int n_req, int total_tiles, hipStream_t s);
// The same for a batch of at most kServeInline requests whose descriptors
// travel in the kernel arguments (no copy of them ahead of the launch).
constexpr int kServeInline = 8;
struct ServeInline {
    ServeDev d[kServeInline];
    int32_t pref[kServeInline + 1];
    int32_t n_req;
};
hipError_t launch_serve_inline(int npt, int vw, const ServeInline &a, hipStream_t s);

// Per-device stream pool shared by all plans and batches (spmv_plan.cpp):
// plan streams 0..n_plan-1 and the send / receive copy streams.
// Copy streams per direction in the per-device pool (per-peer copies of a
// fine-grained program round-robin over them).
constexpr int kCopyStreams = 4;
// send / recv: [kCopyStreams] out.
int pool_streams(int device, int32_t n_plan, hipStream_t *plan_st, hipStream_t *send,
                 hipStream_t *recv);
// Give back one acquisition of the device's pool; the last one destroys
// its streams.
void pool_release(int device);

}  // namespace spmv

// ----------------------------------------------------------------- plan
// The plan object behind the opaque spmv_plan_t (spmv_plan.cpp); batches
// (spmv_batch.hip) read its device arrays and tiles.
namespace spmv {
// Kernel configuration of one product (y_L or y_R).
// The resident step of one plan in two grouped launches (defined with the
// batch kernels): built at plan creation for a share whose y_R is in column
// slabs and whose y_L is in packed tiles of the same window and width.
struct ResidentProg;
int resident_build(spmv_plan *p);
void resident_free(spmv_plan *p);
// part 0: the launch of Pack, y_L and the slab tiles; 1: the slab sums;
// -1: both in that order.
hipError_t resident_launch(const spmv_plan *p, int part, const double *x, double *y,
                           hipStream_t s);

struct CsrCfg {
    int32_t kernel = SPMV_KERNEL_VECTOR;
    int32_t lanes = 1, rows = 1;   // vector CSR
    int32_t chunk = 8, width = 2;  // stream CSR (lanes = summing lanes)
    int32_t form = 1;              // stream: 1 packed tiles, 2 sliced ELL,
                                   // 3 sliced ELL with 16-bit column offsets,
                                   // 4 packed tiles with 16-bit column offsets,
                                   // 5 column slabs (y_R)
    std::vector<int32_t> sell_ptr, sell_col;   // forms 2/3, host copies for upload
    std::vector<int16_t> sell_off;             // form 3 (sell_col then empty)
    std::vector<int16_t> tile_off;             // form 4
    std::vector<double> sell_val;
    int32_t sell_width = 0;
    bool sell_uniform = false;
    std::vector<int32_t> tile_row, tile_k;
    // form 5: sell_ptr holds the slabs' row pointers, tile_row/tile_k their
    // tiles (concatenated), slab_col/slab_val their entries
    std::vector<int32_t> slab_col;
    std::vector<double> slab_val;
    int64_t slab_nnz[kSlabs + 1] = {}, slab_tiles[kSlabs + 1] = {};
};
}  // namespace spmv

struct spmv_plan {
    spmv::Share share;
    spmv::Schedule sch;
    spmv::CsrCfg cfg[2];           // [0] = y_L, [1] = y_R
    int32_t xcd_remap = 1;
    bool fuse_unpack = false, fused_combine = false, host_only = false, profile = false;
    bool pool_held = false;        // holds one acquisition of the stream pool
    bool use_buffer = true;
    int device = 0;

    // device arena and its views
    void *arena = nullptr;
    size_t arena_bytes = 0;
    int32_t *dL_ptr = nullptr, *dL_col = nullptr;
    double *dL_val = nullptr;
    int32_t *dR_rows = nullptr, *dR_ptr = nullptr, *dR_col = nullptr;
    double *dR_val = nullptr;
    int32_t *d_send_idx = nullptr, *d_perm = nullptr;
    double *d_sendbuf = nullptr, *d_recvbuf = nullptr, *d_xhalo = nullptr, *d_part = nullptr;
    double *d_slab_part = nullptr;   // form 5: [kSlabs * n_remote_rows]
    spmv::ResidentProg *res = nullptr;   // grouped resident step, or null
    bool resident_seq = false;       // resident step op by op even with res
    // resident step in y_L's launch (rf.mask set): per 64 local rows the
    // mask of remote rows and the first one's compressed index, and A_R's
    // CSR (y_R's own arrays in packed tiles, a copy beside the sliced form)
    spmv::RemoteFuse rf;
    uint64_t *d_rf_mask = nullptr;
    int32_t *d_rf_j0 = nullptr, *d_rf_rp = nullptr, *d_rf_col = nullptr;
    double *d_rf_val = nullptr;
    int32_t *d_rf_tj = nullptr, *d_rf_te = nullptr;
    int32_t *d_tile_row[2] = {}, *d_tile_k[2] = {};
    int32_t *d_sell_ptr[2] = {};

    // pinned host mailboxes
    double *h_inbox = nullptr, *h_outbox = nullptr;

    // streams and events
    hipStream_t st[SPMV_MAX_STREAMS] = {};
    int32_t n_st = 0;           // plan streams owned
    int32_t n_streams_max = 1;  // as requested at creation
    hipStream_t cs_send = nullptr, cs_recv = nullptr;
    hipStream_t cs_send_k[spmv::kCopyStreams] = {}, cs_recv_k[spmv::kCopyStreams] = {};
    hipEvent_t ev_start = nullptr, ev_send = nullptr, ev_recv = nullptr;
    hipEvent_t ev_rec[SPMV_N_VERTICES] = {};
    // fine-grained mode: the order is fsch over fdag (per-peer vertices)
    bool fine = false;
    spmv::FineDag fdag;
    spmv::FineSchedule fsch;
    std::vector<hipEvent_t> ev_pack, ev_psend, ev_precv;   // per peer rank
    // profiling: begin/end per vertex, index SPMV_N_VERTICES = combine
    hipEvent_t ev_b[SPMV_N_VERTICES + 1] = {}, ev_e[SPMV_N_VERTICES + 1] = {};
    double ms[SPMV_N_VERTICES + 1] = {};
    double cnt[SPMV_N_VERTICES + 1] = {};
    // host timeline: summed microseconds from an exec's entry to the end of
    // each token's host call, over host_n execs (reset when the order changes)
    bool host_times = false;
    std::vector<double> host_us;
    double host_n = 0.0;
};
