// Batches: the SpMVs of many rank shares in grouped persistent kernels,
// with the halo staging pipelined per chunk of shares.
//
// Work items are the stream-CSR tiles of every share's y_L and y_R (column
// slabs included: a slab tile, then the sum of a row range's slab partial
// sums) and the gather ranges of every share's Pack and Unpack.  Each
// grouped kernel runs a fixed grid (256 CUs x blocks_per_cu); every block
// walks its own list of items, assigned on the host longest-first to the
// least-loaded block, and, with XCD affinity, only to blocks of the XCD that
// owns the share (share s -> XCD s mod 8) so the share's x stays in that
// XCD's L2; a slab tile always goes to its slab's XCD.  The shares are cut
// into chunks: chunk c's Pack feeds chunk c's send copies while later chunks
// pack, and chunk c's y_R runs as soon as chunk c's receive copies are in,
// under the copies of the chunks after it.  The host-blocking
// synchronisations of the single-share program become stream or graph
// dependencies.
#include <algorithm>
#include <cstring>
#include <deque>
#include <functional>
#include <numeric>
#include <queue>

#include "spmv_internal.h"
#include "spmv_stream.h"

namespace spmv {
namespace {

enum ItemKind : int32_t {
    kPack = 0, kLocal = 1, kUnpack = 2, kRemote = 3,
    kSlab = 4,      // tile a of column slab n of the share's y_R
    kSlabSum = 5,   // y[rows[i]] += the 8 slab partial sums of row i, i in [a, a + n)
    kNop = 6        // padding of the one-block-per-item form
};

// Device view of one share.
struct ShareDev {
    const int32_t *L_tile_row, *L_tile_k, *L_rp, *L_col;
    const double *L_val;
    const int32_t *R_tile_row, *R_tile_k, *R_rp, *R_col, *R_rows;
    const double *R_val;
    const int32_t *send_idx, *perm;
    double *sendbuf, *recvbuf, *xhalo;
    uint32_t L_nnz_alloc, R_nnz_alloc, n_loc, n_halo;
    int32_t L_lanes, R_lanes, fuse_unpack;
    int32_t L_col16;   // A_L columns as int16 offsets from each tile's first row
    // y_R in column slabs: slab k's row pointer at R_rp + k * (n_rr + 1), its
    // entries from slab_nnz[k], its tiles from slab_tile[k] of R_tile_row /
    // R_tile_k; partial sums of slab k at slab_part + k * n_rr
    double *slab_part;
    int32_t n_rr;
    int32_t slab_nnz[kSlabs + 1], slab_tile[kSlabs + 1];
};

struct Item {
    int32_t kind, share, a, n;   // tile a (of slab n), or a range [a, a + n)
};

template <int NPT, int VW, bool C16 = false>
__device__ __forceinline__ void tile_sl(int sl, const StreamArgs &A, int t, double *s_p,
                                        int32_t *s_rp)
{
    switch (sl) {
        case 1: stream_tile<NPT, VW, 1, C16>(A, t, s_p, s_rp); break;
        case 2: stream_tile<NPT, VW, 2, C16>(A, t, s_p, s_rp); break;
        case 4: stream_tile<NPT, VW, 4, C16>(A, t, s_p, s_rp); break;
        case 8: stream_tile<NPT, VW, 8, C16>(A, t, s_p, s_rp); break;
        default: stream_tile<NPT, VW, 16, C16>(A, t, s_p, s_rp); break;
    }
}

// One work item of a share whose x and y are `x`, `y`, by the whole block.
// Contains barriers only in block-uniform control flow.
template <int NPT, int VW>
__device__ __forceinline__ void run_item(const Item &it, const ShareDev &S,
                                         const double *__restrict__ x, double *__restrict__ y,
                                         double *s_p, int32_t *s_rp)
{
    if (it.kind == kPack || it.kind == kUnpack) {
        const double *src = it.kind == kPack ? x : S.recvbuf;
        const int32_t *idx = it.kind == kPack ? S.send_idx : S.perm;
        double *dst = it.kind == kPack ? S.sendbuf : S.xhalo;
        // a range holds at most NPT * kBlock entries: each thread loads all
        // its indices, then gathers all its values, then stores them.  The
        // indices and the stores stream past the L2 (non-temporal): in the
        // resident step they would otherwise evict the x lines of the slab
        // tiles beside them (43.9 against 47.1 us per step of the power-law
        // 4M share); x itself keeps the default policy, its lines are
        // reused by every destination's list
        const int end = it.a + it.n, t0 = it.a + int(threadIdx.x);
        int32_t id[NPT];
        double v[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j)
            id[j] = t0 + j * kBlock < end ? __builtin_nontemporal_load(idx + t0 + j * kBlock) : -1;
#pragma unroll
        for (int j = 0; j < NPT; ++j) v[j] = id[j] >= 0 ? src[id[j]] : 0.0;
#pragma unroll
        for (int j = 0; j < NPT; ++j)
            if (t0 + j * kBlock < end) __builtin_nontemporal_store(v[j], dst + t0 + j * kBlock);
        for (int k = t0 + NPT * kBlock; k < end; k += kBlock) dst[k] = src[idx[k]];
    } else if (it.kind == kLocal) {
        StreamArgs A;
        A.tile_row = S.L_tile_row;
        A.tile_k = S.L_tile_k;
        A.rp = S.L_rp;
        A.col = S.L_col;
        A.rows = nullptr;
        A.val = S.L_val;
        A.x = x;
        A.out = y;
        A.acc = nullptr;
        A.nnz_alloc = S.L_nnz_alloc;
        A.n_x = S.n_loc;
        if (S.L_col16)
            tile_sl<NPT, VW, true>(S.L_lanes, A, it.a, s_p, s_rp);
        else
            tile_sl<NPT, VW, false>(S.L_lanes, A, it.a, s_p, s_rp);
    } else if (it.kind == kRemote) {
        StreamArgs A;
        A.tile_row = S.R_tile_row;
        A.tile_k = S.R_tile_k;
        A.rp = S.R_rp;
        A.col = S.R_col;
        A.rows = S.R_rows;
        A.val = S.R_val;
        A.x = S.fuse_unpack ? S.recvbuf : S.xhalo;
        A.out = nullptr;
        A.acc = y;
        A.nnz_alloc = S.R_nnz_alloc;
        A.n_x = S.n_halo;
        tile_sl<NPT, VW>(S.R_lanes, A, it.a, s_p, s_rp);
    } else if (it.kind == kSlab) {
        // as k_csr_slabs: slab n's tile a, partial sums stored
        const int k = it.n;
        StreamArgs A;
        A.tile_row = S.R_tile_row + S.slab_tile[k];
        A.tile_k = S.R_tile_k + S.slab_tile[k];
        A.rp = S.R_rp + int64_t(k) * (S.n_rr + 1);
        A.col = S.R_col + S.slab_nnz[k];
        A.rows = nullptr;
        A.val = S.R_val + S.slab_nnz[k];
        A.x = S.fuse_unpack ? S.recvbuf : S.xhalo;
        A.out = S.slab_part + int64_t(k) * S.n_rr;
        A.acc = nullptr;
        A.nnz_alloc = S.R_nnz_alloc - uint32_t(S.slab_nnz[k]);
        A.n_x = S.n_halo;
        tile_sl<NPT, VW>(S.R_lanes, A, it.a, s_p, s_rp);
    } else if (it.kind == kSlabSum) {
        // as k_slab_sum adding into y: the partial sums in slab order
        const int64_t n = S.n_rr;
        for (int r = it.a + int(threadIdx.x); r < it.a + it.n; r += kBlock) {
            double s = S.slab_part[r];
#pragma unroll
            for (int k = 1; k < kSlabs; ++k) s += S.slab_part[k * n + r];
            y[S.R_rows[r]] += s;
        }
    }
    // kNop: nothing
}

// Persistent form: block b walks its own item list.
template <int NPT, int VW>
__global__ __launch_bounds__(kBlock) void k_grouped(const ShareDev *__restrict__ sh,
                                                    const double *const *__restrict__ xs,
                                                    double *const *__restrict__ ys,
                                                    const Item *__restrict__ items,
                                                    const int32_t *__restrict__ blk_ptr)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock + 1];
    const int b = int(blockIdx.x);
    const int i1 = blk_ptr[b + 1];
    for (int i = blk_ptr[b]; i < i1; ++i) {
        const Item it = items[i];
        run_item<NPT, VW>(it, sh[it.share], xs[it.share], ys[it.share], s_p, s_rp);
        __syncthreads();
    }
}

// One block per item: block b runs item b (blocks are dealt to the XCDs
// round-robin, so the host places an item that must run on XCD g at an
// index b with b % 8 == g, padding with kNop).  blk_ptr is not used.
template <int NPT, int VW>
__global__ __launch_bounds__(kBlock) void k_grouped_flat(const ShareDev *__restrict__ sh,
                                                         const double *const *__restrict__ xs,
                                                         double *const *__restrict__ ys,
                                                         const Item *__restrict__ items,
                                                         const int32_t *__restrict__ blk_ptr)
{
    (void)blk_ptr;
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock + 1];
    const Item it = items[blockIdx.x];
    run_item<NPT, VW>(it, sh[it.share], xs[it.share], ys[it.share], s_p, s_rp);
}

// Tile t of one request: y = A x over the request's matrix.
template <int NPT, int VW>
__device__ __forceinline__ void serve_tile(const ServeDev &S, int t, double *s_p, int32_t *s_rp)
{
    StreamArgs A;
    A.tile_row = S.tile_row;
    A.tile_k = S.tile_k;
    A.rp = S.rp;
    A.col = S.col;
    A.rows = nullptr;
    A.val = S.val;
    A.x = S.x;
    A.out = S.y;
    A.acc = nullptr;
    A.nnz_alloc = S.nnz_alloc;
    A.n_x = S.n;
    tile_sl<NPT, VW>(S.lanes, A, t, s_p, s_rp);
}

// Serving: grid-stride over the tiles of a batch of requests (each request
// one resident single-rank matrix); request s owns global tiles
// [pref[s], pref[s+1]).
template <int NPT, int VW>
__global__ __launch_bounds__(kBlock) void k_serve(const ServeDev *__restrict__ d,
                                                  const int32_t *__restrict__ pref, int n_req)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock + 1];
    const int total = pref[n_req];
    for (int g = int(blockIdx.x); g < total; g += int(gridDim.x)) {
        int lo = 0, hi = n_req;   // largest s with pref[s] <= g
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pref[mid] <= g)
                lo = mid;
            else
                hi = mid;
        }
        serve_tile<NPT, VW>(d[lo], g - pref[lo], s_p, s_rp);
        __syncthreads();
    }
}

using GroupedFn = void (*)(const ShareDev *, const double *const *, double *const *, const Item *,
                           const int32_t *);

GroupedFn grouped_fn(int npt, int vw, bool flat)
{
    if (vw == 2) {
        if (npt == 4) return flat ? k_grouped_flat<4, 2> : k_grouped<4, 2>;
        if (npt == 8) return flat ? k_grouped_flat<8, 2> : k_grouped<8, 2>;
        if (npt == 16) return flat ? k_grouped_flat<16, 2> : k_grouped<16, 2>;
    } else if (vw == 4) {
        if (npt == 4) return flat ? k_grouped_flat<4, 4> : k_grouped<4, 4>;
        if (npt == 8) return flat ? k_grouped_flat<8, 4> : k_grouped<8, 4>;
        if (npt == 16) return flat ? k_grouped_flat<16, 4> : k_grouped<16, 4>;
    }
    return nullptr;
}

constexpr int kCUs = 256;

}  // namespace

// Small batches: the descriptors come in the kernel arguments.
template <int NPT, int VW>
__global__ __launch_bounds__(kBlock) void k_serve_inline(const ServeInline a)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock + 1];
    const int total = a.pref[a.n_req];
    for (int g = int(blockIdx.x); g < total; g += int(gridDim.x)) {
        int lo = 0;   // largest s with pref[s] <= g
        for (int s = 1; s < a.n_req; ++s)
            if (a.pref[s] <= g) lo = s;
        serve_tile<NPT, VW>(a.d[lo], g - a.pref[lo], s_p, s_rp);
        __syncthreads();
    }
}

hipError_t launch_serve_inline(int npt, int vw, const ServeInline &a, hipStream_t s)
{
    if (a.n_req < 1 || a.n_req > kServeInline) return hipErrorInvalidValue;
    const int total = a.pref[a.n_req];
    if (total <= 0) return hipSuccess;
    const unsigned grid = unsigned(std::min(total, kCUs * 8));
    void (*fn)(const ServeInline) = nullptr;
    if (vw == 2) fn = npt == 4 ? k_serve_inline<4, 2> : npt == 8 ? k_serve_inline<8, 2> : npt == 16 ? k_serve_inline<16, 2> : nullptr;
    if (vw == 4) fn = npt == 4 ? k_serve_inline<4, 4> : npt == 8 ? k_serve_inline<8, 4> : npt == 16 ? k_serve_inline<16, 4> : nullptr;
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_serve(int npt, int vw, const ServeDev *d_desc, const int32_t *d_pref, int n_req,
                        int total_tiles, hipStream_t s)
{
    if (total_tiles <= 0) return hipSuccess;
    const unsigned grid = unsigned(std::min(total_tiles, kCUs * 8));
    void (*fn)(const ServeDev *, const int32_t *, int) = nullptr;
    if (vw == 2) fn = npt == 4 ? k_serve<4, 2> : npt == 8 ? k_serve<8, 2> : npt == 16 ? k_serve<16, 2> : nullptr;
    if (vw == 4) fn = npt == 4 ? k_serve<4, 4> : npt == 8 ? k_serve<8, 4> : npt == 16 ? k_serve<16, 4> : nullptr;
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), 0, s, d_desc, d_pref, n_req);
    return hipGetLastError();
}

}  // namespace spmv

using namespace spmv;

struct spmv_batch {
    std::vector<spmv_plan *> plans;
    int32_t n = 0, npt = 8, vw = 2, n_blocks = 0;
    bool use_graph = true, xcd_aff = false, staging = true;
    int device = 0;
    GroupedFn fn = nullptr;

    // Launch groups in issue order: per chunk c a Pack group; then y_L of
    // every share; then per chunk Unpack, y_R (packed and slab tiles) and
    // the slab sums.  Each group is one grouped launch over its items.
    enum GroupKind : int32_t { gPack = 0, gLocal = 1, gUnpack = 2, gRemote = 3, gSlabSum = 4 };
    struct Group {
        int32_t kind, chunk;
        int64_t n_items;      // entries of d_items (kNop padding included)
        unsigned grid;        // blocks of its launch
        Item *d_items;
        int32_t *d_blk;
    };
    bool flat = false;        // one block per item instead of persistent blocks
    std::vector<Group> groups;
    int32_t n_chunks = 1;
    std::vector<int32_t> chunk_lo;   // shares [chunk_lo[c], chunk_lo[c+1]) form chunk c

    void *arena = nullptr;
    size_t arena_bytes = 0;
    ShareDev *d_sh = nullptr;
    const double **d_x = nullptr;   // [n], then d_y right after (one table)
    double **d_y = nullptr;
    int64_t n_items[3] = {};        // totals: Pack + y_L, Unpack, y_R (incl. slab sums)
    void **h_xy = nullptr;          // pinned [2n]: x pointers then y pointers

    int32_t n_cs = 1;                                   // copy streams per direction
    hipStream_t cs_send_k[kCopyStreams] = {}, cs_recv_k[kCopyStreams] = {};
    hipEvent_t ev_f = nullptr;
    std::vector<hipEvent_t> ev_pack;                    // [n_chunks]: chunk's Pack done
    std::vector<hipEvent_t> ev_recv;                    // [n_chunks * n_cs]: chunk's copies in
    hipEvent_t ev_sk[kCopyStreams] = {};                // each send stream drained
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t dev_bytes = 0, link_bytes = 0;
    bool pool_held = false;         // holds one acquisition of the stream pool
};

namespace {

void batch_release(spmv_batch *b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_f) (void)hipEventDestroy(b->ev_f);
    for (hipEvent_t e : b->ev_pack)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->ev_recv)
        if (e) (void)hipEventDestroy(e);
    for (int k = 0; k < kCopyStreams; ++k)
        if (b->ev_sk[k]) (void)hipEventDestroy(b->ev_sk[k]);
    if (b->arena) (void)hipFree(b->arena);
    if (b->h_xy) (void)hipHostFree(b->h_xy);
    if (b->pool_held) pool_release(b->device);
    delete b;
}

// Assignment of items to blocks.  An item's XCD group g (0..7) restricts it
// to blocks b with b % 8 == g (the XCD the hardware deals block b to); -1
// lets it go to any block.  Items marked `ordered` are dealt round-robin in
// their given order over their group's blocks, so every block walks them in
// that order (column-slab tiles in share order: an XCD's blocks then work
// on the slabs of one or two shares at a time, which fit its L2); the others
// go longest-first to the least-loaded block.  Returns items grouped by
// block and the per-block offsets.
void assign(const std::vector<Item> &items, const std::vector<int64_t> &cost,
            const std::vector<int8_t> &xcd, const std::vector<uint8_t> &ordered, int n_blocks,
            std::vector<Item> &out, std::vector<int32_t> &blk_ptr)
{
    std::vector<int64_t> load(size_t(n_blocks), 0);
    std::vector<int32_t> owner(items.size(), -1);
    std::vector<int64_t> cursor(size_t(kXcds) + 1, 0);
    for (size_t i = 0; i < items.size(); ++i) {
        if (!ordered[i]) continue;
        const int g = xcd[i];
        int32_t b;
        if (g < 0) {
            b = int32_t(cursor[size_t(kXcds)]++ % n_blocks);
        } else {
            const int64_t per = (n_blocks - g + kXcds - 1) / kXcds;   // blocks with b % 8 == g
            b = int32_t(g + kXcds * (cursor[size_t(g)]++ % per));
        }
        owner[i] = b;
        load[size_t(b)] += cost[i];
    }
    std::vector<size_t> order;
    for (size_t i = 0; i < items.size(); ++i)
        if (!ordered[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    using Slot = std::pair<int64_t, int32_t>;   // (load, block)
    using Heap = std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>>;
    // one heap per XCD and one over every block; a block's entry is renewed
    // in both whenever its load grows, and older entries (a smaller load
    // than the block's current one: costs are positive) are dropped when met
    std::vector<Heap> heaps(size_t(kXcds) + 1);
    for (int32_t b = 0; b < n_blocks; ++b) {
        heaps[size_t(b % kXcds)].push({load[size_t(b)], b});
        heaps[size_t(kXcds)].push({load[size_t(b)], b});
    }
    for (size_t i : order) {
        Heap &h = heaps[size_t(xcd[i] < 0 ? kXcds : xcd[i])];
        while (h.top().first != load[size_t(h.top().second)]) h.pop();
        const int32_t b = h.top().second;
        h.pop();
        owner[i] = b;
        load[size_t(b)] += cost[i];
        heaps[size_t(b % kXcds)].push({load[size_t(b)], b});
        heaps[size_t(kXcds)].push({load[size_t(b)], b});
    }
    blk_ptr.assign(size_t(n_blocks) + 1, 0);
    for (size_t i = 0; i < items.size(); ++i) ++blk_ptr[size_t(owner[i]) + 1];
    for (int32_t b = 0; b < n_blocks; ++b) blk_ptr[size_t(b) + 1] += blk_ptr[size_t(b)];
    out.resize(items.size());
    std::vector<int32_t> fill(blk_ptr.begin(), blk_ptr.end() - 1);
    for (size_t i = 0; i < items.size(); ++i) out[size_t(fill[size_t(owner[i])]++)] = items[i];
}

// One block per item: slot i of the list runs on XCD i % 8, so an item that
// must run on XCD g takes the next free slot of that residue (in its given
// order), items without a group fill the other slots, and slots left over
// before the last item hold kNop.
void interleave(const std::vector<Item> &items, const std::vector<int8_t> &xcd,
                std::vector<Item> &out)
{
    std::deque<size_t> q[kXcds + 1];
    for (size_t i = 0; i < items.size(); ++i) q[xcd[i] < 0 ? kXcds : xcd[i]].push_back(i);
    out.clear();
    size_t left = items.size();
    for (size_t slot = 0; left > 0; ++slot) {
        std::deque<size_t> &mine = q[slot % kXcds];
        std::deque<size_t> &any = q[kXcds];
        std::deque<size_t> *from = !mine.empty() ? &mine : !any.empty() ? &any : nullptr;
        if (from) {
            out.push_back(items[from->front()]);
            from->pop_front();
            --left;
        } else {
            out.push_back({kNop, 0, 0, 0});
        }
    }
}

int64_t tile_cost(const std::vector<int32_t> &tk, size_t t) { return int64_t(tk[t + 1] - tk[t]) + 64; }

// Device view of one plan's share.
ShareDev share_dev(const spmv_plan *p)
{
    const Share &S = p->share;
    const CsrCfg &cr = p->cfg[1];
    ShareDev d;
    d.L_tile_row = p->d_tile_row[0];
    d.L_tile_k = p->d_tile_k[0];
    d.L_rp = p->dL_ptr;
    d.L_col = p->dL_col;
    d.L_val = p->dL_val;
    d.R_tile_row = p->d_tile_row[1];
    d.R_tile_k = p->d_tile_k[1];
    d.R_rp = cr.form == 5 ? p->d_sell_ptr[1] : p->dR_ptr;
    d.R_col = p->dR_col;
    d.R_rows = p->dR_rows;
    d.R_val = p->dR_val;
    d.send_idx = p->d_send_idx;
    d.perm = p->d_perm;
    d.sendbuf = p->d_sendbuf;
    d.recvbuf = p->d_recvbuf;
    d.xhalo = p->d_xhalo;
    d.L_nnz_alloc = uint32_t(S.L_col.size() + kEntryPad);
    d.R_nnz_alloc = uint32_t((cr.form == 5 ? cr.slab_col.size() : S.R_col.size()) + kEntryPad);
    d.n_loc = uint32_t(S.n_loc);
    d.n_halo = uint32_t(S.halo.size());
    d.L_lanes = p->cfg[0].lanes;
    d.R_lanes = cr.lanes;
    d.fuse_unpack = p->fuse_unpack ? 1 : 0;
    d.L_col16 = p->cfg[0].form == 4 ? 1 : 0;
    d.slab_part = p->d_slab_part;
    d.n_rr = int32_t(S.R_rows.size());
    for (int k = 0; k <= kSlabs; ++k) {
        d.slab_nnz[k] = cr.form == 5 ? int32_t(cr.slab_nnz[k]) : 0;
        d.slab_tile[k] = cr.form == 5 ? int32_t(cr.slab_tiles[k]) : 0;
    }
    return d;
}

hipError_t launch_group(const spmv_batch *b, const spmv_batch::Group &g, hipStream_t s)
{
    if (g.n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(b->fn, dim3(g.grid), dim3(kBlock), 0, s, b->d_sh, b->d_x, b->d_y,
                       g.d_items, g.d_blk);
    return hipGetLastError();
}

// One batch on stream s (stream launches): the pointer table; every
// receive copy, chunk by chunk, on the copy streams (they need nothing from
// this batch); per chunk its Pack, then its send copies behind it; y_L of
// every share; per chunk, once its receive copies are in, its Unpack, y_R
// and slab sums; then the join of the send copies.
int issue(spmv_batch *b, hipStream_t s)
{
    const int32_t K = b->n_cs, C = b->n_chunks;
    SPMV_HIP(hipMemcpyAsync(b->d_x, b->h_xy, size_t(2 * b->n) * sizeof(void *),
                            hipMemcpyHostToDevice, s));
    SPMV_HIP(hipEventRecord(b->ev_f, s));
    for (int32_t k = 0; k < K; ++k) {
        SPMV_HIP(hipStreamWaitEvent(b->cs_recv_k[k], b->ev_f, 0));
        SPMV_HIP(hipStreamWaitEvent(b->cs_send_k[k], b->ev_f, 0));
    }
    for (int32_t c = 0; c < C; ++c) {
        if (b->staging)
            for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
                const spmv_plan *p = b->plans[size_t(i)];
                const size_t nh = p->share.halo.size() * 8;
                if (nh)
                    SPMV_HIP(hipMemcpyAsync(p->d_recvbuf, p->h_inbox, nh, hipMemcpyHostToDevice,
                                            b->cs_recv_k[i % K]));
            }
        for (int32_t k = 0; k < K; ++k)
            SPMV_HIP(hipEventRecord(b->ev_recv[size_t(c * K + k)], b->cs_recv_k[k]));
    }
    for (const auto &g : b->groups) {
        if (g.kind == spmv_batch::gLocal) SPMV_HIP(launch_group(b, g, s));
        if (g.kind != spmv_batch::gPack) continue;
        SPMV_HIP(launch_group(b, g, s));
        SPMV_HIP(hipEventRecord(b->ev_pack[size_t(g.chunk)], s));
        for (int32_t k = 0; k < K; ++k)
            SPMV_HIP(hipStreamWaitEvent(b->cs_send_k[k], b->ev_pack[size_t(g.chunk)], 0));
        if (b->staging)
            for (int32_t i = b->chunk_lo[size_t(g.chunk)]; i < b->chunk_lo[size_t(g.chunk) + 1];
                 ++i) {
                const spmv_plan *p = b->plans[size_t(i)];
                const size_t ns = p->share.send_idx.size() * 8;
                if (ns)
                    SPMV_HIP(hipMemcpyAsync(p->h_outbox, p->d_sendbuf, ns, hipMemcpyDeviceToHost,
                                            b->cs_send_k[i % K]));
            }
    }
    int32_t waited = -1;
    for (const auto &g : b->groups) {
        if (g.kind == spmv_batch::gPack || g.kind == spmv_batch::gLocal) continue;
        if (g.chunk > waited) {
            for (int32_t k = 0; k < K; ++k)
                SPMV_HIP(hipStreamWaitEvent(s, b->ev_recv[size_t(g.chunk * K + k)], 0));
            waited = g.chunk;
        }
        SPMV_HIP(launch_group(b, g, s));
    }
    for (int32_t k = 0; k < K; ++k) {
        SPMV_HIP(hipEventRecord(b->ev_sk[k], b->cs_send_k[k]));
        SPMV_HIP(hipStreamWaitEvent(s, b->ev_sk[k], 0));
    }
    return SPMV_OK;
}

// The same schedule as one graph: each direction's copies form one chain
// (concurrent copies of one direction share the host link), the groups
// follow stream order, and chunk c's first y_R-side group also waits for the
// receive copy that closes chunk c.
int build_graph(spmv_batch *b)
{
    SPMV_HIP(hipGraphCreate(&b->graph, 0));
    hipGraphNode_t n_t;
    SPMV_HIP(hipGraphAddMemcpyNode1D(&n_t, b->graph, nullptr, 0, b->d_x, b->h_xy,
                                     size_t(2 * b->n) * sizeof(void *), hipMemcpyHostToDevice));
    auto kernel_node = [&](const spmv_batch::Group &g, const std::vector<hipGraphNode_t> &deps,
                           hipGraphNode_t *node) -> int {
        hipKernelNodeParams kp{};
        Item *items = g.d_items;
        int32_t *blk = g.d_blk;
        void *args[] = {&b->d_sh, &b->d_x, &b->d_y, &items, &blk};
        kp.func = reinterpret_cast<void *>(b->fn);
        kp.gridDim = dim3(g.grid);
        kp.blockDim = dim3(kBlock);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        SPMV_HIP(hipGraphAddKernelNode(node, b->graph, deps.data(), deps.size(), &kp));
        return SPMV_OK;
    };
    // receive chain, the node closing each chunk
    std::vector<hipGraphNode_t> recv_done(size_t(b->n_chunks), nullptr);
    hipGraphNode_t prev_recv = n_t;
    for (int32_t c = 0; c < b->n_chunks; ++c) {
        if (b->staging)
            for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
                const spmv_plan *p = b->plans[size_t(i)];
                const size_t nh = p->share.halo.size() * 8;
                if (!nh) continue;
                hipGraphNode_t nd;
                SPMV_HIP(hipGraphAddMemcpyNode1D(&nd, b->graph, &prev_recv, 1, p->d_recvbuf,
                                                 p->h_inbox, nh, hipMemcpyHostToDevice));
                prev_recv = nd;
            }
        recv_done[size_t(c)] = prev_recv;
    }
    hipGraphNode_t prev_k = n_t, prev_send = n_t;
    int32_t waited = -1;
    for (const auto &g : b->groups) {
        if (g.n_items == 0 && g.kind != spmv_batch::gPack) continue;
        std::vector<hipGraphNode_t> deps{prev_k};
        if (g.kind != spmv_batch::gPack && g.kind != spmv_batch::gLocal && g.chunk > waited) {
            deps.push_back(recv_done[size_t(g.chunk)]);
            waited = g.chunk;
        }
        hipGraphNode_t nd = nullptr;
        if (g.n_items > 0) {
            if (int rc = kernel_node(g, deps, &nd)) return rc;
        } else {
            SPMV_HIP(hipGraphAddEmptyNode(&nd, b->graph, deps.data(), deps.size()));
        }
        prev_k = nd;
        if (g.kind == spmv_batch::gPack && b->staging) {
            // the chunk's send copies after its Pack, chained behind earlier sends
            for (int32_t i = b->chunk_lo[size_t(g.chunk)]; i < b->chunk_lo[size_t(g.chunk) + 1];
                 ++i) {
                const spmv_plan *p = b->plans[size_t(i)];
                const size_t ns = p->share.send_idx.size() * 8;
                if (!ns) continue;
                hipGraphNode_t sd;
                hipGraphNode_t sdeps[2] = {prev_send, nd};
                SPMV_HIP(hipGraphAddMemcpyNode1D(&sd, b->graph, sdeps, 2, p->h_outbox,
                                                 p->d_sendbuf, ns, hipMemcpyDeviceToHost));
                prev_send = sd;
            }
        }
    }
    if (waited < b->n_chunks - 1 && b->n_chunks > 0) {
        // chunks without y_R work still join the receive chain
        hipGraphNode_t nd;
        hipGraphNode_t deps[2] = {prev_k, recv_done[size_t(b->n_chunks - 1)]};
        SPMV_HIP(hipGraphAddEmptyNode(&nd, b->graph, deps, 2));
        prev_k = nd;
    }
    if (prev_send != n_t) {
        hipGraphNode_t nd;
        hipGraphNode_t deps[2] = {prev_k, prev_send};
        SPMV_HIP(hipGraphAddEmptyNode(&nd, b->graph, deps, 2));
    }
    SPMV_HIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    return SPMV_OK;
}

}  // namespace

extern "C" int spmv_batch_create(spmv_plan_t *const *plans, int32_t n,
                                 const spmv_batch_opts_t *opts, spmv_batch_t **out)
{
    if (!out) return set_error(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || n < 1) return set_error(SPMV_EINVAL, "need at least one plan");
    spmv_batch_opts_t o{};
    if (opts) o = *opts;
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 32 || o.use_graph < 0 || o.use_graph > 2 ||
        o.persistent < 0 || o.persistent > 2 ||
        o.xcd_affinity < 0 || o.xcd_affinity > 2 || o.staging < 0 || o.staging > 1 ||
        o.copy_streams < 0 || o.copy_streams > kCopyStreams || o.chunks < 0 || o.chunks > 256)
        return set_error(SPMV_EINVAL, "batch option out of range");
    const int npt = plans[0] ? plans[0]->cfg[0].chunk : 0;
    const int vw = plans[0] ? plans[0]->cfg[0].width : 0;
    for (int32_t i = 0; i < n; ++i) {
        const spmv_plan *p = plans[i];
        if (!p) return set_error(SPMV_EINVAL, "plan " + std::to_string(i) + " is NULL");
        if (p->host_only || p->device != plans[0]->device)
            return set_error(SPMV_EINVAL, "plan " + std::to_string(i) +
                                              " is host-only or on another device");
        for (int side = 0; side < 2; ++side) {
            const CsrCfg &c = p->cfg[side];
            const bool form_ok = c.form == 1 || (side == 0 && c.form == 4) ||
                                 (side == 1 && c.form == 5 && c.rows <= 1);
            if (c.kernel != SPMV_KERNEL_STREAM || c.chunk != npt || c.width != vw || !form_ok)
                return set_error(SPMV_EINVAL, "plan " + std::to_string(i) +
                                                  ": batched shares need stream-CSR products "
                                                  "in packed tiles (y_R also in column slabs "
                                                  "of 256 / lanes rows per tile) with one "
                                                  "common chunk and width");
        }
    }
    const int dev = plans[0]->device;
    int cur_dev = 0;
    SPMV_HIP(hipGetDevice(&cur_dev));
    if (cur_dev != dev) SPMV_HIP(hipSetDevice(dev));
    auto *b = new (std::nothrow) spmv_batch();
    if (!b) return set_error(SPMV_ENOMEM, "batch allocation");
    b->plans.assign(plans, plans + n);
    b->n = n;
    b->npt = npt;
    b->vw = vw;
    b->device = dev;
    // automatic: one block per item (the persistent blocks pay a chain of
    // dependent loads per item: item, share descriptor, tile bounds)
    b->flat = o.persistent != 1;
    b->fn = grouped_fn(npt, vw, b->flat);
    b->n_blocks = kCUs * (o.blocks_per_cu ? o.blocks_per_cu : 8);
    // automatic: stream launches when the halo is staged (the graph runs its
    // copy nodes one after another: 46 ms per batch of 64 power-law shares
    // against 31-37 ms with one copy stream per direction), the graph when
    // only the grouped kernels run
    b->use_graph = o.use_graph == 1 || (o.use_graph == 0 && o.staging == 1);
    b->staging = o.staging == 0;
    b->n_cs = o.copy_streams ? o.copy_streams : 1;
    // automatic chunks: one per 8 shares (y_R of a chunk overlaps the
    // copies of later chunks, and with XCD affinity a chunk's Pack and y_L
    // keep one share per XCD)
    b->n_chunks = o.chunks ? std::min<int32_t>(o.chunks, n) : std::max<int32_t>(1, n / kXcds);
    // automatic affinity: when every chunk holds at least one share per XCD
    // (with fewer, the XCDs without a share would idle through that chunk's
    // Pack and y_L)
    b->xcd_aff = o.xcd_affinity == 1 || (o.xcd_affinity == 0 && n / b->n_chunks >= kXcds);
    b->chunk_lo.resize(size_t(b->n_chunks) + 1);
    for (int32_t c = 0; c <= b->n_chunks; ++c)
        b->chunk_lo[size_t(c)] = int32_t(int64_t(c) * n / b->n_chunks);

    // descriptors and work items
    std::vector<ShareDev> sh(static_cast<size_t>(n));
    struct Work {
        int32_t kind, chunk;
        std::vector<Item> items;
        std::vector<int64_t> cost;
        std::vector<int8_t> xcd;
        std::vector<uint8_t> ordered;
    };
    std::deque<Work> work;   // references stay valid while groups are added
    auto add_group = [&](int32_t kind, int32_t chunk) -> Work & {
        work.push_back({kind, chunk, {}, {}, {}, {}});
        return work.back();
    };
    const int gather_len = kBlock * npt;
    const int C = b->n_chunks;
    // per-share descriptors
    for (int32_t i = 0; i < n; ++i) {
        spmv_plan *p = plans[i];
        const Share &S = p->share;
        const CsrCfg &cr = p->cfg[1];
        sh[size_t(i)] = share_dev(p);
        // algorithmic bytes, as for one exec of the share
        const int64_t n_send = int64_t(S.send_idx.size()), n_halo = int64_t(S.halo.size());
        const int64_t nl = int64_t(S.L_col.size()), nr = int64_t(S.R_col.size());
        const int64_t rr = int64_t(S.R_rows.size()), nloc = S.n_loc;
        b->dev_bytes += 20 * n_send + 12 * nl + 4 * (nloc + 1) + 16 * nloc +
                        (p->fuse_unpack ? 0 : 20 * n_halo) + 12 * nr + 8 * rr + 4 + 8 * n_halo +
                        16 * rr;
        if (o.staging == 0) b->link_bytes += 8 * (n_send + n_halo);
    }
    auto share_xcd = [&](int32_t i) -> int8_t { return b->xcd_aff ? int8_t(i % kXcds) : int8_t(-1); };
    for (int32_t c = 0; c < C; ++c) {
        Work &w = add_group(spmv_batch::gPack, c);
        for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
            const int64_t n_send = int64_t(plans[i]->share.send_idx.size());
            for (int64_t a = 0; a < n_send; a += gather_len) {
                const int32_t len = int32_t(std::min<int64_t>(gather_len, n_send - a));
                w.items.push_back({kPack, i, int32_t(a), len});
                w.cost.push_back(len / 2 + 64);
                w.xcd.push_back(share_xcd(i));
                w.ordered.push_back(0);
            }
        }
        Work &wl = add_group(spmv_batch::gLocal, c);
        for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
            const auto &tl = plans[i]->cfg[0].tile_k;
            for (size_t t = 0; t + 1 < tl.size(); ++t) {
                wl.items.push_back({kLocal, i, int32_t(t), 0});
                wl.cost.push_back(tile_cost(tl, t));
                wl.xcd.push_back(share_xcd(i));
                wl.ordered.push_back(0);
            }
        }
    }
    for (int32_t c = 0; c < C; ++c) {
        Work &wu = add_group(spmv_batch::gUnpack, c);
        for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
            if (plans[i]->fuse_unpack) continue;
            const int64_t n_halo = int64_t(plans[i]->share.halo.size());
            for (int64_t a = 0; a < n_halo; a += gather_len) {
                const int32_t len = int32_t(std::min<int64_t>(gather_len, n_halo - a));
                wu.items.push_back({kUnpack, i, int32_t(a), len});
                wu.cost.push_back(len / 2 + 64);
                wu.xcd.push_back(share_xcd(i));
                wu.ordered.push_back(0);
            }
        }
        Work &wr = add_group(spmv_batch::gRemote, c);
        for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
            const CsrCfg &cr = plans[i]->cfg[1];
            const auto &tr = cr.tile_k;
            if (cr.form == 5) {
                for (int k = 0; k < kSlabs; ++k)
                    for (int64_t t = cr.slab_tiles[k]; t + 1 < cr.slab_tiles[k + 1]; ++t) {
                        wr.items.push_back({kSlab, i, int32_t(t - cr.slab_tiles[k]), k});
                        wr.cost.push_back(tile_cost(tr, size_t(t)));
                        wr.xcd.push_back(int8_t(k));   // the slab's XCD
                        wr.ordered.push_back(1);       // in share order
                    }
            } else {
                for (size_t t = 0; t + 1 < tr.size(); ++t) {
                    wr.items.push_back({kRemote, i, int32_t(t), 0});
                    wr.cost.push_back(tile_cost(tr, t));
                    wr.xcd.push_back(share_xcd(i));
                    wr.ordered.push_back(0);
                }
            }
        }
        Work &ws = add_group(spmv_batch::gSlabSum, c);
        for (int32_t i = b->chunk_lo[size_t(c)]; i < b->chunk_lo[size_t(c) + 1]; ++i) {
            if (plans[i]->cfg[1].form != 5) continue;
            const int64_t n_rr = int64_t(plans[i]->share.R_rows.size());
            for (int64_t a = 0; a < n_rr; a += gather_len) {
                const int32_t len = int32_t(std::min<int64_t>(gather_len, n_rr - a));
                ws.items.push_back({kSlabSum, i, int32_t(a), len});
                ws.cost.push_back(len + 64);
                ws.xcd.push_back(share_xcd(i));
                ws.ordered.push_back(0);
            }
        }
    }
    std::vector<std::vector<Item>> grouped(work.size());
    std::vector<std::vector<int32_t>> blk(work.size());
    for (size_t g = 0; g < work.size(); ++g) {
        if (b->flat) {
            interleave(work[g].items, work[g].xcd, grouped[g]);
            blk[g].assign(1, 0);
        } else {
            assign(work[g].items, work[g].cost, work[g].xcd, work[g].ordered, b->n_blocks,
                   grouped[g], blk[g]);
        }
        const int64_t ni = int64_t(work[g].items.size());
        const int32_t kind = work[g].kind;
        b->n_items[kind == spmv_batch::gPack || kind == spmv_batch::gLocal ? 0
                   : kind == spmv_batch::gUnpack                          ? 1
                                                                          : 2] += ni;
    }

    // one device arena: descriptors, pointer tables, items, block offsets
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off_sh = 0;
    size_t off_xy = off_sh + al(sh.size() * sizeof(ShareDev));
    size_t cur = off_xy + al(size_t(2 * n) * sizeof(void *));
    std::vector<size_t> off_items(work.size()), off_blk(work.size());
    for (size_t g = 0; g < work.size(); ++g) {
        off_items[g] = cur;
        cur += al(std::max<size_t>(grouped[g].size(), 1) * sizeof(Item));
        off_blk[g] = cur;
        cur += al(blk[g].size() * sizeof(int32_t));
    }
    int rc = SPMV_OK;
    auto fail = [&](int code) {
        batch_release(b);
        return code;
    };
    hipError_t e = hipMalloc(&b->arena, cur);
    if (e != hipSuccess) return fail(hip_error(e, "hipMalloc(batch arena)"));
    b->arena_bytes = cur;
    char *base = static_cast<char *>(b->arena);
    b->d_sh = reinterpret_cast<ShareDev *>(base + off_sh);
    b->d_x = reinterpret_cast<const double **>(base + off_xy);
    b->d_y = reinterpret_cast<double **>(base + off_xy + size_t(n) * sizeof(void *));
    e = hipMemcpy(b->d_sh, sh.data(), sh.size() * sizeof(ShareDev), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_error(e, "hipMemcpy(batch descriptors)"));
    for (size_t g = 0; g < work.size(); ++g) {
        spmv_batch::Group G;
        G.kind = work[g].kind;
        G.chunk = work[g].chunk;
        G.n_items = int64_t(grouped[g].size());
        G.grid = b->flat ? unsigned(std::max<size_t>(grouped[g].size(), 1))
                         : unsigned(b->n_blocks);
        G.d_items = reinterpret_cast<Item *>(base + off_items[g]);
        G.d_blk = reinterpret_cast<int32_t *>(base + off_blk[g]);
        if (!grouped[g].empty()) {
            e = hipMemcpy(G.d_items, grouped[g].data(), grouped[g].size() * sizeof(Item),
                          hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(hip_error(e, "hipMemcpy(batch items)"));
        }
        e = hipMemcpy(G.d_blk, blk[g].data(), blk[g].size() * sizeof(int32_t),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(hip_error(e, "hipMemcpy(batch offsets)"));
        b->groups.push_back(G);
    }
    e = hipHostMalloc((void **)&b->h_xy, size_t(2 * n) * sizeof(void *), hipHostMallocDefault);
    if (e != hipSuccess) return fail(hip_error(e, "hipHostMalloc(batch table)"));
    std::memset(b->h_xy, 0, size_t(2 * n) * sizeof(void *));
    hipStream_t plan_st[1];
    hipStream_t send_k[kCopyStreams], recv_k[kCopyStreams];
    if ((rc = pool_streams(dev, 1, plan_st, send_k, recv_k))) return fail(rc);
    b->pool_held = true;
    for (int k = 0; k < kCopyStreams; ++k) {
        b->cs_send_k[k] = send_k[k];
        b->cs_recv_k[k] = recv_k[k];
    }
    e = hipEventCreateWithFlags(&b->ev_f, hipEventDisableTiming);
    if (e != hipSuccess) return fail(hip_error(e, "hipEventCreate(batch)"));
    b->ev_pack.assign(size_t(C), nullptr);
    b->ev_recv.assign(size_t(C) * size_t(b->n_cs), nullptr);
    for (auto *v : {&b->ev_pack, &b->ev_recv})
        for (hipEvent_t &ev : *v) {
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return fail(hip_error(e, "hipEventCreate(batch)"));
        }
    for (int k = 0; k < b->n_cs; ++k) {
        e = hipEventCreateWithFlags(&b->ev_sk[k], hipEventDisableTiming);
        if (e != hipSuccess) return fail(hip_error(e, "hipEventCreate(batch)"));
    }
    if (b->use_graph && (rc = build_graph(b))) return fail(rc);
    *out = b;
    return SPMV_OK;
}

extern "C" int spmv_batch_exec(spmv_batch_t *b, const double *const *x, double *const *y,
                               void *stream_v)
{
    if (!b || !x || !y) return set_error(SPMV_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream_v);
    for (int32_t i = 0; i < b->n; ++i) {
        if (b->plans[size_t(i)]->share.n_loc > 0 && (!x[i] || !y[i] || x[i] == y[i]))
            return set_error(SPMV_EINVAL, "share " + std::to_string(i) + ": bad x/y");
        b->h_xy[i] = const_cast<double *>(x[i]);
        b->h_xy[b->n + i] = y[i];
    }
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev != b->device) SPMV_HIP(hipSetDevice(b->device));
    if (b->use_graph) {
        SPMV_HIP(hipGraphLaunch(b->gexec, s));
        SPMV_HIP(hipStreamSynchronize(s));
        return SPMV_OK;
    }
    if (int rc = issue(b, s)) return rc;
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

extern "C" int spmv_batch_info(const spmv_batch_t *b, spmv_batch_info_t *info)
{
    if (!b || !info) return set_error(SPMV_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n_shares = b->n;
    info->n_blocks = b->n_blocks;
    for (int ph = 0; ph < 3; ++ph) info->n_items[ph] = b->n_items[ph];
    info->device_bytes = b->dev_bytes;
    info->host_link_bytes = b->link_bytes;
    info->chunk = b->npt;
    info->width = b->vw;
    info->use_graph = b->use_graph ? 1 : 0;
    info->staging = b->staging ? 0 : 1;
    info->xcd_affinity = b->xcd_aff ? 1 : 0;
    info->n_chunks = b->n_chunks;
    info->persistent = b->flat ? 0 : 1;
    return SPMV_OK;
}

extern "C" int spmv_batch_destroy(spmv_batch_t *b)
{
    if (!b) return SPMV_OK;
    (void)hipDeviceSynchronize();
    batch_release(b);
    return SPMV_OK;
}

// ------------------------------------------------------------------------
// The resident step of one plan in two grouped launches, for a share whose
// y_R is in column slabs.  With the halo already in the receive buffer (read
// in place: fused Unpack), Pack, y_L and the slab tiles read nothing another
// of them writes, so they run as the work items of one launch, one block
// per item, each slab tile on its slab's XCD: Pack's streaming and y_L run
// beside the slabs' L2-bound gathers instead of before them.  The second
// launch adds the slab sums into y, which needs y_L's result there.  Each
// item runs the device code of the single-share kernels, so y has the bits
// of spmv_exec.  On the power-law 4M share (P = 16, rank 5) the step took
// 49.7 us against 57.0 op by op; with Pack and y_L mixed among the slab
// tiles instead of before them 53.4 us (y_L's x then shares each XCD's L2
// with the slab's x).  Where y_R is in packed tiles there is no such
// overlap to win and the generic item (its table entry, the share
// descriptor, then the tile) cost more than the launches it saves: 30.6-
// 31.8 us against 28.7-29.3 on the 27-point share, so those shares stay
// op by op.

namespace spmv {

struct ResidentProg {
    void *arena = nullptr;
    ShareDev *d_sh = nullptr;
    Item *d_a = nullptr, *d_b = nullptr;
    unsigned grid_a = 0, grid_b = 0;
    void (*fn)(const ShareDev *, const double *, double *, const Item *) = nullptr;
};

namespace {

template <int NPT, int VW>
__global__ __launch_bounds__(kBlock) void k_resident(const ShareDev *__restrict__ sh,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ y,
                                                     const Item *__restrict__ items)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock + 1];
    run_item<NPT, VW>(items[blockIdx.x], *sh, x, y, s_p, s_rp);
}

using ResidentFn = void (*)(const ShareDev *, const double *, double *, const Item *);

ResidentFn resident_fn(int npt, int vw)
{
    if (vw == 2) return npt == 4 ? k_resident<4, 2> : npt == 8 ? k_resident<8, 2> : npt == 16 ? k_resident<16, 2> : nullptr;
    if (vw == 4) return npt == 4 ? k_resident<4, 4> : npt == 8 ? k_resident<8, 4> : npt == 16 ? k_resident<16, 4> : nullptr;
    return nullptr;
}

// A launch's list, one block per item: block b runs on XCD b % 8, so the
// list is built in rounds of 8 slots, slot g of each round taking the next
// item of XCD g's queue (kNop once that queue is empty); XCD g's queue
// holds its `first` items, then its `second` items.
std::vector<Item> place_items(const std::vector<Item> (&first)[kXcds],
                              const std::vector<Item> (&second)[kXcds])
{
    std::vector<Item> q[kXcds];
    size_t rounds = 0;
    for (int g = 0; g < kXcds; ++g) {
        q[g] = first[g];
        q[g].insert(q[g].end(), second[g].begin(), second[g].end());
        rounds = std::max(rounds, q[g].size());
    }
    const Item nop{kNop, 0, 0, 0};
    std::vector<Item> out;
    out.reserve(rounds * kXcds);
    for (size_t r = 0; r < rounds; ++r)
        for (int g = 0; g < kXcds; ++g) out.push_back(r < q[g].size() ? q[g][r] : nop);
    while (!out.empty() && out.back().kind == kNop) out.pop_back();
    return out;
}

}  // namespace

int resident_build(spmv_plan *p)
{
    p->res = nullptr;
    const Share &S = p->share;
    const CsrCfg &cl = p->cfg[0], &cr = p->cfg[1];
    if (p->host_only || !p->fuse_unpack || S.n_loc <= 0 || S.R_rows.empty()) return SPMV_OK;
    if (cl.kernel != SPMV_KERNEL_STREAM || (cl.form != 1 && cl.form != 4)) return SPMV_OK;
    if (cr.kernel != SPMV_KERNEL_STREAM || cr.form != 5 || cr.rows > 1 || cr.chunk != cl.chunk ||
        cr.width != cl.width)
        return SPMV_OK;
    const ResidentFn fn = resident_fn(cl.chunk, cl.width);
    if (!fn) return SPMV_OK;
    const int gather_len = kBlock * cl.chunk;
    // y_L tiles, then Pack ranges, go to the XCDs by contiguous ranges (item
    // i of n on XCD 8 i / n), as the single-share kernels order their
    // blocks, and run after the XCD's slab tiles, filling the slab tiles'
    // ragged end: 42.6-42.9 us per step against 43.7-44.2 with y_L and Pack
    // first (y_L, slab tiles, Pack: 42.9-43.6; slab tiles, Pack, y_L:
    // 43.9-44.4; y_L and Pack alternating after the slab tiles: 0.6 us
    // slower; Pack spread evenly among the slab tiles, y_L and Pack
    // first: 2.7 us slower); the slab sums likewise
    auto xcd_of = [](int64_t i, int64_t n) { return int(i * kXcds / std::max<int64_t>(n, 1)); };
    std::vector<Item> a1[kXcds], a2[kXcds], b1[kXcds], none[kXcds];
    const int64_t n_lt = int64_t(cl.tile_k.size()) - 1;
    for (int64_t t = 0; t < n_lt; ++t) a1[xcd_of(t, n_lt)].push_back({kLocal, 0, int32_t(t), 0});
    const int64_t n_send = int64_t(S.send_idx.size());
    const int64_t n_pk = (n_send + gather_len - 1) / gather_len;
    for (int64_t j = 0; j < n_pk; ++j) {
        const int64_t a = j * gather_len;
        a1[xcd_of(j, n_pk)].push_back({kPack, 0, int32_t(a), int32_t(std::min<int64_t>(gather_len, n_send - a))});
    }
    for (int k = 0; k < kSlabs; ++k)
        for (int64_t t = cr.slab_tiles[k]; t + 1 < cr.slab_tiles[k + 1]; ++t)
            a2[k].push_back({kSlab, 0, int32_t(t - cr.slab_tiles[k]), k});
    // slab sums: one row per thread, so that each thread's 8 partial-sum
    // loads are its only trip before the y update
    const int64_t n_rr = int64_t(S.R_rows.size());
    const int64_t n_sum = (n_rr + kBlock - 1) / kBlock;
    for (int64_t j = 0; j < n_sum; ++j) {
        const int64_t a = j * kBlock;
        b1[xcd_of(j, n_sum)].push_back({kSlabSum, 0, int32_t(a), int32_t(std::min<int64_t>(kBlock, n_rr - a))});
    }
    const std::vector<Item> a_items = place_items(a2, a1);
    const std::vector<Item> b_items = place_items(b1, none);
    auto *r = new (std::nothrow) ResidentProg();
    if (!r) return set_error(SPMV_ENOMEM, "resident program");
    const size_t sh_bytes = (sizeof(ShareDev) + 255) & ~size_t(255);
    const size_t a_bytes = ((a_items.size() * sizeof(Item)) + 255) & ~size_t(255);
    const size_t b_bytes = std::max<size_t>(b_items.size() * sizeof(Item), 1);
    if (hipMalloc(&r->arena, sh_bytes + a_bytes + b_bytes) != hipSuccess) {
        delete r;
        return set_error(SPMV_EHIP, "resident program: hipMalloc failed");
    }
    char *base = static_cast<char *>(r->arena);
    r->d_sh = reinterpret_cast<ShareDev *>(base);
    r->d_a = reinterpret_cast<Item *>(base + sh_bytes);
    r->d_b = reinterpret_cast<Item *>(base + sh_bytes + a_bytes);
    const ShareDev d = share_dev(p);
    hipError_t e = hipMemcpy(r->d_sh, &d, sizeof(d), hipMemcpyHostToDevice);
    if (e == hipSuccess && !a_items.empty())
        e = hipMemcpy(r->d_a, a_items.data(), a_items.size() * sizeof(Item), hipMemcpyHostToDevice);
    if (e == hipSuccess && !b_items.empty())
        e = hipMemcpy(r->d_b, b_items.data(), b_items.size() * sizeof(Item), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(r->arena);
        delete r;
        return set_error(SPMV_EHIP, std::string("resident program: ") + hipGetErrorString(e));
    }
    r->grid_a = unsigned(a_items.size());
    r->grid_b = unsigned(b_items.size());
    r->fn = fn;
    p->res = r;
    return SPMV_OK;
}

void resident_free(spmv_plan *p)
{
    if (!p || !p->res) return;
    if (p->res->arena) (void)hipFree(p->res->arena);
    delete p->res;
    p->res = nullptr;
}

hipError_t resident_launch(const spmv_plan *p, int part, const double *x, double *y,
                           hipStream_t s)
{
    const ResidentProg *r = p->res;
    if (part != 1 && r->grid_a)
        hipLaunchKernelGGL(r->fn, dim3(r->grid_a), dim3(kBlock), 0, s, r->d_sh, x, y, r->d_a);
    if (part != 0 && r->grid_b)
        hipLaunchKernelGGL(r->fn, dim3(r->grid_b), dim3(kBlock), 0, s, r->d_sh, x, y, r->d_b);
    return hipGetLastError();
}

}  // namespace spmv
