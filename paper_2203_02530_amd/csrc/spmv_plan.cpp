// Plans and the executor: device upload of one rank share, and the token by
// token execution of a plan's operation order on HIP streams (Sec. III-A:
// the program is a traversal of its DAG; Table III: how its synchronisation
// tokens act).
//
// The halo exchange is emulated on one GPU: PostSend copies the packed send
// buffer into a pinned host outbox and PostRecv copies a pinned host inbox
// (filled by the caller with the values the other ranks would send) into the
// device receive buffer, each on a private copy stream; WaitSend/WaitRecv
// block the host on the copy's completion event, as MPI_Wait would.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>

#include "spmv_device.h"
#include "spmv_internal.h"

namespace spmv {

// Streams are shared by every plan on a device: plan stream i of any plan is
// pool stream i, plus one send and one receive copy stream.  Plans on one
// device then use a handful of HIP streams however many plans exist (many
// streams would be multiplexed over the few hardware queues and add latency),
// and since an exec ends with all its work finished, sharing adds no
// ordering that an exec on the same thread did not already have.  The pool
// counts its users (plans and batches); when the last one is released the
// streams are destroyed, so a process that destroys its objects leaves no
// HIP object of this library behind for the runtime's teardown at exit.
struct StreamPool {
    std::array<hipStream_t, SPMV_MAX_STREAMS + 2 * kCopyStreams> st{};
    int64_t users = 0;
};

namespace {
std::mutex g_pool_mu;
std::map<int, StreamPool> g_pools;
}  // namespace

int pool_streams(int device, int32_t n_plan, hipStream_t *plan_st, hipStream_t *send,
                 hipStream_t *recv)
{
    std::lock_guard<std::mutex> lock(g_pool_mu);
    StreamPool &pool = g_pools[device];
    auto get = [&](int32_t slot) -> int {
        if (!pool.st[size_t(slot)])
            SPMV_HIP(hipStreamCreateWithFlags(&pool.st[size_t(slot)], hipStreamNonBlocking));
        return SPMV_OK;
    };
    for (int32_t i = 0; i < n_plan; ++i) {
        if (int rc = get(i)) return rc;
        plan_st[i] = pool.st[size_t(i)];
    }
    // copy streams: [0] the coarse program's, all kCopyStreams for per-peer copies
    for (int32_t k = 0; k < kCopyStreams; ++k) {
        if (int rc = get(SPMV_MAX_STREAMS + k)) return rc;
        if (int rc = get(SPMV_MAX_STREAMS + kCopyStreams + k)) return rc;
        send[k] = pool.st[size_t(SPMV_MAX_STREAMS + k)];
        recv[k] = pool.st[size_t(SPMV_MAX_STREAMS + kCopyStreams + k)];
    }
    ++pool.users;   // only a successful acquisition is counted
    return SPMV_OK;
}

void pool_release(int device)
{
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_pools.find(device);
    if (it == g_pools.end() || it->second.users <= 0) return;
    if (--it->second.users > 0) return;
    for (hipStream_t &st : it->second.st)
        if (st) {
            (void)hipStreamDestroy(st);
            st = nullptr;
        }
}

namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// y_L's kernel can run Pack as extra blocks of its launch: the stream-CSR
// packed tiles (forms 1, 4) and the 16-bit sliced form (3).
bool packs_with_yl(const spmv_plan *p)
{
    const CsrCfg &c = p->cfg[0];
    return c.kernel == SPMV_KERNEL_STREAM && (c.form == 1 || c.form == 3 || c.form == 4);
}

// y_R can be added where y_L stores its rows (the resident step in one
// launch): y_L's kernel takes the extra work, the Unpack is fused, and
// y_R's kernel sums a row the way the fused sum does: the sliced form (an
// fma chain), or packed tiles with one summing lane and no row longer than
// a window (those a block sums with fma chains and a tree).  With y_L in
// packed tiles and y_R's rounded products, each tile's block loads its
// rows' remote entries beside its own (at most tile_remote_cap per tile)
// and the rows' storing lanes add them up from LDS; otherwise each row's
// storing lane walks its remote entries after its local sum, so the rows
// must be short: the remote rows of a contiguous row block sit in its
// first and last tiles, on two XCDs.  Measured steps: 7-point share (one
// entry per remote row, sliced y_L) 10.6 us against 12.9 with y_R in a
// launch of its own, 10.1 once the last XCD takes its tiles from the end;
// 27-point share (nine) 30.2 us with the rows walked against 26.3-27.2,
// 26.5-27.6 with the tiles split among the XCDs by a cost that counts a
// remote entry three times, 24.9-26.7 with the tiles' blocks loading them.
constexpr int kFuseMaxRemote = 4;

int tile_remote_cap(const spmv_plan *p)
{
    return std::min(kTileRemoteCap, stream_cap(p->cfg[0].chunk));
}

bool remote_by_tile(const spmv_plan *p) { return p->cfg[0].form != 3 && p->cfg[1].form == 1; }

// The tiles of a one-launch step whose tiles load their rows' remote
// entries go to the XCDs in contiguous ranges (neighbouring tiles share x
// lines in one L2) of equal cost, a remote entry counted twice a local
// one: the remote rows of a contiguous row block sit in its first and
// last tiles, which equal ranges put on two XCDs (27-point share: 24.0-25.4
// us against 25.0-26.2 with equal ranges; weights 1, 3, 4 and 6 measured
// 23.9-25.2, 24.5-25.5, 24.7-25.6 and 25.8-27.2).
constexpr double kRemoteEntryCost = 2.0;

void xcd_ranges(const CsrCfg &c, const std::vector<int32_t> &te, RemoteFuse &rf)
{
    const int64_t nt = int64_t(c.tile_row.size()) - 1;
    std::vector<double> pre(size_t(nt + 1), 0.0);
    for (int64_t t = 0; t < nt; ++t)
        pre[size_t(t + 1)] = pre[size_t(t)] + double(c.tile_k[size_t(t + 1)] - c.tile_k[size_t(t)]) +
                             kRemoteEntryCost * double(te[size_t(t + 1)] - te[size_t(t)]);
    int64_t t = 0, longest = 0;
    rf.xr[0] = 0;
    for (int x = 1; x < kXcds; ++x) {
        const double target = pre[size_t(nt)] * x / kXcds;
        while (t < nt && pre[size_t(t + 1)] <= target) ++t;
        rf.xr[x] = int32_t(t);
    }
    rf.xr[kXcds] = int32_t(nt);
    for (int x = 0; x < kXcds; ++x) longest = std::max<int64_t>(longest, rf.xr[x + 1] - rf.xr[x]);
    rf.n_grid = int32_t(kXcds * longest);
}

bool fuses_remote(const spmv_plan *p)
{
    const Share &S = p->share;
    const CsrCfg &c = p->cfg[1];
    if (!packs_with_yl(p) || !p->fuse_unpack || S.R_rows.empty()) return false;
    if (int64_t(S.send_idx.size()) > kPackTailMax || c.kernel != SPMV_KERNEL_STREAM) return false;
    if (c.form == 1) {
        if (c.lanes != 1) return false;
        const int cap = stream_cap(c.chunk);
        for (size_t t = 0; t + 1 < c.tile_row.size(); ++t)
            if (c.tile_row[t + 1] - c.tile_row[t] == 1 &&
                c.tile_k[t + 1] - (c.tile_k[t] & ~(c.width - 1)) > cap)
                return false;
    } else if (c.form != 2) {
        return false;
    }
    if (remote_by_tile(p)) {
        const std::vector<int32_t> &tr = p->cfg[0].tile_row;
        const int cap = tile_remote_cap(p);
        size_t j = 0;
        int32_t e_prev = 0;
        for (size_t t = 1; t < tr.size(); ++t) {
            while (j < S.R_rows.size() && S.R_rows[j] < tr[t]) ++j;
            if (S.R_ptr[j] - e_prev > cap) return false;
            e_prev = S.R_ptr[j];
        }
    } else {
        for (size_t j = 0; j + 1 < S.R_ptr.size(); ++j)
            if (S.R_ptr[j + 1] - S.R_ptr[j] > kFuseMaxRemote) return false;
    }
    return true;
}

void release(spmv_plan *p)
{
    if (!p) return;
    hipEvent_t *evs[] = {&p->ev_start, &p->ev_send, &p->ev_recv};
    for (hipEvent_t *e : evs)
        if (*e) (void)hipEventDestroy(*e);
    for (auto &e : p->ev_rec)
        if (e) (void)hipEventDestroy(e);
    for (auto *v : {&p->ev_pack, &p->ev_psend, &p->ev_precv})
        for (auto &e : *v)
            if (e) (void)hipEventDestroy(e);
    for (int i = 0; i <= SPMV_N_VERTICES; ++i) {
        if (p->ev_b[i]) (void)hipEventDestroy(p->ev_b[i]);
        if (p->ev_e[i]) (void)hipEventDestroy(p->ev_e[i]);
    }
    resident_free(p);
    if (p->arena) (void)hipFree(p->arena);
    if (p->h_inbox) (void)hipHostFree(p->h_inbox);
    if (p->h_outbox) (void)hipHostFree(p->h_outbox);
    if (p->pool_held) pool_release(p->device);
    delete p;
}

int allocate_and_upload(spmv_plan *p)
{
    const Share &S = p->share;
    SPMV_HIP(hipGetDevice(&p->device));
    // one arena: int32 arrays first, then FP64 arrays, each 256-byte aligned
    struct Item {
        void **dst;
        size_t bytes;
        const void *src;
        size_t pad;  // zero bytes after the data
    };
    const size_t n_halo = S.halo.size(), n_send = S.send_idx.size(), n_rr = S.R_rows.size();
    const size_t pad = kEntryPad;
    // the resident step in y_L's launch: masks of remote rows per 64 local
    // rows, and A_R's CSR where y_R's arrays hold the sliced layout
    const bool rf = fuses_remote(p);
    const bool rf_copy = rf && p->cfg[1].form != 1;
    std::vector<uint64_t> rf_mask;
    std::vector<int32_t> rf_j0, rf_tj, rf_te;
    if (rf && remote_by_tile(p)) {   // each tile's compressed rows and entries
        const std::vector<int32_t> &tr = p->cfg[0].tile_row;
        rf_tj.resize(tr.size());
        rf_te.resize(tr.size());
        size_t j = 0;
        for (size_t t = 0; t < tr.size(); ++t) {
            while (j < n_rr && S.R_rows[j] < tr[t]) ++j;
            rf_tj[t] = int32_t(j);
            rf_te[t] = S.R_ptr[j];
        }
    }
    if (rf) {
        const int64_t ng = (S.n_loc + 63) / 64;
        rf_mask.assign(size_t(ng), 0);
        rf_j0.assign(size_t(ng), 0);
        size_t j = 0;
        for (int64_t g = 0; g < ng; ++g) {
            rf_j0[size_t(g)] = int32_t(j);
            for (; j < n_rr && S.R_rows[j] < (g + 1) * 64; ++j)
                rf_mask[size_t(g)] |= uint64_t(1) << (S.R_rows[j] - g * 64);
        }
    }
    // col/val of each product: the CSR arrays, or the sliced layout (form
    // 2), whose columns form 3 replaces by 16-bit offsets
    auto sliced = [&](int side) { return p->cfg[side].form == 2 || p->cfg[side].form == 3; };
    auto colsz = [&](int side) {
        if (p->cfg[side].form == 5) return p->cfg[side].slab_col.size() * 4;
        if (p->cfg[side].form == 3) return p->cfg[side].sell_off.size() * 2;
        if (p->cfg[side].form == 4) return p->cfg[side].tile_off.size() * 2;
        return (sliced(side) ? p->cfg[side].sell_col.size()
                             : (side == 0 ? S.L_col.size() : S.R_col.size())) * 4;
    };
    auto coldata = [&](int side) -> const void * {
        if (p->cfg[side].form == 5) return p->cfg[side].slab_col.data();
        if (p->cfg[side].form == 3) return p->cfg[side].sell_off.data();
        if (p->cfg[side].form == 4) return p->cfg[side].tile_off.data();
        return sliced(side) ? p->cfg[side].sell_col.data()
                            : (side == 0 ? S.L_col.data() : S.R_col.data());
    };
    auto valsz = [&](int side) {
        if (p->cfg[side].form == 5) return p->cfg[side].slab_val.size() * 8;
        return (sliced(side) ? p->cfg[side].sell_val.size()
                             : (side == 0 ? S.L_val.size() : S.R_val.size())) * 8;
    };
    auto valdata = [&](int side) -> const void * {
        if (p->cfg[side].form == 5) return p->cfg[side].slab_val.data();
        return sliced(side) ? p->cfg[side].sell_val.data()
                            : (side == 0 ? S.L_val.data() : S.R_val.data());
    };
    Item items[] = {
        {(void **)&p->dL_ptr, S.L_ptr.size() * 4, S.L_ptr.data(), 0},
        {(void **)&p->dL_col, colsz(0), coldata(0), pad * 4},
        {(void **)&p->dR_rows, S.R_rows.size() * 4, S.R_rows.data(), 0},
        {(void **)&p->dR_ptr, S.R_ptr.size() * 4, S.R_ptr.data(), 0},
        {(void **)&p->dR_col, colsz(1), coldata(1), pad * 4},
        {(void **)&p->d_send_idx, n_send * 4, S.send_idx.data(), 0},
        {(void **)&p->d_perm, n_halo * 4, S.unpack_perm.data(), 0},
        {(void **)&p->d_tile_row[0], p->cfg[0].tile_row.size() * 4, p->cfg[0].tile_row.data(), 0},
        {(void **)&p->d_tile_k[0], p->cfg[0].tile_k.size() * 4, p->cfg[0].tile_k.data(), 0},
        {(void **)&p->d_tile_row[1], p->cfg[1].tile_row.size() * 4, p->cfg[1].tile_row.data(), 0},
        {(void **)&p->d_tile_k[1], p->cfg[1].tile_k.size() * 4, p->cfg[1].tile_k.data(), 0},
        {(void **)&p->d_sell_ptr[0], p->cfg[0].sell_ptr.size() * 4, p->cfg[0].sell_ptr.data(), 0},
        {(void **)&p->d_sell_ptr[1], p->cfg[1].sell_ptr.size() * 4, p->cfg[1].sell_ptr.data(), 0},
        {(void **)&p->dL_val, valsz(0), valdata(0), pad * 8},
        {(void **)&p->dR_val, valsz(1), valdata(1), pad * 8},
        {(void **)&p->d_sendbuf, n_send * 8, nullptr, 0},
        {(void **)&p->d_recvbuf, n_halo * 8, nullptr, 0},
        {(void **)&p->d_xhalo, p->fuse_unpack ? 0 : n_halo * 8, nullptr, 0},
        {(void **)&p->d_part, n_rr * 8, nullptr, 0},
        {(void **)&p->d_slab_part, p->cfg[1].form == 5 ? kSlabs * n_rr * 8 : 0, nullptr, 0},
        {(void **)&p->d_rf_mask, rf_mask.size() * 8, rf_mask.data(), 0},
        {(void **)&p->d_rf_j0, rf_j0.size() * 4, rf_j0.data(), 0},
        {(void **)&p->d_rf_rp, rf_copy ? S.R_ptr.size() * 4 : 0, S.R_ptr.data(), 0},
        {(void **)&p->d_rf_col, rf_copy ? S.R_col.size() * 4 : 0, S.R_col.data(), 0},
        {(void **)&p->d_rf_val, rf_copy ? S.R_val.size() * 8 : 0, S.R_val.data(), 0},
        {(void **)&p->d_rf_tj, rf_tj.size() * 4, rf_tj.data(), 0},
        {(void **)&p->d_rf_te, rf_te.size() * 4, rf_te.data(), 0},
    };
    size_t total = 0;
    for (const Item &it : items) total += align_up(std::max<size_t>(it.bytes + it.pad, 1));
    SPMV_HIP(hipMalloc(&p->arena, total));
    p->arena_bytes = total;
    // zero everything first: padding after col/val, and the buffers
    SPMV_HIP(hipMemset(p->arena, 0, total));
    char *cur = static_cast<char *>(p->arena);
    for (const Item &it : items) {
        *it.dst = cur;
        if (it.src && it.bytes) SPMV_HIP(hipMemcpy(cur, it.src, it.bytes, hipMemcpyHostToDevice));
        cur += align_up(std::max<size_t>(it.bytes + it.pad, 1));
    }
    SPMV_HIP(hipHostMalloc((void **)&p->h_inbox, std::max<size_t>(n_halo * 8, 8),
                           hipHostMallocDefault));
    SPMV_HIP(hipHostMalloc((void **)&p->h_outbox, std::max<size_t>(n_send * 8, 8),
                           hipHostMallocDefault));
    std::memset(p->h_inbox, 0, std::max<size_t>(n_halo * 8, 8));
    std::memset(p->h_outbox, 0, std::max<size_t>(n_send * 8, 8));

    p->n_st = std::max<int32_t>(std::max(p->sch.n_streams_used, p->n_streams_max), 1);
    if (int rc = pool_streams(p->device, p->n_st, p->st, p->cs_send_k, p->cs_recv_k)) return rc;
    p->pool_held = true;
    p->cs_send = p->cs_send_k[0];
    p->cs_recv = p->cs_recv_k[0];
    SPMV_HIP(hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming));
    SPMV_HIP(hipEventCreateWithFlags(&p->ev_send, hipEventDisableTiming));
    SPMV_HIP(hipEventCreateWithFlags(&p->ev_recv, hipEventDisableTiming));
    for (auto &e : p->ev_rec) SPMV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (p->profile)
        for (int i = 0; i <= SPMV_N_VERTICES; ++i) {
            SPMV_HIP(hipEventCreate(&p->ev_b[i]));
            SPMV_HIP(hipEventCreate(&p->ev_e[i]));
        }
    if (rf) {
        p->rf.mask = p->d_rf_mask;
        p->rf.j0 = p->d_rf_j0;
        p->rf.rp = rf_copy ? p->d_rf_rp : p->dR_ptr;
        p->rf.col = rf_copy ? p->d_rf_col : p->dR_col;
        p->rf.val = rf_copy ? p->d_rf_val : p->dR_val;
        p->rf.xh = p->d_recvbuf;
        p->rf.fma_chain = p->cfg[1].form == 2 ? 1 : 0;
        if (!rf_tj.empty()) {
            p->rf.tj = p->d_rf_tj;
            p->rf.te = p->d_rf_te;
            p->rf.tile_cap = tile_remote_cap(p);
            if (p->xcd_remap == 1) xcd_ranges(p->cfg[0], rf_te, p->rf);
        }
    }
    if (int rc = resident_build(p)) return rc;
    SPMV_HIP(hipDeviceSynchronize());
    return SPMV_OK;
}

// y_R adds into y itself when it runs after y_L on the same stream;
// otherwise its partial sums are added by a combine step at end.
bool fuses_combine(const Schedule &sch)
{
    if (!sch.multi) return false;
    auto pos = [&](int32_t tok) {
        return std::find(sch.order.begin(), sch.order.end(), tok) - sch.order.begin();
    };
    return sch.stream[SPMV_OP_YL] == sch.stream[SPMV_OP_YR] && pos(SPMV_OP_YL) < pos(SPMV_OP_YR);
}

}  // namespace
}  // namespace spmv

using namespace spmv;

namespace {

CsrDev local_csr(const spmv_plan *p)
{
    CsrDev A;
    A.n_rows = int32_t(p->share.n_loc);
    A.rp = p->dL_ptr;
    A.col = p->dL_col;
    A.val = p->dL_val;
    A.nnz_alloc = int64_t(p->share.L_col.size()) + kEntryPad;
    A.n_x = p->share.n_loc;
    return A;
}

CsrDev remote_csr(const spmv_plan *p)
{
    CsrDev A;
    A.n_rows = int32_t(p->share.R_rows.size());
    A.rp = p->dR_ptr;
    A.col = p->dR_col;
    A.val = p->dR_val;
    A.rows = p->dR_rows;
    A.nnz_alloc = int64_t(p->share.R_col.size()) + kEntryPad;
    A.n_x = int64_t(p->share.halo.size());
    return A;
}

// The padding a sliced layout may add (padded entries / entries), and the
// widest rows for which the automatic choice takes the sliced form: on the
// 7-point share (rows <= 7, one width for all slices) it ran y_L in 10.8 us
// against 11.7 for packed tiles; on the 27-point share packed tiles won
// (25.3 vs 28.2 us).
constexpr double kSellMaxRatio = 1.15;
constexpr int32_t kAutoSellWidth = 8;

// Resolve the automatic choices for one product and cut its stream tiles.
void configure(CsrCfg &c, const std::vector<int32_t> &rp, int64_t n_rows, int32_t kernel,
               int32_t lanes, int32_t rows, int32_t chunk, int32_t width, int32_t form)
{
    const int64_t nnz = n_rows > 0 ? rp[size_t(n_rows)] : 0;
    // Stream CSR measured faster than vector CSR on the stencil shares
    // (7-point 12.0 vs 15.4 us, 27-point 27.3 vs 35.1 us on MI355X); the
    // vector kernel remains for arrays beyond 32-bit buffer offsets.
    const int64_t kMax = (int64_t(1) << 32) - 64;
    const bool fits = (nnz + kEntryPad) * 8 < kMax;
    // knobs that only the vector kernel has (rows per group, > 16 lanes)
    // select it when the kernel is left automatic
    const bool vector_knobs = rows != 0 || lanes > 16;
    c.kernel = kernel ? kernel
                      : (fits && !vector_knobs ? SPMV_KERNEL_STREAM : SPMV_KERNEL_VECTOR);
    if (c.kernel == SPMV_KERNEL_VECTOR) {
        c.lanes = lanes ? lanes : auto_lanes(nnz, n_rows);
        c.rows = rows ? rows : auto_rows(c.lanes, n_rows);
        return;
    }
    // A window of 1024 entries (chunk 4) measured best for short and long
    // stencil rows alike (7-point 11.7 us vs 12.3 with chunk 8; 27-point
    // 25.0 vs 25.5), width 2 beat width 4 on both.  Summing lanes: about
    // one per 7 entries of the mean row (27-point, 25.8 entries: 2 lanes
    // 25.0 us, 1 lane 26.5, 4 lanes 25.8; power-law remote rows, 15.3
    // entries: 2 lanes 65 us, 1 lane 70.8; 7-point: 1 lane).
    const double mean_len = n_rows > 0 ? double(nnz) / double(n_rows) : 1.0;
    c.chunk = chunk ? chunk : 4;
    c.width = width ? width : 2;
    if (lanes) {
        c.lanes = lanes;
    } else {
        c.lanes = 1;
        while (c.lanes < 16 && double(c.lanes) * 14.0 <= mean_len) c.lanes <<= 1;
    }
    build_tiles(rp, n_rows, stream_cap(c.chunk), stream_maxr(c.lanes), c.width, c.tile_row,
                c.tile_k);
    c.form = form;   // 0 = automatic, resolved by select_sell
}

// Sliced ELL for a stream product when its form asks for it (2 or 3) and
// its rows are even enough (padding within kSellMaxRatio), or when the form
// is automatic (0) and moreover every slice has one width of at most
// kAutoSellWidth; otherwise packed tiles stay.  U (entries per batch of
// loads) is the chunk when given, else the smallest of 4, 8, 16 that covers
// the widest slice (16 beyond).  Form 3 (and the automatic choice, once
// sliced) stores the columns as 16-bit offsets from the row when the
// product's columns index the rows' own vector (y_L: `row_relative`), every
// slice has one width and every offset fits; else form 2 stays.  Its U is
// 8 or 16 (a chunk of 4 or 8 gives 8).
void select_sell(CsrCfg &c, const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                 const std::vector<double> &val, int64_t n_rows, int32_t chunk,
                 bool row_relative)
{
    const bool ask = c.kernel == SPMV_KERNEL_STREAM && c.form != 1 && c.form != 4;
    const bool ok = ask && build_sell(rp, col, val, n_rows, kSellMaxRatio, c.sell_ptr,
                                      c.sell_col, c.sell_val, c.sell_width, c.sell_uniform);
    if (!ok || (c.form == 0 && !(c.sell_uniform && c.sell_width <= kAutoSellWidth))) {
        c.form = 1;
        c.sell_ptr.clear();
        c.sell_col.clear();
        c.sell_val.clear();
        return;
    }
    const int32_t asked = c.form;
    c.form = 2;
    c.chunk = chunk ? chunk : c.sell_width <= 4 ? 4 : c.sell_width <= 8 ? 8 : 16;
    c.lanes = 1;
    c.tile_row.clear();
    c.tile_k.clear();
    if (row_relative && c.sell_uniform && c.sell_width > 0 && (asked == 3 || asked == 0) &&
        build_sell16(rp, col, n_rows, c.sell_width, c.sell_off)) {
        c.form = 3;
        c.sell_col.clear();
        c.sell_col.shrink_to_fit();
        pair_values(c.sell_val, int64_t(c.sell_ptr.size()) - 1, c.sell_width);
        c.chunk = chunk ? (chunk <= 8 ? 8 : 16) : (c.sell_width <= 8 ? 8 : 16);
    }
}

// Form 4 for y_L in packed tiles when asked for (4) or automatic (0):
// columns as int16 offsets from the first row of each tile, when they fit;
// else the 32-bit columns stay (form 1).
void select_tile16(CsrCfg &c, const std::vector<int32_t> &col, int32_t asked)
{
    if (c.kernel != SPMV_KERNEL_STREAM || c.form != 1 || (asked != 0 && asked != 4)) return;
    if (build_tile16(col, c.tile_row, c.tile_k, c.tile_off)) c.form = 4;
}

// Column slabs (form 5) when asked for, or automatically for a y_R whose
// halo is larger than one XCD's L2: there every gather of the packed form
// fetches a cache line from the MALL or HBM (the power-law share's y_R moved
// 6.3 times its bytes in packed tiles), while a slab's eighth of the halo
// stays in its XCD's L2.
constexpr int64_t kXcdL2Bytes = int64_t(4) << 20;

bool want_slabs(int32_t form, int32_t kernel, int64_t n_halo, int64_t n_remote_rows)
{
    if (kernel == SPMV_KERNEL_VECTOR) return false;
    return form == 5 || (form == 0 && n_remote_rows > 0 && n_halo * 8 > kXcdL2Bytes);
}

// Form 5 for y_R: column slabs (see SlabDev), each cut into stream tiles.
// Rows per thread `rows` > 1 selects wide tiles of up to rows * 256 rows
// with one thread per row and windows of 256 * chunk entries (chunk 8 unless
// given); otherwise (the automatic choice) tiles of 256 / lanes rows with
// summing lanes by the mean row length within a slab (at most 4).  On the
// power-law 4M share (about 2 entries per row and slab) wide tiles measured
// 36.1-42.9 us against 35.8 us for tiles of 256 rows: the slab's gathers
// from L2 bound both, so filling the windows gains nothing.  Without remote
// rows the packed form stays.  Returns whether the slabs were built.
bool select_slabs(CsrCfg &c, const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                  const std::vector<double> &val, int64_t n_rows, int64_t n_x, int32_t lanes,
                  int32_t rows, int32_t chunk)
{
    if (c.kernel != SPMV_KERNEL_STREAM || c.form != 5) return false;
    if (n_rows <= 0 || n_x <= 0) {
        c.form = 1;
        return false;
    }
    const double mean = double(rp[size_t(n_rows)]) / double(kSlabs * n_rows);
    const int32_t lanes_packed = c.lanes, chunk_packed = c.chunk;
    const bool wide = rows > 1;
    if (wide) {
        c.rows = rows > 1 ? rows : 4;
        c.lanes = 1;
        c.chunk = chunk ? chunk : 8;
    } else {
        c.rows = 1;
        if (lanes) {
            c.lanes = lanes;
        } else {
            c.lanes = 1;
            while (c.lanes < 4 && double(c.lanes) * 14.0 <= mean) c.lanes <<= 1;
        }
    }
    const int maxr = wide ? c.rows * stream_maxr(1) : stream_maxr(c.lanes);
    std::vector<int32_t> tile_row, tile_k;
    build_slabs(rp, col, val, n_rows, n_x, stream_cap(c.chunk), maxr, c.width, c.sell_ptr,
                c.slab_col, c.slab_val, tile_row, tile_k, c.slab_nnz, c.slab_tiles);
    // the stream kernel addresses the values through 32-bit byte offsets;
    // the slabs' alignment padding can push a share at the limit past it
    constexpr int64_t kMax = (int64_t(1) << 32) - 64;
    if ((int64_t(c.slab_val.size()) + kEntryPad) * 8 >= kMax) {
        c.form = 1;
        c.lanes = lanes_packed;
        c.chunk = chunk_packed;
        c.rows = 1;
        c.sell_ptr.clear();
        c.slab_col.clear();
        c.slab_val.clear();
        return false;
    }
    c.tile_row.swap(tile_row);
    c.tile_k.swap(tile_k);
    return true;
}

// `tail`: Pack blocks appended to the launch (y_L in a stream-CSR packed or
// 16-bit sliced form only, see packs_with_yl).
hipError_t launch_product(const spmv_plan *p, int side, const double *x, double *out,
                          double *acc, hipStream_t s, const PackTail &tail = PackTail(),
                          const RemoteFuse &rem = RemoteFuse())
{
    CsrDev A = side == 0 ? local_csr(p) : remote_csr(p);
    const CsrCfg &c = p->cfg[side];
    if (c.kernel == SPMV_KERNEL_STREAM && c.form == 5) {
        SlabDev D;
        D.rp = p->d_sell_ptr[side];
        D.col = A.col;
        D.val = A.val;
        D.tile_row = p->d_tile_row[side];
        D.tile_k = p->d_tile_k[side];
        D.rows = A.rows;
        D.x = x;
        D.part = p->d_slab_part;
        D.out = out;
        D.acc = acc;
        D.n_rows = A.n_rows;
        D.chunk = c.chunk;
        D.width = c.width;
        D.lanes = c.lanes;
        D.rpt = c.rows;
        for (int k = 0; k <= kSlabs; ++k) {
            D.nnz_off[k] = c.slab_nnz[k];
            D.tile_off[k] = c.slab_tiles[k];
        }
        D.nnz_alloc = int64_t(c.slab_col.size()) + kEntryPad;
        D.n_x = A.n_x;
        return launch_slabs(D, s);
    }
    if (c.kernel == SPMV_KERNEL_STREAM && (c.form == 2 || c.form == 3)) {
        A.sell_ptr = p->d_sell_ptr[side];
        A.n_slices = int32_t(c.sell_ptr.size()) - 1;
        A.sell_u = c.chunk;
        A.sell_width = c.sell_uniform ? c.sell_width : 0;
        A.nnz_alloc = int64_t(c.sell_val.size()) + kEntryPad;
        if (c.form == 3) {
            A.off_bytes = uint32_t((c.sell_off.size() + 2 * kEntryPad) * 2);
            return launch_sell16(A, x, out, p->xcd_remap, s, tail, rem);
        }
        return launch_sell(A, x, out, acc, p->xcd_remap, s);
    }
    if (c.kernel == SPMV_KERNEL_STREAM) {
        A.tile_row = p->d_tile_row[side];
        A.tile_k = p->d_tile_k[side];
        A.n_tiles = int32_t(c.tile_row.size()) - 1;
        A.col16 = c.form == 4;
        return launch_csr_stream(A, x, out, acc, c.chunk, c.width, c.lanes, p->xcd_remap, s,
                                 tail, rem);
    }
    return launch_csr(A, x, out, acc, c.lanes, c.rows, p->xcd_remap, p->use_buffer, s);
}

}  // namespace

namespace {

template <class Build>
int create_plan(Build build_share_fn, int32_t nranks, const int32_t *op_order, int32_t n_ops,
                const int32_t *stream_map, int32_t n_streams, const spmv_tune_t *tune,
                spmv_plan_t **out)
{
    if (!out) return set_error(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    spmv_tune_t t{};
    if (tune) t = *tune;
    auto valid_lanes = [](int32_t l) { return l == 0 || (l >= 1 && l <= 64 && !(l & (l - 1))); };
    auto valid_rows = [](int32_t r) { return r == 0 || r == 1 || r == 2 || r == 4 || r == 8; };
    auto valid_chunk = [](int32_t c) { return c == 0 || c == 4 || c == 8 || c == 16; };
    if (!valid_lanes(t.lanes_local) || !valid_lanes(t.lanes_remote))
        return set_error(SPMV_EINVAL, "lanes per row must be 0 or a power of two <= 64");
    if (!valid_rows(t.rows_local) || !valid_rows(t.rows_remote))
        return set_error(SPMV_EINVAL, "rows per lane group must be 0, 1, 2, 4 or 8");
    if (!valid_chunk(t.chunk_local) || !valid_chunk(t.chunk_remote))
        return set_error(SPMV_EINVAL, "chunk must be 0, 4, 8 or 16");
    if (t.kernel_local < 0 || t.kernel_local > 2 || t.kernel_remote < 0 || t.kernel_remote > 2)
        return set_error(SPMV_EINVAL, "kernel must be 0, 1 or 2");
    if ((t.kernel_local == SPMV_KERNEL_STREAM && t.lanes_local > 16) ||
        (t.kernel_remote == SPMV_KERNEL_STREAM && t.lanes_remote > 16))
        return set_error(SPMV_EINVAL, "stream CSR sums with at most 16 lanes per row");
    if (t.width != 0 && t.width != 2 && t.width != 4)
        return set_error(SPMV_EINVAL, "width must be 0, 2 or 4");
    if (t.xcd_remap < 0 || t.xcd_remap > 2 || t.fuse_unpack < 0 || t.fuse_unpack > 2)
        return set_error(SPMV_EINVAL, "tune field out of range");
    if (t.form < 0 || t.form > 5) return set_error(SPMV_EINVAL, "form must be 0 to 5");
    if (t.form == 5 && t.lanes_remote > 4)
        return set_error(SPMV_EINVAL, "column slabs sum with at most 4 lanes per row");
    if (t.form == 5 && t.rows_remote > 1 && t.lanes_remote > 1)
        return set_error(SPMV_EINVAL, "wide slab tiles (rows_remote > 1) sum with one lane");

    std::vector<int32_t> def_ops;
    int32_t def_map[SPMV_N_VERTICES];
    if (!op_order) {
        default_order(nranks, def_ops, def_map);
        op_order = def_ops.data();
        n_ops = int32_t(def_ops.size());
        stream_map = def_map;
        n_streams = std::max<int32_t>(n_streams, nranks > 1 ? 2 : 1);
    }
    auto *p = new (std::nothrow) spmv_plan();
    if (!p) return set_error(SPMV_ENOMEM, "plan allocation");
    int rc = validate_schedule(nranks, op_order, n_ops, stream_map, n_streams, p->sch);
    if (rc == SPMV_OK) rc = build_share_fn(p->share);
    if (rc != SPMV_OK) {
        delete p;
        return rc;
    }
    const Share &S = p->share;
    {
        // the stream kernel addresses col/val/x through 32-bit buffer offsets
        const int64_t kMax = (int64_t(1) << 32) - 64;
        const bool big_l = (int64_t(S.L_col.size()) + kEntryPad) * 8 >= kMax || S.n_loc * 8 >= kMax;
        const bool big_r = (int64_t(S.R_col.size()) + kEntryPad) * 8 >= kMax ||
                           int64_t(S.halo.size()) * 8 >= kMax;
        if ((t.kernel_local == SPMV_KERNEL_STREAM && big_l) ||
            (t.kernel_remote == SPMV_KERNEL_STREAM && big_r)) {
            delete p;
            return set_error(SPMV_EINVAL, "stream CSR needs arrays below 4 GiB");
        }
    }
    // form 5 concerns y_R only; y_L then takes the automatic form
    const int32_t form_l = t.form == 5 ? 0 : t.form;
    const bool slabs = want_slabs(t.form, t.kernel_remote, int64_t(S.halo.size()),
                                  int64_t(S.R_rows.size()));
    configure(p->cfg[0], S.L_ptr, S.n_loc, t.kernel_local, t.lanes_local, t.rows_local,
              t.chunk_local, t.width, form_l);
    // in column slabs rows_remote counts rows per thread, not vector rows
    configure(p->cfg[1], S.R_ptr, int64_t(S.R_rows.size()), t.kernel_remote, t.lanes_remote,
              slabs ? 0 : t.rows_remote, t.chunk_remote, t.width, slabs ? 5 : t.form);
    select_sell(p->cfg[0], S.L_ptr, S.L_col, S.L_val, S.n_loc, t.chunk_local, true);
    select_tile16(p->cfg[0], S.L_col, form_l);
    if (!select_slabs(p->cfg[1], S.R_ptr, S.R_col, S.R_val, int64_t(S.R_rows.size()),
                      int64_t(S.halo.size()), t.lanes_remote, t.rows_remote, t.chunk_remote))
        select_sell(p->cfg[1], S.R_ptr, S.R_col, S.R_val, int64_t(S.R_rows.size()),
                    t.chunk_remote, false);
    p->xcd_remap = t.xcd_remap ? t.xcd_remap : 1;
    // y_R can read the receive buffer in place exactly when the unpack
    // permutation is the identity (always, with the halo and the receive
    // buffer both in ascending global column order); the explicit kernel
    // stays available on request (fuse_unpack = 2)
    bool identity = true;
    for (size_t i = 0; i < S.unpack_perm.size() && identity; ++i)
        identity = S.unpack_perm[i] == int32_t(i);
    if (t.fuse_unpack == 1 && !identity) {
        delete p;
        return set_error(SPMV_EINVAL, "fuse_unpack = 1 needs the identity unpack permutation");
    }
    p->fuse_unpack = t.fuse_unpack == 1 || (t.fuse_unpack == 0 && identity);
    p->host_only = (t.flags & SPMV_F_HOST_ONLY) != 0;
    p->profile = (t.flags & SPMV_F_PROFILE) != 0;
    p->use_buffer = (t.flags & SPMV_F_NO_BUFFER) == 0;
    p->resident_seq = (t.flags & SPMV_F_RESIDENT_SEQUENTIAL) != 0;
    p->fused_combine = fuses_combine(p->sch);
    p->n_streams_max = n_streams;
    if (nranks > 1) p->fdag.build(p->share);
    if (!p->host_only) {
        rc = allocate_and_upload(p);
        if (rc != SPMV_OK) {
            release(p);
            return rc;
        }
    }
    *out = p;
    return SPMV_OK;
}

}  // namespace

extern "C" int spmv_plan_create_ex(const spmv_csr_t *csr, int32_t nranks, int32_t rank,
                                   const int32_t *op_order, int32_t n_ops,
                                   const int32_t *stream_map, int32_t n_streams,
                                   const spmv_tune_t *tune, spmv_plan_t **out)
{
    return create_plan([&](Share &S) { return build_share(csr, nranks, rank, S); }, nranks,
                       op_order, n_ops, stream_map, n_streams, tune, out);
}

extern "C" int spmv_plan_create_local(const spmv_csr_t *local, int64_t n_global, int32_t nranks,
                                      int32_t rank, const int32_t *send_idx,
                                      const int32_t *send_off, const int32_t *op_order,
                                      int32_t n_ops, const int32_t *stream_map,
                                      int32_t n_streams, const spmv_tune_t *tune,
                                      spmv_plan_t **out)
{
    return create_plan(
        [&](Share &S) {
            return build_share_local(local, n_global, nranks, rank, send_idx, send_off, S);
        },
        nranks, op_order, n_ops, stream_map, n_streams, tune, out);
}

extern "C" int spmv_plan_create(const spmv_csr_t *csr, int32_t nranks, int32_t rank,
                                const int32_t *op_order, int32_t n_ops,
                                const int32_t *stream_map, int32_t n_streams, spmv_plan_t **out)
{
    return spmv_plan_create_ex(csr, nranks, rank, op_order, n_ops, stream_map, n_streams,
                               nullptr, out);
}

extern "C" int spmv_plan_destroy(spmv_plan_t *plan)
{
    if (!plan) return SPMV_OK;
    if (!plan->host_only) {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && dev != plan->device) (void)hipSetDevice(plan->device);
        (void)hipDeviceSynchronize();
    }
    release(plan);
    return SPMV_OK;
}

namespace {

inline hipError_t prof_begin(spmv_plan *p, int slot, hipStream_t s)
{
    return p->profile ? hipEventRecord(p->ev_b[slot], s) : hipSuccess;
}
inline hipError_t prof_end(spmv_plan *p, int slot, hipStream_t s)
{
    return p->profile ? hipEventRecord(p->ev_e[slot], s) : hipSuccess;
}

}  // namespace

namespace {

// Host timeline of one exec (profiling mode 2): marks the end of each
// token's host call, relative to the exec's entry.
struct HostMarks {
    spmv_plan_t *p;
    std::chrono::steady_clock::time_point t0;
    size_t k = 0;
    HostMarks(spmv_plan_t *plan, size_t n_tokens) : p(plan)
    {
        if (!p->host_times) return;
        if (p->host_us.size() != n_tokens) {
            p->host_us.assign(n_tokens, 0.0);
            p->host_n = 0.0;
        }
        t0 = std::chrono::steady_clock::now();
    }
    void mark()
    {
        if (p->host_times && k < p->host_us.size())
            p->host_us[k] += std::chrono::duration<double, std::micro>(
                                 std::chrono::steady_clock::now() - t0).count();
        ++k;
    }
    void done()
    {
        if (p->host_times) p->host_n += 1.0;
    }
};

// The streams an exec runs its plan streams on: plan stream 0 is the
// caller's stream itself (so a one-stream plan needs no start or end
// events), the others come from the device pool.
void plan_streams(const spmv_plan_t *p, hipStream_t caller, int32_t n_used, hipStream_t *st)
{
    st[0] = caller;
    for (int32_t i = 1; i < n_used; ++i) st[i] = p->st[i];
}

// start: the plan streams other than the caller's wait for work already
// issued to the caller's stream.  When that stream is idle there is nothing
// to wait for, and the record/wait pair (about 11 us of host time on a
// legacy null stream) is skipped.
hipError_t start_join(spmv_plan_t *p, hipStream_t caller, int32_t n_used, const hipStream_t *st)
{
    if (n_used <= 1) return hipSuccess;
    const hipError_t q = hipStreamQuery(caller);
    if (q == hipSuccess) return hipSuccess;
    if (q != hipErrorNotReady) return q;
    hipError_t e = hipEventRecord(p->ev_start, caller);
    for (int32_t i = 1; i < n_used && e == hipSuccess; ++i)
        e = hipStreamWaitEvent(st[i], p->ev_start, 0);
    return e;
}

// end: the host waits for the other plan streams itself (the exec returns
// only after everything, so later work on the caller's stream is ordered
// after it without a device-side wait, which cost a cross-queue round
// trip); a stream synchronisation returns at once on an idle stream, where
// a freshly recorded event would cost a round trip through the device.
hipError_t end_join(int32_t n_used, const hipStream_t *st)
{
    for (int32_t i = 1; i < n_used; ++i) {
        const hipError_t e = hipStreamSynchronize(st[i]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One exec of a fine-grained order (per-peer Pack, copies and waits; see
// spmv_fine.cpp).  Per-op profiling is not kept in this mode.
int exec_fine(spmv_plan_t *p, const double *x, double *y, hipStream_t caller)
{
    const Share &S = p->share;
    const FineSchedule &F = p->fsch;
    const int32_t n_used = std::max<int32_t>(F.n_streams_used, 1);
    const int64_t n_halo = int64_t(S.halo.size()), n_rr = int64_t(S.R_rows.size());
    std::vector<int32_t> pack_stream(size_t(S.nranks), 0);
    for (size_t k = 0; k < F.order.size(); ++k)
        if (tok_kind(F.order[k]) == 0 && tok_op(F.order[k]) == SPMV_OP_PACK)
            pack_stream[size_t(tok_peer(F.order[k]))] = F.ostream[k];
    hipStream_t st[SPMV_MAX_STREAMS];
    plan_streams(p, caller, n_used, st);
    HostMarks hm(p, F.order.size());
    bool combine = false;
    for (size_t k = 0; k < F.order.size(); ++k) {
        const int32_t t = F.order[k], kind = tok_kind(t), op = tok_op(t), q = tok_peer(t);
        if (kind == SPMV_SYNC_CER) {
            SPMV_HIP(hipEventRecord(p->ev_pack[size_t(q)], st[pack_stream[size_t(q)]]));
            hm.mark();
            continue;
        }
        if (kind == SPMV_SYNC_CES) {
            SPMV_HIP(hipEventSynchronize(p->ev_pack[size_t(q)]));
            hm.mark();
            continue;
        }
        const hipStream_t s = F.ostream[k] >= 0 ? st[F.ostream[k]] : nullptr;
        const int64_t so = q >= 0 ? S.send_off[size_t(q)] : 0;
        const int64_t sn = q >= 0 ? S.send_off[size_t(q) + 1] - so : 0;
        const int64_t ro = q >= 0 ? S.recv_off[size_t(q)] : 0;
        const int64_t rn = q >= 0 ? S.recv_off[size_t(q) + 1] - ro : 0;
        switch (op) {
            case SPMV_OP_START:
                SPMV_HIP(start_join(p, caller, n_used, st));
                break;
            case SPMV_OP_PACK:
                SPMV_HIP(launch_pack(x, p->d_send_idx + so, p->d_sendbuf + so, sn, s));
                break;
            case SPMV_OP_YL: SPMV_HIP(launch_product(p, 0, x, y, nullptr, s)); break;
            case SPMV_OP_POST_SEND: {
                // each peer's copy on its own copy stream, like concurrent sends
                const hipStream_t cs = p->cs_send_k[size_t(q) % kCopyStreams];
                SPMV_HIP(hipMemcpyAsync(p->h_outbox + so, p->d_sendbuf + so, size_t(sn) * 8,
                                        hipMemcpyDeviceToHost, cs));
                SPMV_HIP(hipEventRecord(p->ev_psend[size_t(q)], cs));
                break;
            }
            case SPMV_OP_POST_RECV: {
                const hipStream_t cs = p->cs_recv_k[size_t(q) % kCopyStreams];
                SPMV_HIP(hipMemcpyAsync(p->d_recvbuf + ro, p->h_inbox + ro, size_t(rn) * 8,
                                        hipMemcpyHostToDevice, cs));
                SPMV_HIP(hipEventRecord(p->ev_precv[size_t(q)], cs));
                break;
            }
            case SPMV_OP_WAIT_SEND: SPMV_HIP(hipEventSynchronize(p->ev_psend[size_t(q)])); break;
            case SPMV_OP_WAIT_RECV: SPMV_HIP(hipEventSynchronize(p->ev_precv[size_t(q)])); break;
            case SPMV_OP_YR: {
                // Unpack, implied on y_R's stream right before it
                if (!p->fuse_unpack)
                    SPMV_HIP(launch_unpack(p->d_recvbuf, p->d_perm, p->d_xhalo, n_halo, s));
                const double *xh = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
                if (p->fused_combine)
                    SPMV_HIP(launch_product(p, 1, xh, nullptr, y, s));
                else
                    SPMV_HIP(launch_product(p, 1, xh, p->d_part, nullptr, s));
                combine = !p->fused_combine && n_rr > 0;
                break;
            }
            case SPMV_OP_END:
                SPMV_HIP(end_join(n_used, st));
                if (combine) SPMV_HIP(launch_combine(p->dR_rows, p->d_part, y, n_rr, caller));
                SPMV_HIP(hipStreamSynchronize(caller));
                break;
            default: return set_error(SPMV_EPLAN, "unexpected token in fine-grained schedule");
        }
        hm.mark();
    }
    hm.done();
    return SPMV_OK;
}

}  // namespace

extern "C" int spmv_exec(spmv_plan_t *p, const double *x, double *y, void *stream_v)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    const Share &S = p->share;
    if (S.n_loc > 0 && (!x || !y)) return set_error(SPMV_EINVAL, "x or y is NULL");
    if (x && y && x == y) return set_error(SPMV_EINVAL, "x and y alias");
    hipStream_t caller = static_cast<hipStream_t>(stream_v);
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev != p->device) SPMV_HIP(hipSetDevice(p->device));
    if (p->fine) return exec_fine(p, x, y, caller);

    const int32_t *smap = p->sch.stream;
    const int64_t n_send = int64_t(S.send_idx.size()), n_halo = int64_t(S.halo.size());
    const int64_t n_rr = int64_t(S.R_rows.size());
    bool ran[SPMV_N_VERTICES + 1] = {};
    bool combine = false;
    const int32_t n_used = std::max<int32_t>(p->sch.n_streams_used, 1);
    hipStream_t st[SPMV_MAX_STREAMS];
    plan_streams(p, caller, n_used, st);
    HostMarks hm(p, p->sch.order.size());

    for (int32_t tok : p->sch.order) {
        if (is_sync(tok)) {
            const int32_t kind = sync_kind(tok), v = sync_operand(tok);
            if (kind == SPMV_SYNC_CER) {
                SPMV_HIP(hipEventRecord(p->ev_rec[v], st[smap[v]]));
            } else {
                // the wait acts on the records of v's GPU predecessors
                const int32_t u = v == SPMV_OP_POST_SEND ? SPMV_OP_PACK
                                  : v == SPMV_OP_YR     ? SPMV_OP_UNPACK
                                                        : -1;
                if (u < 0) return set_error(SPMV_EPLAN, "synchronisation without a GPU predecessor");
                if (kind == SPMV_SYNC_CES)
                    SPMV_HIP(hipEventSynchronize(p->ev_rec[u]));
                else
                    SPMV_HIP(hipStreamWaitEvent(st[smap[v]], p->ev_rec[u], 0));
            }
            hm.mark();
            continue;
        }
        switch (tok) {
            case SPMV_OP_START:
                SPMV_HIP(start_join(p, caller, n_used, st));
                break;
            case SPMV_OP_PACK: {
                hipStream_t s = st[smap[tok]];
                SPMV_HIP(prof_begin(p, tok, s));
                SPMV_HIP(launch_pack(x, p->d_send_idx, p->d_sendbuf, n_send, s));
                SPMV_HIP(prof_end(p, tok, s));
                ran[tok] = true;
                break;
            }
            case SPMV_OP_YL: {
                hipStream_t s = st[smap[tok]];
                SPMV_HIP(prof_begin(p, tok, s));
                SPMV_HIP(launch_product(p, 0, x, y, nullptr, s));
                SPMV_HIP(prof_end(p, tok, s));
                ran[tok] = true;
                break;
            }
            case SPMV_OP_POST_SEND:
                SPMV_HIP(prof_begin(p, tok, p->cs_send));
                if (n_send)
                    SPMV_HIP(hipMemcpyAsync(p->h_outbox, p->d_sendbuf, size_t(n_send) * 8,
                                            hipMemcpyDeviceToHost, p->cs_send));
                SPMV_HIP(prof_end(p, tok, p->cs_send));
                SPMV_HIP(hipEventRecord(p->ev_send, p->cs_send));
                ran[tok] = true;
                break;
            case SPMV_OP_POST_RECV:
                SPMV_HIP(prof_begin(p, tok, p->cs_recv));
                if (n_halo)
                    SPMV_HIP(hipMemcpyAsync(p->d_recvbuf, p->h_inbox, size_t(n_halo) * 8,
                                            hipMemcpyHostToDevice, p->cs_recv));
                SPMV_HIP(prof_end(p, tok, p->cs_recv));
                SPMV_HIP(hipEventRecord(p->ev_recv, p->cs_recv));
                ran[tok] = true;
                break;
            case SPMV_OP_WAIT_SEND: SPMV_HIP(hipEventSynchronize(p->ev_send)); break;
            case SPMV_OP_WAIT_RECV: SPMV_HIP(hipEventSynchronize(p->ev_recv)); break;
            case SPMV_OP_UNPACK: {
                if (p->fuse_unpack) break;
                hipStream_t s = st[smap[tok]];
                SPMV_HIP(prof_begin(p, tok, s));
                SPMV_HIP(launch_unpack(p->d_recvbuf, p->d_perm, p->d_xhalo, n_halo, s));
                SPMV_HIP(prof_end(p, tok, s));
                ran[tok] = true;
                break;
            }
            case SPMV_OP_YR: {
                hipStream_t s = st[smap[tok]];
                const double *xh = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
                SPMV_HIP(prof_begin(p, tok, s));
                if (p->fused_combine)
                    SPMV_HIP(launch_product(p, 1, xh, nullptr, y, s));
                else
                    SPMV_HIP(launch_product(p, 1, xh, p->d_part, nullptr, s));
                SPMV_HIP(prof_end(p, tok, s));
                combine = !p->fused_combine && n_rr > 0;
                ran[tok] = true;
                break;
            }
            case SPMV_OP_END:
                SPMV_HIP(end_join(n_used, st));
                if (combine) {
                    SPMV_HIP(prof_begin(p, SPMV_N_VERTICES, caller));
                    SPMV_HIP(launch_combine(p->dR_rows, p->d_part, y, n_rr, caller));
                    SPMV_HIP(prof_end(p, SPMV_N_VERTICES, caller));
                    ran[SPMV_N_VERTICES] = true;
                }
                SPMV_HIP(hipStreamSynchronize(caller));
                break;
            default: return set_error(SPMV_EPLAN, "unexpected token in schedule");
        }
        hm.mark();
    }
    hm.done();
    if (p->profile) {
        for (int i = 0; i <= SPMV_N_VERTICES; ++i) {
            if (!ran[i]) continue;
            float ms = 0.f;
            SPMV_HIP(hipEventElapsedTime(&ms, p->ev_b[i], p->ev_e[i]));
            p->ms[i] += double(ms);
            p->cnt[i] += 1.0;
        }
    }
    return SPMV_OK;
}

extern "C" int spmv_exec_resident(spmv_plan_t *p, const double *x, double *y, void *stream_v)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    const Share &S = p->share;
    if (S.n_loc > 0 && (!x || !y)) return set_error(SPMV_EINVAL, "x or y is NULL");
    if (x && y && x == y) return set_error(SPMV_EINVAL, "x and y alias");
    hipStream_t s = static_cast<hipStream_t>(stream_v);
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev != p->device) SPMV_HIP(hipSetDevice(p->device));
    if (p->res && !p->resident_seq) {
        SPMV_HIP(resident_launch(p, -1, x, y, s));
        return SPMV_OK;
    }
    // Pack, y_L, Unpack, y_R in the order of the DAG's GPU vertices, on one
    // stream: y_R adds into what y_L stored, so y = fl(s_L + s_R) as in
    // every plan of spmv_exec.  Pack (it reads only x) runs as extra blocks
    // of y_L's launch where y_L's kernel takes them.
    const int64_t n_send = int64_t(S.send_idx.size());
    PackTail t;
    t.x = x;
    t.idx = p->d_send_idx;
    t.dst = p->d_sendbuf;
    t.n = int32_t(std::min<int64_t>(n_send, kPackTailMax));
    if (!p->resident_seq && p->rf.mask) {
        // the whole step in y_L's launch: Pack as extra blocks, each row's
        // remote sum added where its local sum is stored
        SPMV_HIP(launch_product(p, 0, x, y, nullptr, s, t, p->rf));
        return SPMV_OK;
    }
    if (!p->resident_seq && n_send > 0 && n_send <= kPackTailMax && packs_with_yl(p)) {
        SPMV_HIP(launch_product(p, 0, x, y, nullptr, s, t));
    } else {
        SPMV_HIP(launch_pack(x, p->d_send_idx, p->d_sendbuf, n_send, s));
        SPMV_HIP(launch_product(p, 0, x, y, nullptr, s));
    }
    if (!p->fuse_unpack)
        SPMV_HIP(launch_unpack(p->d_recvbuf, p->d_perm, p->d_xhalo, int64_t(S.halo.size()), s));
    if (!S.R_rows.empty()) {
        const double *xh = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
        SPMV_HIP(launch_product(p, 1, xh, nullptr, y, s));
    }
    return SPMV_OK;
}

extern "C" int spmv_exec_resident_part(spmv_plan_t *p, int32_t part, const double *x, double *y,
                                       void *stream_v)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    if (!p->res || p->resident_seq)
        return set_error(SPMV_ESTATE, "the plan's resident step is not grouped");
    if (part != 0 && part != 1) return set_error(SPMV_EINVAL, "part must be 0 or 1");
    if (!x || !y) return set_error(SPMV_EINVAL, "x or y is NULL");
    if (x == y) return set_error(SPMV_EINVAL, "x and y alias");
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev != p->device) SPMV_HIP(hipSetDevice(p->device));
    SPMV_HIP(resident_launch(p, part, x, y, static_cast<hipStream_t>(stream_v)));
    return SPMV_OK;
}

extern "C" int spmv_plan_device_buffers(const spmv_plan_t *p, double **send_dev, int64_t *n_send,
                                        double **recv_dev, int64_t *n_halo)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    if (send_dev) *send_dev = p->d_sendbuf;
    if (n_send) *n_send = int64_t(p->share.send_idx.size());
    if (recv_dev) *recv_dev = p->d_recvbuf;
    if (n_halo) *n_halo = int64_t(p->share.halo.size());
    return SPMV_OK;
}

extern "C" int spmv_op_launch(spmv_plan_t *p, int32_t op, const double *x, double *y,
                              void *stream_v)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    const Share &S = p->share;
    hipStream_t s = static_cast<hipStream_t>(stream_v);
    const int64_t n_rr = int64_t(S.R_rows.size());
    switch (op) {
        case SPMV_OP_PACK:
            if (!x && !S.send_idx.empty()) return set_error(SPMV_EINVAL, "x is NULL");
            SPMV_HIP(launch_pack(x, p->d_send_idx, p->d_sendbuf, int64_t(S.send_idx.size()), s));
            return SPMV_OK;
        case SPMV_OP_YL: {
            if (S.n_loc > 0 && (!x || !y)) return set_error(SPMV_EINVAL, "x or y is NULL");
            SPMV_HIP(launch_product(p, 0, x, y, nullptr, s));
            return SPMV_OK;
        }
        case SPMV_OP_UNPACK:
            if (!p->fuse_unpack)
                SPMV_HIP(launch_unpack(p->d_recvbuf, p->d_perm, p->d_xhalo,
                                       int64_t(S.halo.size()), s));
            return SPMV_OK;
        case SPMV_OP_YR: {
            if (n_rr > 0 && !y) return set_error(SPMV_EINVAL, "y is NULL");
            const double *xh = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
            SPMV_HIP(launch_product(p, 1, xh, nullptr, y, s));
            return SPMV_OK;
        }
        default: return set_error(SPMV_EINVAL, "not a GPU operation: " + std::to_string(op));
    }
}

extern "C" int spmv_plan_reorder(spmv_plan_t *p, const int32_t *op_order, int32_t n_ops,
                                 const int32_t *stream_map, int32_t n_streams)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    Schedule sch;
    if (int rc = validate_schedule(p->share.nranks, op_order, n_ops, stream_map, n_streams, sch))
        return rc;
    if (!p->host_only && sch.n_streams_used > p->n_st)
        return set_error(SPMV_EPLAN, "order uses " + std::to_string(sch.n_streams_used) +
                                         " streams, the plan owns " + std::to_string(p->n_st));
    p->sch = std::move(sch);
    p->fine = false;
    p->host_us.clear();
    p->host_n = 0.0;
    p->fused_combine = fuses_combine(p->sch);
    return SPMV_OK;
}

extern "C" int spmv_plan_set_fine(spmv_plan_t *p, const int32_t *op_order,
                                  const int32_t *op_stream, int32_t n_ops, int32_t n_streams)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->share.nranks < 2) return set_error(SPMV_EINVAL, "a single rank has no fine-grained DAG");
    FineSchedule f;
    std::vector<int32_t> def_ops, def_st;
    if (!op_order) {
        fine_default(p->fdag, def_ops, def_st);
        op_order = def_ops.data();
        op_stream = def_st.data();
        n_ops = int32_t(def_ops.size());
        n_streams = std::max<int32_t>(n_streams, 2);
    }
    if (int rc = validate_fine(p->fdag, op_order, op_stream, n_ops, n_streams, f)) return rc;
    if (!p->host_only && f.n_streams_used > p->n_st)
        return set_error(SPMV_EPLAN, "order uses " + std::to_string(f.n_streams_used) +
                                         " streams, the plan owns " + std::to_string(p->n_st));
    if (!p->host_only && p->ev_pack.empty()) {
        const size_t P = size_t(p->share.nranks);
        for (auto *v : {&p->ev_pack, &p->ev_psend, &p->ev_precv}) {
            v->assign(P, nullptr);
            for (auto &e : *v) SPMV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
    }
    // y_R adds into y itself when it follows y_L on the same stream
    int32_t pos_l = -1, pos_r = -1;
    for (size_t k = 0; k < f.order.size(); ++k) {
        if (f.order[k] == SPMV_OP_YL) pos_l = int32_t(k);
        if (f.order[k] == SPMV_OP_YR) pos_r = int32_t(k);
    }
    p->fsch = std::move(f);
    p->fine = true;
    p->host_us.clear();
    p->host_n = 0.0;
    p->fused_combine = pos_l < pos_r && p->fsch.ostream[size_t(pos_l)] == p->fsch.ostream[size_t(pos_r)];
    return SPMV_OK;
}

extern "C" int spmv_plan_time(spmv_plan_t *const *plans, int32_t n_plans, const double *const *x,
                              double *const *y, void *stream, double t_measure, int32_t n_measure,
                              double *times)
{
    if (!plans || n_plans < 1 || !x || !y || !times || n_measure < 1 || !(t_measure > 0))
        return set_error(SPMV_EINVAL, "bad argument to spmv_plan_time");
    using clock = std::chrono::steady_clock;
    for (int32_t j = 0; j < n_plans; ++j) {
        if (!plans[j]) return set_error(SPMV_EINVAL, "plan is NULL");
        if (plans[j]->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    }
    // the measurements start from an idle device (this also ends a state in
    // which the first send and receive copies of a process ran one after the
    // other, until the first device-wide synchronisation after them)
    SPMV_HIP(hipDeviceSynchronize());
    int64_t i = 0;
    for (int32_t m = 0; m < n_measure; ++m) {
        const auto t0 = clock::now();
        int64_t samples = 0;
        double el = 0.0;
        do {
            const int32_t j = int32_t(i++ % n_plans);
            if (int rc = spmv_exec(plans[j], x[j], y[j], stream)) return rc;
            ++samples;
            el = std::chrono::duration<double>(clock::now() - t0).count();
        } while (el < t_measure);
        times[m] = el / double(samples);
    }
    return SPMV_OK;
}

extern "C" int spmv_plan_info(const spmv_plan_t *p, spmv_info_t *info)
{
    if (!p || !info) return set_error(SPMV_EINVAL, "NULL argument");
    const Share &S = p->share;
    std::memset(info, 0, sizeof(*info));
    info->n_global = S.n_global;
    info->lo = S.lo;
    info->n_loc = S.n_loc;
    info->nnz_local = int64_t(S.L_col.size());
    info->nnz_remote = int64_t(S.R_col.size());
    info->n_halo = int64_t(S.halo.size());
    info->n_send = int64_t(S.send_idx.size());
    info->n_remote_rows = int64_t(S.R_rows.size());
    info->device_bytes = int64_t(p->arena_bytes);
    info->nranks = S.nranks;
    info->rank = S.rank;
    info->n_streams = p->n_st;
    info->n_ops = int32_t(p->fine ? p->fsch.order.size() : p->sch.order.size());
    info->fine = p->fine ? 1 : 0;
    info->kernel_local = p->cfg[0].kernel;
    info->kernel_remote = p->cfg[1].kernel;
    info->lanes_local = p->cfg[0].lanes;
    info->lanes_remote = p->cfg[1].lanes;
    info->rows_local = p->cfg[0].rows;
    info->rows_remote = p->cfg[1].rows;
    info->chunk_local = p->cfg[0].chunk;
    info->chunk_remote = p->cfg[1].chunk;
    info->width = p->cfg[0].kernel == SPMV_KERNEL_STREAM ? p->cfg[0].width : p->cfg[1].width;
    auto tiles = [](const CsrCfg &c) {
        if (c.kernel == SPMV_KERNEL_STREAM && c.form == 5)
            return int32_t(c.slab_tiles[kSlabs] - kSlabs);   // every slab's tiles
        return c.kernel == SPMV_KERNEL_STREAM && (c.form == 1 || c.form == 4)
                   ? int32_t(c.tile_row.size()) - 1
                   : 0;
    };
    auto slices = [](const CsrCfg &c) {
        return c.kernel == SPMV_KERNEL_STREAM && (c.form == 2 || c.form == 3)
                   ? int32_t(c.sell_ptr.size()) - 1
                   : 0;
    };
    info->n_tiles_local = tiles(p->cfg[0]);
    info->n_tiles_remote = tiles(p->cfg[1]);
    info->n_slices_local = slices(p->cfg[0]);
    info->n_slices_remote = slices(p->cfg[1]);
    info->form_local = p->cfg[0].kernel == SPMV_KERNEL_STREAM ? p->cfg[0].form : 0;
    info->form_remote = p->cfg[1].kernel == SPMV_KERNEL_STREAM ? p->cfg[1].form : 0;
    info->xcd_remap = p->xcd_remap;
    info->fuse_unpack = p->fuse_unpack;
    info->fused_combine = p->fused_combine;
    info->device = p->host_only ? -1 : p->device;
    info->resident_grouped = p->resident_seq ? 0
                             : p->res        ? 1
                             : p->rf.mask    ? 3
                             : (!p->host_only && !p->share.send_idx.empty() &&
                                int64_t(p->share.send_idx.size()) <= kPackTailMax && packs_with_yl(p)) ? 2
                                             : 0;
    return SPMV_OK;
}

extern "C" int spmv_plan_get_i32(const spmv_plan_t *p, int32_t which, int32_t *out, int64_t n)
{
    if (!p || (!out && n > 0)) return set_error(SPMV_EINVAL, "NULL argument");
    const Share &S = p->share;
    const std::vector<int32_t> *src = nullptr;
    std::vector<int32_t> tmp;
    switch (which) {
        case SPMV_I32_HALO_COLS: src = &S.halo; break;
        case SPMV_I32_RECV_OFF: src = &S.recv_off; break;
        case SPMV_I32_SEND_IDX: src = &S.send_idx; break;
        case SPMV_I32_SEND_OFF: src = &S.send_off; break;
        case SPMV_I32_AL_PTR: src = &S.L_ptr; break;
        case SPMV_I32_AL_COLS: src = &S.L_col; break;
        case SPMV_I32_AR_ROWS: src = &S.R_rows; break;
        case SPMV_I32_AR_PTR: src = &S.R_ptr; break;
        case SPMV_I32_AR_COLS: src = &S.R_col; break;
        case SPMV_I32_UNPACK_PERM: src = &S.unpack_perm; break;
        case SPMV_I32_OP_ORDER: src = p->fine ? &p->fsch.order : &p->sch.order; break;
        case SPMV_I32_OP_STREAM:
            if (p->fine) {
                src = &p->fsch.ostream;
            } else {
                for (int32_t t : p->sch.order)
                    tmp.push_back(is_vertex(t) && vertex_type(t) == VType::GPU ? p->sch.stream[t] : -1);
                src = &tmp;
            }
            break;
        case SPMV_I32_STREAM_MAP:
            tmp.assign(p->sch.stream, p->sch.stream + SPMV_N_VERTICES);
            src = &tmp;
            break;
        case SPMV_I32_TILE_ROW_L: src = &p->cfg[0].tile_row; break;
        case SPMV_I32_TILE_K_L: src = &p->cfg[0].tile_k; break;
        case SPMV_I32_TILE_ROW_R: src = &p->cfg[1].tile_row; break;
        case SPMV_I32_TILE_K_R: src = &p->cfg[1].tile_k; break;
        default: return set_error(SPMV_EINVAL, "unknown i32 selector");
    }
    if (n < int64_t(src->size()))
        return set_error(SPMV_EINVAL, "output too small: need " + std::to_string(src->size()));
    std::copy(src->begin(), src->end(), out);
    return SPMV_OK;
}

extern "C" int spmv_plan_get_f64(spmv_plan_t *p, int32_t which, double *out, int64_t n)
{
    if (!p || (!out && n > 0)) return set_error(SPMV_EINVAL, "NULL argument");
    const Share &S = p->share;
    const double *host = nullptr;
    const double *dev = nullptr;
    int64_t len = 0;
    switch (which) {
        case SPMV_F64_AL_VAL: host = S.L_val.data(); len = int64_t(S.L_val.size()); break;
        case SPMV_F64_AR_VAL: host = S.R_val.data(); len = int64_t(S.R_val.size()); break;
        case SPMV_F64_SENDBUF: dev = p->d_sendbuf; len = int64_t(S.send_idx.size()); break;
        case SPMV_F64_RECVBUF: dev = p->d_recvbuf; len = int64_t(S.halo.size()); break;
        case SPMV_F64_X_HALO:
            dev = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
            len = int64_t(S.halo.size());
            break;
        case SPMV_F64_OP_MS: host = p->ms; len = SPMV_N_VERTICES + 1; break;
        case SPMV_F64_OP_COUNT: host = p->cnt; len = SPMV_N_VERTICES + 1; break;
        case SPMV_F64_HOST_US: {
            const size_t n_ops = p->fine ? p->fsch.order.size() : p->sch.order.size();
            if (p->host_us.size() != n_ops) {
                p->host_us.assign(n_ops, 0.0);
                p->host_n = 0.0;
            }
            host = p->host_us.data();
            len = int64_t(n_ops);
            break;
        }
        case SPMV_F64_HOST_COUNT: host = &p->host_n; len = 1; break;
        default: return set_error(SPMV_EINVAL, "unknown f64 selector");
    }
    if (n < len) return set_error(SPMV_EINVAL, "output too small: need " + std::to_string(len));
    if (dev) {
        if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
        if (len) SPMV_HIP(hipMemcpy(out, dev, size_t(len) * 8, hipMemcpyDeviceToHost));
    } else if (len) {
        std::memcpy(out, host, size_t(len) * 8);
    }
    return SPMV_OK;
}

extern "C" int spmv_plan_set_profile(spmv_plan_t *p, int32_t on)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    if (on < 0 || on > 3) return set_error(SPMV_EINVAL, "profile mode must be 0 to 3");
    if ((on & 1) && !p->ev_b[0]) {
        int dev = 0;
        SPMV_HIP(hipGetDevice(&dev));
        if (dev != p->device) SPMV_HIP(hipSetDevice(p->device));
        for (int i = 0; i <= SPMV_N_VERTICES; ++i) {
            SPMV_HIP(hipEventCreate(&p->ev_b[i]));
            SPMV_HIP(hipEventCreate(&p->ev_e[i]));
        }
        if (dev != p->device) SPMV_HIP(hipSetDevice(dev));
    }
    p->profile = (on & 1) != 0;
    p->host_times = (on & 2) != 0;
    return SPMV_OK;
}

extern "C" int spmv_plan_reset_times(spmv_plan_t *p)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    std::fill(p->ms, p->ms + SPMV_N_VERTICES + 1, 0.0);
    std::fill(p->cnt, p->cnt + SPMV_N_VERTICES + 1, 0.0);
    std::fill(p->host_us.begin(), p->host_us.end(), 0.0);
    p->host_n = 0.0;
    return SPMV_OK;
}

extern "C" int spmv_plan_inbox(spmv_plan_t *p, double **host_ptr, int64_t *n)
{
    if (!p || !host_ptr || !n) return set_error(SPMV_EINVAL, "NULL argument");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    *host_ptr = p->h_inbox;
    *n = int64_t(p->share.halo.size());
    return SPMV_OK;
}

extern "C" int spmv_plan_outbox(spmv_plan_t *p, double **host_ptr, int64_t *n)
{
    if (!p || !host_ptr || !n) return set_error(SPMV_EINVAL, "NULL argument");
    if (p->host_only) return set_error(SPMV_ESTATE, "plan was created host-only");
    *host_ptr = p->h_outbox;
    *n = int64_t(p->share.send_idx.size());
    return SPMV_OK;
}
