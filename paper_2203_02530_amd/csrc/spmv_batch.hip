// Batches: the SpMVs of many rank shares in three grouped persistent
// kernels inside one hipGraph.
//
// Work items are the stream-CSR tiles of every share's y_L and y_R and the
// gather ranges of every share's Pack and Unpack.  Each grouped kernel runs a
// fixed grid (256 CUs x blocks_per_cu); every block walks its own list of
// items, assigned on the host longest-first to the least-loaded block, and,
// with XCD affinity, only to blocks of the XCD that owns the share (share s
// -> XCD s mod 8) so the share's x stays in that XCD's L2.  The host-blocking
// synchronisations of the single-share program become graph edges.
#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>

#include "spmv_internal.h"
#include "spmv_stream.h"

namespace spmv {
namespace {

enum ItemKind : int32_t { kPack = 0, kLocal = 1, kUnpack = 2, kRemote = 3 };

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
};

struct Item {
    int32_t kind, share, a, n;   // tile a, or gather range [a, a + n)
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
        const ShareDev &S = sh[it.share];
        if (it.kind == kPack || it.kind == kUnpack) {
            const double *src = it.kind == kPack ? xs[it.share] : S.recvbuf;
            const int32_t *idx = it.kind == kPack ? S.send_idx : S.perm;
            double *dst = it.kind == kPack ? S.sendbuf : S.xhalo;
            for (int k = it.a + int(threadIdx.x); k < it.a + it.n; k += kBlock) dst[k] = src[idx[k]];
        } else if (it.kind == kLocal) {
            StreamArgs A;
            A.tile_row = S.L_tile_row;
            A.tile_k = S.L_tile_k;
            A.rp = S.L_rp;
            A.col = S.L_col;
            A.rows = nullptr;
            A.val = S.L_val;
            A.x = xs[it.share];
            A.out = ys[it.share];
            A.acc = nullptr;
            A.nnz_alloc = S.L_nnz_alloc;
            A.n_x = S.n_loc;
            if (S.L_col16)
                tile_sl<NPT, VW, true>(S.L_lanes, A, it.a, s_p, s_rp);
            else
                tile_sl<NPT, VW, false>(S.L_lanes, A, it.a, s_p, s_rp);
        } else {
            StreamArgs A;
            A.tile_row = S.R_tile_row;
            A.tile_k = S.R_tile_k;
            A.rp = S.R_rp;
            A.col = S.R_col;
            A.rows = S.R_rows;
            A.val = S.R_val;
            A.x = S.fuse_unpack ? S.recvbuf : S.xhalo;
            A.out = nullptr;
            A.acc = ys[it.share];
            A.nnz_alloc = S.R_nnz_alloc;
            A.n_x = S.n_halo;
            tile_sl<NPT, VW>(S.R_lanes, A, it.a, s_p, s_rp);
        }
        __syncthreads();
    }
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

GroupedFn grouped_fn(int npt, int vw)
{
    if (vw == 2) {
        if (npt == 4) return k_grouped<4, 2>;
        if (npt == 8) return k_grouped<8, 2>;
        if (npt == 16) return k_grouped<16, 2>;
    } else if (vw == 4) {
        if (npt == 4) return k_grouped<4, 4>;
        if (npt == 8) return k_grouped<8, 4>;
        if (npt == 16) return k_grouped<16, 4>;
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

    void *arena = nullptr;
    size_t arena_bytes = 0;
    ShareDev *d_sh = nullptr;
    const double **d_x = nullptr;   // [n], then d_y right after (one table)
    double **d_y = nullptr;
    Item *d_items[3] = {};
    int32_t *d_blk[3] = {};
    int64_t n_items[3] = {};
    void **h_xy = nullptr;          // pinned [2n]: x pointers then y pointers

    int32_t n_cs = 1;                                   // copy streams per direction
    hipStream_t cs_send_k[kCopyStreams] = {}, cs_recv_k[kCopyStreams] = {};
    hipEvent_t ev_a = nullptr, ev_s = nullptr, ev_r = nullptr, ev_f = nullptr;
    hipEvent_t ev_sk[kCopyStreams] = {}, ev_rk[kCopyStreams] = {};
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
    for (hipEvent_t e : {b->ev_a, b->ev_s, b->ev_r, b->ev_f})
        if (e) (void)hipEventDestroy(e);
    for (int k = 0; k < kCopyStreams; ++k) {
        if (b->ev_sk[k]) (void)hipEventDestroy(b->ev_sk[k]);
        if (b->ev_rk[k]) (void)hipEventDestroy(b->ev_rk[k]);
    }
    if (b->arena) (void)hipFree(b->arena);
    if (b->h_xy) (void)hipHostFree(b->h_xy);
    if (b->pool_held) pool_release(b->device);
    delete b;
}

// Longest-first assignment of items to blocks; with affinity, an item of
// share s only goes to blocks b with b % 8 == s % 8.  Returns items grouped
// by block and the per-block offsets.
void assign(const std::vector<Item> &items, const std::vector<int64_t> &cost, int n_blocks,
            bool aff, std::vector<Item> &out, std::vector<int32_t> &blk_ptr)
{
    std::vector<size_t> order(items.size());
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    using Slot = std::pair<int64_t, int32_t>;   // (load, block)
    const int groups = aff ? kXcds : 1;
    std::vector<std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>>> heaps(
        static_cast<size_t>(groups));
    for (int32_t b = 0; b < n_blocks; ++b) heaps[size_t(aff ? b % kXcds : 0)].push({0, b});
    std::vector<int32_t> owner(items.size());
    for (size_t i : order) {
        auto &h = heaps[size_t(aff ? items[i].share % kXcds : 0)];
        Slot s = h.top();
        h.pop();
        owner[i] = s.second;
        s.first += cost[i];
        h.push(s);
    }
    blk_ptr.assign(size_t(n_blocks) + 1, 0);
    for (size_t i = 0; i < items.size(); ++i) ++blk_ptr[size_t(owner[i]) + 1];
    for (int32_t b = 0; b < n_blocks; ++b) blk_ptr[size_t(b) + 1] += blk_ptr[size_t(b)];
    out.resize(items.size());
    std::vector<int32_t> fill(blk_ptr.begin(), blk_ptr.end() - 1);
    for (size_t i = 0; i < items.size(); ++i) out[size_t(fill[size_t(owner[i])]++)] = items[i];
}

int64_t tile_cost(const std::vector<int32_t> &tk, size_t t) { return int64_t(tk[t + 1] - tk[t]) + 64; }

// One batch on stream s: the pointer table, the receive copies (forked
// onto the copy streams right away: they need nothing from this batch),
// Pack + y_L, the send copies behind it, Unpack once every receive copy is
// in, y_R, and the join of the send copies (stream launches).
int issue(spmv_batch *b, hipStream_t s)
{
    auto launch = [&](int ph) -> hipError_t {
        if (b->n_items[ph] == 0) return hipSuccess;
        hipLaunchKernelGGL(b->fn, dim3(unsigned(b->n_blocks)), dim3(kBlock), 0, s, b->d_sh,
                           b->d_x, b->d_y, b->d_items[ph], b->d_blk[ph]);
        return hipGetLastError();
    };
    SPMV_HIP(hipMemcpyAsync(b->d_x, b->h_xy, size_t(2 * b->n) * sizeof(void *),
                            hipMemcpyHostToDevice, s));
    SPMV_HIP(hipEventRecord(b->ev_f, s));
    for (int32_t k = 0; k < b->n_cs; ++k) SPMV_HIP(hipStreamWaitEvent(b->cs_recv_k[k], b->ev_f, 0));
    // receive copies need nothing from this batch: issue them first, on
    // n_cs streams, then Pack + y_L, then the send copies behind it
    const int32_t K = b->n_cs;
    if (b->staging) {
        for (int32_t i = 0; i < b->n; ++i) {
            const spmv_plan *p = b->plans[size_t(i)];
            const size_t nh = p->share.halo.size() * 8;
            if (nh)
                SPMV_HIP(hipMemcpyAsync(p->d_recvbuf, p->h_inbox, nh, hipMemcpyHostToDevice,
                                        b->cs_recv_k[i % K]));
        }
    }
    SPMV_HIP(launch(0));
    SPMV_HIP(hipEventRecord(b->ev_a, s));
    for (int32_t k = 0; k < K; ++k) SPMV_HIP(hipStreamWaitEvent(b->cs_send_k[k], b->ev_a, 0));
    if (b->staging) {
        for (int32_t i = 0; i < b->n; ++i) {
            const spmv_plan *p = b->plans[size_t(i)];
            const size_t ns = p->share.send_idx.size() * 8;
            if (ns)
                SPMV_HIP(hipMemcpyAsync(p->h_outbox, p->d_sendbuf, ns, hipMemcpyDeviceToHost,
                                        b->cs_send_k[i % K]));
        }
    }
    for (int32_t k = 0; k < K; ++k) {
        SPMV_HIP(hipEventRecord(b->ev_sk[k], b->cs_send_k[k]));
        SPMV_HIP(hipEventRecord(b->ev_rk[k], b->cs_recv_k[k]));
        SPMV_HIP(hipStreamWaitEvent(s, b->ev_rk[k], 0));
    }
    SPMV_HIP(launch(1));
    SPMV_HIP(launch(2));
    for (int32_t k = 0; k < K; ++k) SPMV_HIP(hipStreamWaitEvent(s, b->ev_sk[k], 0));
    return SPMV_OK;
}

int build_graph(spmv_batch *b)
{
    SPMV_HIP(hipGraphCreate(&b->graph, 0));
    hipGraphNode_t n_t;
    SPMV_HIP(hipGraphAddMemcpyNode1D(&n_t, b->graph, nullptr, 0, b->d_x, b->h_xy,
                                     size_t(2 * b->n) * sizeof(void *), hipMemcpyHostToDevice));
    auto kernel_node = [&](int phase, const hipGraphNode_t *deps, size_t nd,
                           hipGraphNode_t *node) -> int {
        hipKernelNodeParams kp{};
        void *args[] = {&b->d_sh, &b->d_x, &b->d_y, &b->d_items[phase], &b->d_blk[phase]};
        kp.func = reinterpret_cast<void *>(b->fn);
        kp.gridDim = dim3(unsigned(b->n_blocks));
        kp.blockDim = dim3(kBlock);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        SPMV_HIP(hipGraphAddKernelNode(node, b->graph, deps, nd, &kp));
        return SPMV_OK;
    };
    hipGraphNode_t n_a = nullptr, n_b = nullptr, n_c = nullptr;
    if (int rc = kernel_node(0, &n_t, 1, &n_a)) return rc;
    // the copies of each direction form one chain: concurrent copies of one
    // direction share the host link and measured slower (64 power-law
    // shares: 31.7 ms per batch with one copy stream per direction, 40.9
    // with two, 49.4 with four)
    std::vector<hipGraphNode_t> recv;
    hipGraphNode_t prev_send = n_a, prev_recv = nullptr;
    for (spmv_plan *p : b->staging ? b->plans : std::vector<spmv_plan *>{}) {
        const size_t ns = p->share.send_idx.size() * 8, nh = p->share.halo.size() * 8;
        if (ns) {
            hipGraphNode_t n;
            SPMV_HIP(hipGraphAddMemcpyNode1D(&n, b->graph, &prev_send, 1, p->h_outbox,
                                             p->d_sendbuf, ns, hipMemcpyDeviceToHost));
            prev_send = n;
        }
        if (nh) {
            hipGraphNode_t n;
            SPMV_HIP(hipGraphAddMemcpyNode1D(&n, b->graph, prev_recv ? &prev_recv : nullptr,
                                             prev_recv ? 1 : 0, p->d_recvbuf, p->h_inbox, nh,
                                             hipMemcpyHostToDevice));
            prev_recv = n;
        }
    }
    if (prev_recv) recv.push_back(prev_recv);
    std::vector<hipGraphNode_t> deps_c{n_a};
    if (b->n_items[1] > 0) {
        if (int rc = kernel_node(1, recv.data(), recv.size(), &n_b)) return rc;
        deps_c.push_back(n_b);
    } else {
        deps_c.insert(deps_c.end(), recv.begin(), recv.end());
    }
    if (b->n_items[2] > 0)
        if (int rc = kernel_node(2, deps_c.data(), deps_c.size(), &n_c)) return rc;
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
        o.xcd_affinity < 0 || o.xcd_affinity > 2 || o.staging < 0 || o.staging > 1 ||
        o.copy_streams < 0 || o.copy_streams > kCopyStreams)
        return set_error(SPMV_EINVAL, "batch option out of range");
    const int npt = plans[0] ? plans[0]->cfg[0].chunk : 0;
    const int vw = plans[0] ? plans[0]->cfg[0].width : 0;
    for (int32_t i = 0; i < n; ++i) {
        const spmv_plan *p = plans[i];
        if (!p) return set_error(SPMV_EINVAL, "plan " + std::to_string(i) + " is NULL");
        if (p->host_only || p->device != plans[0]->device)
            return set_error(SPMV_EINVAL, "plan " + std::to_string(i) +
                                              " is host-only or on another device");
        for (int side = 0; side < 2; ++side)
            if (p->cfg[side].kernel != SPMV_KERNEL_STREAM || p->cfg[side].chunk != npt ||
                p->cfg[side].width != vw ||
                !(p->cfg[side].form == 1 || (side == 0 && p->cfg[side].form == 4)))
                return set_error(SPMV_EINVAL, "plan " + std::to_string(i) +
                                                  ": batched shares need packed-tile stream-CSR "
                                                  "products with one common chunk and width");
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
    b->fn = grouped_fn(npt, vw);
    b->n_blocks = kCUs * (o.blocks_per_cu ? o.blocks_per_cu : 8);
    // automatic: stream launches when the halo is staged (the graph runs its
    // copy nodes one after another: 46 ms per batch of 64 power-law shares
    // against 31-37 ms with one copy stream per direction), the graph when
    // only the grouped kernels run
    b->use_graph = o.use_graph == 1 || (o.use_graph == 0 && o.staging == 1);
    b->xcd_aff = o.xcd_affinity == 1 || (o.xcd_affinity == 0 && n >= kXcds);
    b->staging = o.staging == 0;
    b->n_cs = o.copy_streams ? o.copy_streams : 1;

    // descriptors and work items
    std::vector<ShareDev> sh(static_cast<size_t>(n));
    std::vector<Item> items[3];
    std::vector<int64_t> cost[3];
    const int gather_len = kBlock * npt;
    for (int32_t i = 0; i < n; ++i) {
        spmv_plan *p = plans[i];
        const Share &S = p->share;
        ShareDev &d = sh[size_t(i)];
        d.L_tile_row = p->d_tile_row[0];
        d.L_tile_k = p->d_tile_k[0];
        d.L_rp = p->dL_ptr;
        d.L_col = p->dL_col;
        d.L_val = p->dL_val;
        d.R_tile_row = p->d_tile_row[1];
        d.R_tile_k = p->d_tile_k[1];
        d.R_rp = p->dR_ptr;
        d.R_col = p->dR_col;
        d.R_rows = p->dR_rows;
        d.R_val = p->dR_val;
        d.send_idx = p->d_send_idx;
        d.perm = p->d_perm;
        d.sendbuf = p->d_sendbuf;
        d.recvbuf = p->d_recvbuf;
        d.xhalo = p->d_xhalo;
        d.L_nnz_alloc = uint32_t(S.L_col.size() + kEntryPad);
        d.R_nnz_alloc = uint32_t(S.R_col.size() + kEntryPad);
        d.n_loc = uint32_t(S.n_loc);
        d.n_halo = uint32_t(S.halo.size());
        d.L_lanes = p->cfg[0].lanes;
        d.R_lanes = p->cfg[1].lanes;
        d.fuse_unpack = p->fuse_unpack ? 1 : 0;
        d.L_col16 = p->cfg[0].form == 4 ? 1 : 0;
        const int64_t n_send = int64_t(S.send_idx.size()), n_halo = int64_t(S.halo.size());
        for (int64_t a = 0; a < n_send; a += gather_len) {
            const int32_t len = int32_t(std::min<int64_t>(gather_len, n_send - a));
            items[0].push_back({kPack, i, int32_t(a), len});
            cost[0].push_back(len / 2 + 64);
        }
        const auto &tl = p->cfg[0].tile_k;
        for (size_t t = 0; t + 1 < tl.size(); ++t) {
            items[0].push_back({kLocal, i, int32_t(t), 0});
            cost[0].push_back(tile_cost(tl, t));
        }
        if (!p->fuse_unpack)
            for (int64_t a = 0; a < n_halo; a += gather_len) {
                const int32_t len = int32_t(std::min<int64_t>(gather_len, n_halo - a));
                items[1].push_back({kUnpack, i, int32_t(a), len});
                cost[1].push_back(len / 2 + 64);
            }
        const auto &tr = p->cfg[1].tile_k;
        for (size_t t = 0; t + 1 < tr.size(); ++t) {
            items[2].push_back({kRemote, i, int32_t(t), 0});
            cost[2].push_back(tile_cost(tr, t));
        }
        // algorithmic bytes, as for one exec of the share
        const int64_t nl = int64_t(S.L_col.size()), nr = int64_t(S.R_col.size());
        const int64_t rr = int64_t(S.R_rows.size()), nloc = S.n_loc;
        b->dev_bytes += 20 * n_send + 12 * nl + 4 * (nloc + 1) + 16 * nloc +
                        (p->fuse_unpack ? 0 : 20 * n_halo) + 12 * nr + 8 * rr + 4 + 8 * n_halo +
                        16 * rr;
        if (o.staging == 0) b->link_bytes += 8 * (n_send + n_halo);
    }
    std::vector<Item> grouped[3];
    std::vector<int32_t> blk[3];
    for (int ph = 0; ph < 3; ++ph) {
        assign(items[ph], cost[ph], b->n_blocks, b->xcd_aff, grouped[ph], blk[ph]);
        b->n_items[ph] = int64_t(items[ph].size());
    }

    // one device arena: descriptors, pointer tables, items, block offsets
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off_sh = 0;
    size_t off_xy = off_sh + al(sh.size() * sizeof(ShareDev));
    size_t cur = off_xy + al(size_t(2 * n) * sizeof(void *));
    size_t off_items[3], off_blk[3];
    for (int ph = 0; ph < 3; ++ph) {
        off_items[ph] = cur;
        cur += al(std::max<size_t>(grouped[ph].size(), 1) * sizeof(Item));
        off_blk[ph] = cur;
        cur += al(blk[ph].size() * sizeof(int32_t));
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
    for (int ph = 0; ph < 3; ++ph) {
        b->d_items[ph] = reinterpret_cast<Item *>(base + off_items[ph]);
        b->d_blk[ph] = reinterpret_cast<int32_t *>(base + off_blk[ph]);
        if (!grouped[ph].empty()) {
            e = hipMemcpy(b->d_items[ph], grouped[ph].data(), grouped[ph].size() * sizeof(Item),
                          hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(hip_error(e, "hipMemcpy(batch items)"));
        }
        e = hipMemcpy(b->d_blk[ph], blk[ph].data(), blk[ph].size() * sizeof(int32_t),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(hip_error(e, "hipMemcpy(batch offsets)"));
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
    for (hipEvent_t *ev : {&b->ev_a, &b->ev_s, &b->ev_r, &b->ev_f}) {
        e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) return fail(hip_error(e, "hipEventCreate(batch)"));
    }
    for (int k = 0; k < b->n_cs; ++k) {
        for (hipEvent_t *ev : {&b->ev_sk[k], &b->ev_rk[k]}) {
            e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
            if (e != hipSuccess) return fail(hip_error(e, "hipEventCreate(batch)"));
        }
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
    return SPMV_OK;
}

extern "C" int spmv_batch_destroy(spmv_batch_t *b)
{
    if (!b) return SPMV_OK;
    (void)hipDeviceSynchronize();
    batch_release(b);
    return SPMV_OK;
}
