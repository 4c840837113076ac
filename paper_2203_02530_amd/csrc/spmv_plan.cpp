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
#include <cstring>

#include "spmv_internal.h"

struct spmv_plan {
    spmv::Share share;
    spmv::Schedule sch;
    int32_t lanes_local = 1, lanes_remote = 1, rows_local = 1, rows_remote = 1, xcd_remap = 1;
    bool fuse_unpack = false, fused_combine = false, host_only = false, profile = false;
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

    // pinned host mailboxes
    double *h_inbox = nullptr, *h_outbox = nullptr;

    // streams and events
    hipStream_t st[SPMV_MAX_STREAMS] = {};
    int32_t n_st = 0;
    hipStream_t cs_send = nullptr, cs_recv = nullptr;
    hipEvent_t ev_start = nullptr, ev_send = nullptr, ev_recv = nullptr;
    hipEvent_t ev_rec[SPMV_N_VERTICES] = {};
    hipEvent_t ev_join[SPMV_MAX_STREAMS] = {};
    // profiling: begin/end per vertex, index SPMV_N_VERTICES = combine
    hipEvent_t ev_b[SPMV_N_VERTICES + 1] = {}, ev_e[SPMV_N_VERTICES + 1] = {};
    double ms[SPMV_N_VERTICES + 1] = {};
    double cnt[SPMV_N_VERTICES + 1] = {};
};

namespace spmv {
namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

void release(spmv_plan *p)
{
    if (!p) return;
    for (int32_t i = 0; i < p->n_st; ++i)
        if (p->st[i]) (void)hipStreamDestroy(p->st[i]);
    if (p->cs_send) (void)hipStreamDestroy(p->cs_send);
    if (p->cs_recv) (void)hipStreamDestroy(p->cs_recv);
    hipEvent_t *evs[] = {&p->ev_start, &p->ev_send, &p->ev_recv};
    for (hipEvent_t *e : evs)
        if (*e) (void)hipEventDestroy(*e);
    for (auto &e : p->ev_rec)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : p->ev_join)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i <= SPMV_N_VERTICES; ++i) {
        if (p->ev_b[i]) (void)hipEventDestroy(p->ev_b[i]);
        if (p->ev_e[i]) (void)hipEventDestroy(p->ev_e[i]);
    }
    if (p->arena) (void)hipFree(p->arena);
    if (p->h_inbox) (void)hipHostFree(p->h_inbox);
    if (p->h_outbox) (void)hipHostFree(p->h_outbox);
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
    };
    const size_t n_halo = S.halo.size(), n_send = S.send_idx.size(), n_rr = S.R_rows.size();
    Item items[] = {
        {(void **)&p->dL_ptr, S.L_ptr.size() * 4, S.L_ptr.data()},
        {(void **)&p->dL_col, S.L_col.size() * 4, S.L_col.data()},
        {(void **)&p->dR_rows, S.R_rows.size() * 4, S.R_rows.data()},
        {(void **)&p->dR_ptr, S.R_ptr.size() * 4, S.R_ptr.data()},
        {(void **)&p->dR_col, S.R_col.size() * 4, S.R_col.data()},
        {(void **)&p->d_send_idx, n_send * 4, S.send_idx.data()},
        {(void **)&p->d_perm, n_halo * 4, S.unpack_perm.data()},
        {(void **)&p->dL_val, S.L_val.size() * 8, S.L_val.data()},
        {(void **)&p->dR_val, S.R_val.size() * 8, S.R_val.data()},
        {(void **)&p->d_sendbuf, n_send * 8, nullptr},
        {(void **)&p->d_recvbuf, n_halo * 8, nullptr},
        {(void **)&p->d_xhalo, n_halo * 8, nullptr},
        {(void **)&p->d_part, n_rr * 8, nullptr},
    };
    size_t total = 0;
    for (const Item &it : items) total += align_up(std::max<size_t>(it.bytes, 1));
    SPMV_HIP(hipMalloc(&p->arena, total));
    p->arena_bytes = total;
    char *cur = static_cast<char *>(p->arena);
    for (const Item &it : items) {
        *it.dst = cur;
        if (it.src && it.bytes) SPMV_HIP(hipMemcpy(cur, it.src, it.bytes, hipMemcpyHostToDevice));
        cur += align_up(std::max<size_t>(it.bytes, 1));
    }
    SPMV_HIP(hipMemset(p->d_sendbuf, 0, std::max<size_t>(n_send * 8, 1)));
    SPMV_HIP(hipMemset(p->d_recvbuf, 0, std::max<size_t>(n_halo * 8, 1)));
    SPMV_HIP(hipMemset(p->d_xhalo, 0, std::max<size_t>(n_halo * 8, 1)));
    SPMV_HIP(hipHostMalloc((void **)&p->h_inbox, std::max<size_t>(n_halo * 8, 8),
                           hipHostMallocDefault));
    SPMV_HIP(hipHostMalloc((void **)&p->h_outbox, std::max<size_t>(n_send * 8, 8),
                           hipHostMallocDefault));
    std::memset(p->h_inbox, 0, std::max<size_t>(n_halo * 8, 8));
    std::memset(p->h_outbox, 0, std::max<size_t>(n_send * 8, 8));

    p->n_st = std::max<int32_t>(p->sch.n_streams_used, 1);
    for (int32_t i = 0; i < p->n_st; ++i)
        SPMV_HIP(hipStreamCreateWithFlags(&p->st[i], hipStreamNonBlocking));
    SPMV_HIP(hipStreamCreateWithFlags(&p->cs_send, hipStreamNonBlocking));
    SPMV_HIP(hipStreamCreateWithFlags(&p->cs_recv, hipStreamNonBlocking));
    SPMV_HIP(hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming));
    SPMV_HIP(hipEventCreateWithFlags(&p->ev_send, hipEventDisableTiming));
    SPMV_HIP(hipEventCreateWithFlags(&p->ev_recv, hipEventDisableTiming));
    for (auto &e : p->ev_rec) SPMV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int32_t i = 0; i < p->n_st; ++i)
        SPMV_HIP(hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming));
    if (p->profile)
        for (int i = 0; i <= SPMV_N_VERTICES; ++i) {
            SPMV_HIP(hipEventCreate(&p->ev_b[i]));
            SPMV_HIP(hipEventCreate(&p->ev_e[i]));
        }
    SPMV_HIP(hipDeviceSynchronize());
    return SPMV_OK;
}

}  // namespace
}  // namespace spmv

using namespace spmv;

extern "C" int spmv_plan_create_ex(const spmv_csr_t *csr, int32_t nranks, int32_t rank,
                                   const int32_t *op_order, int32_t n_ops,
                                   const int32_t *stream_map, int32_t n_streams,
                                   const spmv_tune_t *tune, spmv_plan_t **out)
{
    if (!out) return set_error(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    spmv_tune_t t{};
    if (tune) t = *tune;
    auto valid_lanes = [](int32_t l) { return l == 0 || (l >= 1 && l <= 64 && !(l & (l - 1))); };
    auto valid_rows = [](int32_t r) { return r == 0 || r == 1 || r == 2 || r == 4 || r == 8; };
    if (!valid_lanes(t.lanes_local) || !valid_lanes(t.lanes_remote))
        return set_error(SPMV_EINVAL, "lanes per row must be 0 or a power of two <= 64");
    if (!valid_rows(t.rows_local) || !valid_rows(t.rows_remote))
        return set_error(SPMV_EINVAL, "rows per lane group must be 0, 1, 2, 4 or 8");
    if (t.xcd_remap < 0 || t.xcd_remap > 2 || t.fuse_unpack < 0 || t.fuse_unpack > 1)
        return set_error(SPMV_EINVAL, "tune field out of range");

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
    if (rc == SPMV_OK) rc = build_share(csr, nranks, rank, p->share);
    if (rc != SPMV_OK) {
        delete p;
        return rc;
    }
    const Share &S = p->share;
    p->lanes_local = t.lanes_local ? t.lanes_local
                                   : auto_lanes(int64_t(S.L_col.size()), S.n_loc);
    p->lanes_remote = t.lanes_remote ? t.lanes_remote
                                     : auto_lanes(int64_t(S.R_col.size()),
                                                  int64_t(S.R_rows.size()));
    p->rows_local = t.rows_local ? t.rows_local : auto_rows(p->lanes_local, S.n_loc);
    p->rows_remote = t.rows_remote ? t.rows_remote
                                   : auto_rows(p->lanes_remote, int64_t(S.R_rows.size()));
    p->xcd_remap = t.xcd_remap ? t.xcd_remap : 1;
    p->fuse_unpack = t.fuse_unpack == 1;
    p->host_only = (t.flags & SPMV_F_HOST_ONLY) != 0;
    p->profile = (t.flags & SPMV_F_PROFILE) != 0;
    // y_R adds into y itself when it runs after y_L on the same stream;
    // otherwise its partial sums are added by a combine step at end.
    if (p->sch.multi) {
        auto pos = [&](int32_t tok) {
            return std::find(p->sch.order.begin(), p->sch.order.end(), tok) - p->sch.order.begin();
        };
        p->fused_combine = p->sch.stream[SPMV_OP_YL] == p->sch.stream[SPMV_OP_YR] &&
                           pos(SPMV_OP_YL) < pos(SPMV_OP_YR);
    }
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

    const int32_t *smap = p->sch.stream;
    const int64_t n_send = int64_t(S.send_idx.size()), n_halo = int64_t(S.halo.size());
    const int64_t n_rr = int64_t(S.R_rows.size());
    bool ran[SPMV_N_VERTICES + 1] = {};
    bool combine = false;

    for (int32_t tok : p->sch.order) {
        if (is_sync(tok)) {
            const int32_t kind = sync_kind(tok), v = sync_operand(tok);
            if (kind == SPMV_SYNC_CER) {
                SPMV_HIP(hipEventRecord(p->ev_rec[v], p->st[smap[v]]));
            } else {
                // the wait acts on the records of v's GPU predecessors
                const int32_t u = v == SPMV_OP_POST_SEND ? SPMV_OP_PACK
                                  : v == SPMV_OP_YR     ? SPMV_OP_UNPACK
                                                        : -1;
                if (u < 0) return set_error(SPMV_EPLAN, "synchronisation without a GPU predecessor");
                if (kind == SPMV_SYNC_CES)
                    SPMV_HIP(hipEventSynchronize(p->ev_rec[u]));
                else
                    SPMV_HIP(hipStreamWaitEvent(p->st[smap[v]], p->ev_rec[u], 0));
            }
            continue;
        }
        switch (tok) {
            case SPMV_OP_START:
                SPMV_HIP(hipEventRecord(p->ev_start, caller));
                for (int32_t i = 0; i < p->n_st; ++i)
                    SPMV_HIP(hipStreamWaitEvent(p->st[i], p->ev_start, 0));
                break;
            case SPMV_OP_PACK: {
                hipStream_t s = p->st[smap[tok]];
                SPMV_HIP(prof_begin(p, tok, s));
                SPMV_HIP(launch_pack(x, p->d_send_idx, p->d_sendbuf, n_send, s));
                SPMV_HIP(prof_end(p, tok, s));
                ran[tok] = true;
                break;
            }
            case SPMV_OP_YL: {
                hipStream_t s = p->st[smap[tok]];
                CsrDev A;
                A.n_rows = int32_t(S.n_loc);
                A.rp = p->dL_ptr;
                A.col = p->dL_col;
                A.val = p->dL_val;
                SPMV_HIP(prof_begin(p, tok, s));
                SPMV_HIP(launch_csr(A, x, y, nullptr, p->lanes_local, p->rows_local, p->xcd_remap, s));
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
                hipStream_t s = p->st[smap[tok]];
                SPMV_HIP(prof_begin(p, tok, s));
                SPMV_HIP(launch_unpack(p->d_recvbuf, p->d_perm, p->d_xhalo, n_halo, s));
                SPMV_HIP(prof_end(p, tok, s));
                ran[tok] = true;
                break;
            }
            case SPMV_OP_YR: {
                hipStream_t s = p->st[smap[tok]];
                CsrDev A;
                A.n_rows = int32_t(n_rr);
                A.rp = p->dR_ptr;
                A.col = p->dR_col;
                A.val = p->dR_val;
                A.rows = p->dR_rows;
                const double *xh = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
                SPMV_HIP(prof_begin(p, tok, s));
                if (p->fused_combine)
                    SPMV_HIP(launch_csr(A, xh, nullptr, y, p->lanes_remote, p->rows_remote,
                                        p->xcd_remap, s));
                else
                    SPMV_HIP(launch_csr(A, xh, p->d_part, nullptr, p->lanes_remote, p->rows_remote,
                                        p->xcd_remap, s));
                SPMV_HIP(prof_end(p, tok, s));
                combine = !p->fused_combine && n_rr > 0;
                ran[tok] = true;
                break;
            }
            case SPMV_OP_END:
                for (int32_t i = 0; i < p->n_st; ++i) {
                    SPMV_HIP(hipEventRecord(p->ev_join[i], p->st[i]));
                    SPMV_HIP(hipStreamWaitEvent(caller, p->ev_join[i], 0));
                }
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
    }
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
            CsrDev A;
            A.n_rows = int32_t(S.n_loc);
            A.rp = p->dL_ptr;
            A.col = p->dL_col;
            A.val = p->dL_val;
            SPMV_HIP(launch_csr(A, x, y, nullptr, p->lanes_local, p->rows_local, p->xcd_remap, s));
            return SPMV_OK;
        }
        case SPMV_OP_UNPACK:
            if (!p->fuse_unpack)
                SPMV_HIP(launch_unpack(p->d_recvbuf, p->d_perm, p->d_xhalo,
                                       int64_t(S.halo.size()), s));
            return SPMV_OK;
        case SPMV_OP_YR: {
            if (n_rr > 0 && !y) return set_error(SPMV_EINVAL, "y is NULL");
            CsrDev A;
            A.n_rows = int32_t(n_rr);
            A.rp = p->dR_ptr;
            A.col = p->dR_col;
            A.val = p->dR_val;
            A.rows = p->dR_rows;
            const double *xh = p->fuse_unpack ? p->d_recvbuf : p->d_xhalo;
            SPMV_HIP(launch_csr(A, xh, nullptr, y, p->lanes_remote, p->rows_remote, p->xcd_remap, s));
            return SPMV_OK;
        }
        default: return set_error(SPMV_EINVAL, "not a GPU operation: " + std::to_string(op));
    }
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
    info->n_ops = int32_t(p->sch.order.size());
    info->lanes_local = p->lanes_local;
    info->lanes_remote = p->lanes_remote;
    info->rows_local = p->rows_local;
    info->rows_remote = p->rows_remote;
    info->xcd_remap = p->xcd_remap;
    info->fuse_unpack = p->fuse_unpack;
    info->fused_combine = p->fused_combine;
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
        case SPMV_I32_OP_ORDER: src = &p->sch.order; break;
        case SPMV_I32_STREAM_MAP:
            tmp.assign(p->sch.stream, p->sch.stream + SPMV_N_VERTICES);
            src = &tmp;
            break;
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

extern "C" int spmv_plan_reset_times(spmv_plan_t *p)
{
    if (!p) return set_error(SPMV_EINVAL, "plan is NULL");
    std::fill(p->ms, p->ms + SPMV_N_VERTICES + 1, 0.0);
    std::fill(p->cnt, p->cnt + SPMV_N_VERTICES + 1, 0.0);
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
