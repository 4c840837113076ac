// spmv_exec_static: one exec of a plan whose per-exec intermediate data
// (send buffer, receive buffer, unpacked halo, remote partial sums, column
// slab partial sums) lives in one fixed device array of this library instead
// of the plan's own arena.  The call allocates nothing.
//
// The array is a file-scope __device__ variable: every GPU the library is
// loaded on holds its own copy, at its own address, until the process ends.
// Host code never passes the array's name to a kernel (on the host it only
// names a stand-in symbol); it looks the device address up once per device
// with hipGetSymbolAddress and uses that pointer.
#include <array>
#include <mutex>

#include "spmv_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(SPMV_STATIC_SCRATCH_BYTES);
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
std::array<char *, kMaxDevices> g_ptr{};   // device address of `scratch`, per device

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// The device address of this device's copy of `scratch`, looked up once with
// `device` current.
int scratch_ptr(int device, char **out)
{
    if (device < 0 || device >= kMaxDevices)
        return spmv::set_error(SPMV_EINVAL, "device " + std::to_string(device) +
                                                " beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[size_t(device)]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return spmv::hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return spmv::set_error(SPMV_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_ptr[size_t(device)] = static_cast<char *>(p);
    }
    *out = g_ptr[size_t(device)];
    return SPMV_OK;
}

// Bytes of static scratch one exec of the plan uses, laid out as send
// buffer, receive buffer, unpacked halo (when Unpack is not fused), remote
// partial sums, column-slab partial sums; each piece 256-byte aligned.
size_t scratch_need(const spmv_plan *p, size_t *off)
{
    const spmv::Share &S = p->share;
    const size_t n_send = S.send_idx.size(), n_halo = S.halo.size(), n_rr = S.R_rows.size();
    const size_t bytes[5] = {n_send * 8, n_halo * 8, p->fuse_unpack ? 0 : n_halo * 8, n_rr * 8,
                             p->cfg[1].form == 5 ? size_t(spmv::kSlabs) * n_rr * 8 : 0};
    size_t cur = 0;
    for (int i = 0; i < 5; ++i) {
        off[i] = cur;
        cur += align_up(bytes[i]);
    }
    return cur;
}

// Points the plan's scratch views at the static array for one call and puts
// the plan's own views back afterwards, also on an error return.
struct ScratchSwap {
    spmv_plan *p;
    double *send, *recv, *xhalo, *part, *slab;
    ScratchSwap(spmv_plan *plan, char *base, const size_t *off)
        : p(plan), send(plan->d_sendbuf), recv(plan->d_recvbuf), xhalo(plan->d_xhalo),
          part(plan->d_part), slab(plan->d_slab_part)
    {
        p->d_sendbuf = reinterpret_cast<double *>(base + off[0]);
        p->d_recvbuf = reinterpret_cast<double *>(base + off[1]);
        p->d_xhalo = p->fuse_unpack ? nullptr : reinterpret_cast<double *>(base + off[2]);
        p->d_part = reinterpret_cast<double *>(base + off[3]);
        p->d_slab_part = p->cfg[1].form == 5 ? reinterpret_cast<double *>(base + off[4]) : nullptr;
    }
    ~ScratchSwap()
    {
        p->d_sendbuf = send;
        p->d_recvbuf = recv;
        p->d_xhalo = xhalo;
        p->d_part = part;
        p->d_slab_part = slab;
    }
};

}  // namespace

extern "C" int spmv_exec_static(spmv_plan_t *p, const double *x, double *y, void *stream)
{
    if (!p) return spmv::set_error(SPMV_EINVAL, "plan is NULL");
    size_t off[5];
    const size_t need = scratch_need(p, off);
    if (need > kScratchBytes)
        return spmv::set_error(SPMV_EINVAL,
                               "the plan's exec needs " + std::to_string(need) +
                                   " bytes of scratch; the static array holds " +
                                   std::to_string(kScratchBytes));
    if (p->host_only) return spmv::set_error(SPMV_ESTATE, "plan was created host-only");
    const spmv::Share &S = p->share;
    if (S.n_loc > 0 && (!x || !y)) return spmv::set_error(SPMV_EINVAL, "x or y is NULL");
    if (x && y && x == y) return spmv::set_error(SPMV_EINVAL, "x and y alias");
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev != p->device) SPMV_HIP(hipSetDevice(p->device));
    char *base = nullptr;
    if (int rc = scratch_ptr(p->device, &base)) return rc;
    // every piece is written in full before it is read (Pack before the
    // send copy, the receive copy before Unpack / y_R, each product's
    // partial sums before their sum), so nothing needs clearing
    ScratchSwap swap(p, base, off);
    return spmv_exec(p, x, y, stream);
}

extern "C" int64_t spmv_static_scratch_bytes(void) { return int64_t(kScratchBytes); }
