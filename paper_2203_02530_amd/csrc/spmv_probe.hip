// HBM probe: STREAM-like read and copy kernels that give the achievable
// bandwidth ceiling of the device for a given transfer size, the yardstick
// the SpMV kernels are compared against beside the 8 TB/s data-sheet peak.
//   read: every byte of src is loaded once (16-byte non-temporal loads) and
//         folded into one value per block, written to dst[block]
//   copy: dst = src with 16-byte loads and stores
#include "spmv_device.h"
#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int kProbeBlock = 256;
typedef double v2d __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kProbeBlock) void k_probe_read(const v2d *__restrict__ src,
                                                            int64_t n, double *__restrict__ out)
{
    const int64_t stride = int64_t(gridDim.x) * kProbeBlock;
    double acc = 0.0;
    int64_t i = int64_t(blockIdx.x) * kProbeBlock + threadIdx.x;
    // four independent 16-byte loads in flight per iteration
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v2d a = __builtin_nontemporal_load(src + i);
        const v2d b = __builtin_nontemporal_load(src + i + stride);
        const v2d c = __builtin_nontemporal_load(src + i + 2 * stride);
        const v2d d = __builtin_nontemporal_load(src + i + 3 * stride);
        acc += (a.x + a.y) + (b.x + b.y) + (c.x + c.y) + (d.x + d.y);
    }
    for (; i < n; i += stride) {
        const v2d a = __builtin_nontemporal_load(src + i);
        acc += a.x + a.y;
    }
    __shared__ double s[kProbeBlock / 64];
    acc = group_sum<64>(acc);
    if ((threadIdx.x & 63) == 63) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_copy(const v2d *__restrict__ src,
                                                            v2d *__restrict__ dst, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kProbeBlock;
    for (int64_t i = int64_t(blockIdx.x) * kProbeBlock + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace
}  // namespace spmv

using namespace spmv;

extern "C" int spmv_hbm_probe(int32_t mode, const void *src, void *dst, int64_t bytes,
                              int32_t blocks, void *stream)
{
    if (!src || !dst || bytes < 16 || (bytes & 15))
        return set_error(SPMV_EINVAL, "probe needs src, dst and a byte count that is a multiple of 16");
    if (blocks <= 0) blocks = 256 * 8;
    const int64_t n = bytes / 16;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (mode == 0) {
        hipLaunchKernelGGL(k_probe_read, dim3(unsigned(blocks)), dim3(kProbeBlock), 0, s,
                           static_cast<const v2d *>(src), n, static_cast<double *>(dst));
    } else if (mode == 1) {
        hipLaunchKernelGGL(k_probe_copy, dim3(unsigned(blocks)), dim3(kProbeBlock), 0, s,
                           static_cast<const v2d *>(src), static_cast<v2d *>(dst), n);
    } else {
        return set_error(SPMV_EINVAL, "probe mode must be 0 (read) or 1 (copy)");
    }
    SPMV_HIP(hipGetLastError());
    return SPMV_OK;
}
