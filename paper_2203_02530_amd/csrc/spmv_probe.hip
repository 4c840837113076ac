// HBM probe: STREAM-like read and copy kernels that give the achievable
// bandwidth ceiling of the device for a given transfer size, the yardstick
// the SpMV kernels are compared against beside the 8 TB/s data-sheet peak.
//   read: every byte of src is loaded once (16-byte non-temporal loads) and
//         folded into one value per block, written to dst[block]
//   copy: dst = src with 16-byte loads and stores
//   gather: random 8-byte loads at hashed indices, 8 per thread, either each
//         block inside the window of its XCD (src cut into 8 equal windows,
//         block b in window b mod 8: the access pattern of the column-slab
//         remote product, served by the XCD's L2) or over all of src (the
//         pattern of a remote product whose halo exceeds the L2), folded
//         into one value per block
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

// An integer hash (xor-shift-multiply rounds) that spreads consecutive
// thread ids over the index space.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

constexpr int kGathersPerThread = 8;

// Every index is base + (hash mod w) with base + w <= 8 * w (per_xcd) or
// base = 0 and w = the whole buffer, so every load stays inside src.
__global__ __launch_bounds__(kProbeBlock) void k_probe_gather(const double *__restrict__ src,
                                                              uint32_t w, int per_xcd,
                                                              double *__restrict__ out)
{
    const uint32_t b = blockIdx.x;
    const uint32_t base = per_xcd ? (b % uint32_t(kXcds)) * w : 0u;
    uint32_t h = probe_hash(b * kProbeBlock + threadIdx.x + 0x9e3779b9u);
    double v[kGathersPerThread];
#pragma unroll
    for (int k = 0; k < kGathersPerThread; ++k) {
        h = probe_hash(h + uint32_t(k));
        v[k] = src[base + h % w];
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kGathersPerThread; ++k) acc += v[k];
    __shared__ double s[kProbeBlock / 64];
    acc = group_sum<64>(acc);
    if ((threadIdx.x & 63) == 63) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

}  // namespace
}  // namespace spmv

using namespace spmv;

extern "C" int64_t spmv_gathers_per_probe_block(void)
{
    return int64_t(kProbeBlock) * kGathersPerThread;
}

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
    } else if (mode == 2 || mode == 3) {
        const int64_t doubles = bytes / 8;
        const int64_t w = mode == 2 ? doubles / kXcds : doubles;
        if (w < 1 || doubles > int64_t(UINT32_MAX))
            return set_error(SPMV_EINVAL, "gather probe needs 8 to 2^32 - 1 doubles");
        hipLaunchKernelGGL(k_probe_gather, dim3(unsigned(blocks)), dim3(kProbeBlock), 0, s,
                           static_cast<const double *>(src), uint32_t(w), mode == 2 ? 1 : 0,
                           static_cast<double *>(dst));
    } else {
        return set_error(SPMV_EINVAL, "probe mode must be 0 (read), 1 (copy), 2 or 3 (gather)");
    }
    SPMV_HIP(hipGetLastError());
    return SPMV_OK;
}
