// gfx950 kernels of the rank-share SpMV: Pack (gather), Unpack (permuted
// copy), the vector-CSR product used for both y_L and y_R, and the combine
// step y[i] = y_L[i] + y_R[i] for plans that run y_R before or beside y_L.
//
// SpMV in FP64 moves >= 12 bytes (value + column) per 2 flops, far below the
// MI355X ridge point, so these kernels are written for HBM streaming, not for
// the matrix cores: every load of the A stream is coalesced across the
// wavefront, the row pointers of a block are staged once in LDS, each row is
// reduced inside its group of lanes with cross-lane moves, and block tiles
// can be laid out so that each XCD (with its private L2) walks a contiguous
// range of rows and reuses the x entries its neighbours touch.
#include "spmv_internal.h"

namespace spmv {
namespace {

constexpr int kBlock = 256;   // 4 wave64 per block
constexpr int kXcds = 8;      // MI355X: 8 XCDs, workgroups dispatched round-robin

// Block b of nb is dispatched to XCD b % 8.  With remap, XCD x processes the
// contiguous tile range [x*per + min(x, rem), ...) instead of every 8th tile,
// so the x entries shared by neighbouring tiles stay in one L2.  Bijective for
// any nb.
__device__ __forceinline__ int tile_of_block(int b, int nb, int remap)
{
    if (remap != 1) return b;
    const int xcd = b % kXcds, local = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    return xcd * per + min(xcd, rem) + local;
}

// Sum over each aligned group of LPR lanes (LPR a power of two <= 64).  The
// butterfly order is fixed, so the result depends only on the lane values.
template <int LPR>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// y = A x over n_rows rows; LPR lanes per row, kBlock/LPR rows per block.
// acc == nullptr: out[row] = sum.  Otherwise acc[rows[row]] += sum (the remote
// product adding into y after the local product on the same stream).
template <int LPR>
__global__ __launch_bounds__(kBlock) void k_csr_vector(
    int n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ x, double *__restrict__ out,
    const int32_t *__restrict__ rows, double *__restrict__ acc, int remap)
{
    constexpr int RPB = kBlock / LPR;
    __shared__ int32_t s_rp[RPB + 1];
    const int tile = tile_of_block(int(blockIdx.x), int(gridDim.x), remap);
    const int row0 = tile * RPB;
    for (int i = int(threadIdx.x); i <= RPB; i += kBlock) s_rp[i] = rp[min(row0 + i, n_rows)];
    __syncthreads();

    const int g = int(threadIdx.x) / LPR, lane = int(threadIdx.x) % LPR;
    const int row = row0 + g;
    double sum = 0.0;
    if (row < n_rows) {
        const int b = s_rp[g], e = s_rp[g + 1];
        for (int k = b + lane; k < e; k += LPR) {
            const int32_t c = __builtin_nontemporal_load(col + k);
            const double a = __builtin_nontemporal_load(val + k);
            sum = fma(a, x[c], sum);
        }
    }
    sum = group_sum<LPR>(sum);
    if (lane == 0 && row < n_rows) {
        if (acc)
            acc[rows[row]] += sum;
        else
            out[row] = sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_gather(const double *__restrict__ src,
                                                   const int32_t *__restrict__ idx,
                                                   double *__restrict__ dst, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = src[idx[i]];
}

__global__ __launch_bounds__(kBlock) void k_combine(const int32_t *__restrict__ rows,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ y, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < n; j += stride)
        y[rows[j]] += part[j];
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    return unsigned(std::min<int64_t>(std::max<int64_t>(b, 1), 65536));
}

template <int LPR>
hipError_t launch_csr_t(const CsrDev &A, const double *x, double *out, double *acc, int remap,
                        hipStream_t s)
{
    constexpr int RPB = kBlock / LPR;
    const int64_t nb = (int64_t(A.n_rows) + RPB - 1) / RPB;
    hipLaunchKernelGGL(k_csr_vector<LPR>, dim3(unsigned(nb)), dim3(kBlock), 0, s, A.n_rows, A.rp,
                       A.col, A.val, x, out, A.rows, acc, remap);
    return hipGetLastError();
}

}  // namespace

int auto_lanes(int64_t nnz, int64_t rows)
{
    if (rows <= 0) return 1;
    const double mean = double(nnz) / double(rows);
    int l = 1;
    while (l < 64 && double(l) < mean) l <<= 1;
    return l;
}

hipError_t launch_pack(const double *x, const int32_t *idx, double *out, int64_t n,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kBlock), 0, s, x, idx, out, n);
    return hipGetLastError();
}

hipError_t launch_unpack(const double *recv, const int32_t *perm, double *xh, int64_t n,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kBlock), 0, s, recv, perm, xh, n);
    return hipGetLastError();
}

hipError_t launch_combine(const int32_t *rows, const double *part, double *y, int64_t n,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine, dim3(grid_for(n)), dim3(kBlock), 0, s, rows, part, y, n);
    return hipGetLastError();
}

hipError_t launch_csr(const CsrDev &A, const double *x, double *out, double *acc, int lanes,
                      int xcd_remap, hipStream_t s)
{
    if (A.n_rows <= 0) return hipSuccess;
    const int remap = xcd_remap == 2 ? 0 : 1;
    switch (lanes) {
        case 1: return launch_csr_t<1>(A, x, out, acc, remap, s);
        case 2: return launch_csr_t<2>(A, x, out, acc, remap, s);
        case 4: return launch_csr_t<4>(A, x, out, acc, remap, s);
        case 8: return launch_csr_t<8>(A, x, out, acc, remap, s);
        case 16: return launch_csr_t<16>(A, x, out, acc, remap, s);
        case 32: return launch_csr_t<32>(A, x, out, acc, remap, s);
        case 64: return launch_csr_t<64>(A, x, out, acc, remap, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spmv
