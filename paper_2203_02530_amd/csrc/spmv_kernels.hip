// gfx950 kernels of the rank-share SpMV: Pack (gather), Unpack (permuted
// copy), the vector-CSR product used for both y_L and y_R, and the combine
// step y[i] = y_L[i] + y_R[i] for plans that run y_R before or beside y_L.
//
// SpMV in FP64 moves >= 12 bytes (value + column) per 2 flops, far below the
// MI355X ridge point, so these kernels are written for HBM streaming, not for
// the matrix cores:
//   - every load of the A stream is coalesced across the wavefront (the lanes
//     of a group walk consecutive entries of one row, consecutive groups take
//     consecutive rows) and marked non-temporal, leaving L2 to x;
//   - the row pointers of a block are staged once in LDS;
//   - each lane group handles ROWS rows at once, issuing all their column and
//     value loads before the first wait, so a wave keeps ROWS times more bytes
//     in flight than a one-row-per-group kernel (the kernel is latency-bound
//     otherwise: one block's work is a short chain of dependent loads);
//   - rows are reduced inside their group with DPP row moves (quad_perm,
//     row_half_mirror, row_mirror) and the gfx950 permlane16/32 swaps, in a
//     fixed butterfly order, so results depend only on the lane values;
//   - block tiles can be laid out so that each XCD (with its private L2) walks
//     a contiguous range of rows and reuses the x entries neighbours touch.
#include "spmv_internal.h"
#include "spmv_stream.h"

namespace spmv {
namespace {

// out = A x over n_rows rows (acc == nullptr), or acc[rows[j]] += (A x)_j.
// LPR lanes per row; each lane group handles ROWS rows of the block's tile of
// (kBlock/LPR)*ROWS consecutive rows.  Row r of the tile belongs to sub-tile
// r / G and group r % G, so at every unrolled step consecutive groups read
// consecutive rows.
template <int LPR, int ROWS>
__global__ __launch_bounds__(kBlock) void k_csr_vector(
    int n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ x, double *__restrict__ out,
    const int32_t *__restrict__ rows, double *__restrict__ acc, int remap)
{
    constexpr int G = kBlock / LPR;
    constexpr int RPB = G * ROWS;
    __shared__ int32_t s_rp[RPB + 1];
    const int tile = tile_of_block(int(blockIdx.x), int(gridDim.x), remap);
    const int row0 = tile * RPB;
    for (int i = int(threadIdx.x); i <= RPB; i += kBlock) s_rp[i] = rp[min(row0 + i, n_rows)];
    __syncthreads();

    const int g = int(threadIdx.x) / LPR, lane = int(threadIdx.x) % LPR;
    const int first = s_rp[0];
    int k[ROWS], e[ROWS];
    double sum[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        k[i] = s_rp[i * G + g] + lane;
        e[i] = s_rp[i * G + g + 1];
        sum[i] = 0.0;
    }
    // Rows past n_rows have s_rp = rp[n_rows] on both ends: empty.  When the
    // whole tile is empty there is no valid entry to clamp to, so skip.
    if (first < s_rp[RPB]) {
        bool more = true;
        while (more) {
            int32_t c[ROWS];
            double a[ROWS];
            // all loads of the step first; a finished slot re-reads the tile's
            // first entry (always valid) and is masked out below
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                const int kc = k[i] < e[i] ? k[i] : first;
                c[i] = __builtin_nontemporal_load(col + kc);
                a[i] = __builtin_nontemporal_load(val + kc);
            }
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                const double xv = x[c[i]];
                const double f = fma(a[i], xv, sum[i]);
                sum[i] = k[i] < e[i] ? f : sum[i];
            }
            more = false;
#pragma unroll
            for (int i = 0; i < ROWS; ++i) {
                k[i] += LPR;
                more |= k[i] < e[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) sum[i] = group_sum<LPR>(sum[i]);
    if (lane == LPR - 1) {
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            const int row = row0 + i * G + g;
            if (row < n_rows) {
                if (acc)
                    acc[rows[row]] += sum[i];
                else
                    out[row] = sum[i];
            }
        }
    }
}

// Buffer-resource form of the same kernel: the A stream, x and the row
// pointers are read with buffer loads (32-bit offsets against a scalar
// resource), which keeps 64-bit addresses out of the vector registers (44 ->
// fewer VGPRs, so ROWS = 8 still runs 8 waves per SIMD) and turns a finished
// slot into an out-of-range load that returns 0 without touching memory.
// Valid while every array is below 4 GiB (checked by the launcher).
template <int LPR, int ROWS>
__global__ __launch_bounds__(kBlock) void k_csr_vector_buf(
    int n_rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ x, double *__restrict__ out,
    const int32_t *__restrict__ rows, double *__restrict__ acc, int remap, uint32_t nnz,
    uint32_t n_x)
{
    constexpr int G = kBlock / LPR;
    constexpr int RPB = G * ROWS;
    __shared__ int32_t s_rp[RPB + 1];
    const auto r_rp = rsrc(rp, uint32_t(n_rows + 1) * 4u);
    const auto r_col = rsrc(col, nnz * 4u);
    const auto r_val = rsrc(val, nnz * 8u);
    const auto r_x = rsrc(x, n_x * 8u);
    const int tile = tile_of_block(int(blockIdx.x), int(gridDim.x), remap);
    const int row0 = tile * RPB;
    for (int i = int(threadIdx.x); i <= RPB; i += kBlock)
        s_rp[i] = __builtin_amdgcn_raw_buffer_load_b32(r_rp, uint32_t(min(row0 + i, n_rows)) * 4u,
                                                       0, 0);
    __syncthreads();

    const int g = int(threadIdx.x) / LPR, lane = int(threadIdx.x) % LPR;
    int k[ROWS], e[ROWS];
    double sum[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        k[i] = s_rp[i * G + g] + lane;
        e[i] = s_rp[i * G + g + 1];
        sum[i] = 0.0;
    }
    bool more = s_rp[0] < s_rp[RPB];
    while (more) {
        int32_t c[ROWS];
        double a[ROWS];
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            const bool v = k[i] < e[i];
            c[i] = __builtin_amdgcn_raw_buffer_load_b32(r_col, v ? uint32_t(k[i]) * 4u : kOff, 0, 2);
            a[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                  r_val, v ? uint32_t(k[i]) * 8u : kOff, 0, 2));
        }
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            const bool v = k[i] < e[i];
            const double xv = __builtin_bit_cast(
                double, __builtin_amdgcn_raw_buffer_load_b64(r_x, v ? uint32_t(c[i]) * 8u : kOff, 0, 0));
            const double f = fma(a[i], xv, sum[i]);
            sum[i] = v ? f : sum[i];
        }
        more = false;
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            k[i] += LPR;
            more |= k[i] < e[i];
        }
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) sum[i] = group_sum<LPR>(sum[i]);
    if (lane == LPR - 1) {
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            const int row = row0 + i * G + g;
            if (row < n_rows) {
                if (acc)
                    acc[rows[row]] += sum[i];
                else
                    out[row] = sum[i];
            }
        }
    }
}

// Block j of a PackTail: entries [j * NT * K, (j + 1) * NT * K), each
// thread's indices first, then its gathers, then its stores; indices and
// stores stream past the L2 (non-temporal), x keeps the default policy.
template <int NT>
__device__ __forceinline__ void pack_block(const PackTail &P, int j)
{
    constexpr int K = kPackPerThread;
    const int t0 = j * NT * K + int(threadIdx.x);
    int32_t id[K];
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        id[k] = t0 + k * NT < P.n ? __builtin_nontemporal_load(P.idx + t0 + k * NT) : -1;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = id[k] >= 0 ? P.x[id[k]] : 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (t0 + k * NT < P.n) __builtin_nontemporal_store(v[k], P.dst + t0 + k * NT);
}

template <int NT>
int pack_blocks(const PackTail &P)
{
    return P.n > 0 ? (P.n + NT * kPackPerThread - 1) / (NT * kPackPerThread) : 0;
}

// Single-share stream-CSR product: one block per tile (see spmv_stream.h);
// with TAIL the n_tiles blocks are followed by the PackTail's blocks (the
// instances without it are the plain product), and with COOP each tile's
// block also loads and sums the remote part of its rows (F.tj, F.te).
template <int NPT, int VW, int SL, bool C16, bool TAIL, bool COOP = false>
__global__ __launch_bounds__(kBlock) void k_csr_stream(StreamArgs A, int remap, int n_tiles,
                                                       PackTail P, RemoteFuse F)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock / SL + 1];
    if constexpr (TAIL) {
        if (int(blockIdx.x) >= n_tiles) {   // whole block, before any barrier
            pack_block<kBlock>(P, int(blockIdx.x) - n_tiles);
            return;
        }
        const int t = (COOP && F.n_grid) ? tile_of_range(int(blockIdx.x), F.xr)
                                         : tile_of_block(int(blockIdx.x), n_tiles, remap);
        if (t < 0) return;   // whole block, before any barrier
        stream_tile<NPT, VW, SL, C16, COOP>(A, t, s_p, s_rp, &F);
    } else {
        stream_tile<NPT, VW, SL, C16>(A, tile_of_block(int(blockIdx.x), int(gridDim.x), remap),
                                      s_p, s_rp);
    }
}

// Sliced-ELL product: one wave per slice of 64 rows; lane l owns row
// 64 s + l and walks its entries in order, U at a time with all their loads
// in flight.  The v-th entries of a slice are contiguous (one 256-byte
// column load and one 512-byte value load per wave), and for banded and
// stencil matrices so are the x values they gather.  Padding entries carry
// column -1 and are skipped, so no row length is read.  With one width for
// all slices (width > 0) the slice offsets are computed, not loaded, and the
// first loads of a wave depend on nothing but its index.  Each row is an fma
// chain in entry order.
struct SellArgs {
    const int32_t *ptr, *col, *rows;
    const double *val, *x;
    double *out, *acc;
    int32_t n_rows, n_slices, width;
    uint32_t n_alloc, n_x;
};

template <int U>
__global__ __launch_bounds__(kBlock) void k_sell(SellArgs A, int remap)
{
    constexpr int kWaves = kBlock / 64;
    const int q = tile_of_block(int(blockIdx.x), int(gridDim.x), remap);
    const int slice = q * kWaves + int(threadIdx.x >> 6);
    if (slice >= A.n_slices) return;   // whole waves; no barrier below
    const int lane = int(threadIdx.x & 63);
    const int r = slice * 64 + lane;
    const auto r_col = rsrc(A.col, A.n_alloc * 4u);
    const auto r_val = rsrc(A.val, A.n_alloc * 8u);
    const auto r_x = rsrc(A.x, A.n_x * 8u);
    const int off = A.width > 0 ? slice * 64 * A.width : A.ptr[slice];
    const int w = A.width > 0 ? A.width : (A.ptr[slice + 1] - off) >> 6;
    double s = 0.0;
    for (int v0 = 0; v0 < w; v0 += U) {
        int32_t c[U];
        double a[U], xv[U];
        // columns first: the x gathers wait only for them, and the values
        // arrive while the gathers are in flight.  Every load is issued
        // unconditionally (slots past the width read out of range, giving 0)
        // so that the wait before the gathers can count the value loads.
        // Columns take the default cache policy, values the streaming one.
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = v0 + u < w;
            const int32_t cc = int32_t(__builtin_amdgcn_raw_buffer_load_b32(
                r_col, in ? uint32_t(off + (v0 + u) * 64 + lane) * 4u : kOff, 0, 0));
            c[u] = in ? cc : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                r_val, v0 + u < w ? uint32_t(off + (v0 + u) * 64 + lane) * 8u : kOff, 0, 2));
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = load_x(r_x, c[u] >= 0 ? uint32_t(c[u]) * 8u : kOff);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) s = fma(a[u], xv[u], s);
    }
    if (r < A.n_rows) {
        if (A.acc)
            A.acc[A.rows[r]] += s;
        else
            A.out[r] = s;
    }
}

struct Sell16Args {
    const void *off;               // grouped 16-bit column offsets
    const double *val, *x;
    double *out;
    int32_t n_rows, n_slices, width, groups;
    uint32_t off_bytes, n_alloc, n_x;
};

// Sliced ELL with the columns stored as 16-bit offsets from the row: per
// group of 8 entries a lane issues one 16-byte load (a wave reads 1 KiB
// contiguous), so a 7-entry stencil row costs 16 bytes of column data
// instead of 28; the values of a slice are stored in pairs, one 16-byte
// load per two entries of a row (9.03 vs 9.40 us with one 8-byte load per
// entry on the 7-point share).  x gathers and the fma chain are those of
// k_sell, in the same entry order, so both forms give the same bits.  One
// wave per block (64-thread blocks measured 2% faster than 256); the
// offsets are read with the default cache policy and the values as
// streaming (non-temporal) data, which measured 0.2-0.3 us faster than
// streaming both.
__device__ __forceinline__ void unpack16(const uint32_t w, int32_t &lo, int32_t &hi)
{
    lo = int32_t(int16_t(uint16_t(w & 0xFFFFu)));
    hi = int32_t(w) >> 16;
}

template <int NG, bool TAIL>
__global__ __launch_bounds__(64) void k_sell16(Sell16Args A, int remap, PackTail P, RemoteFuse F)
{
    constexpr int U = 8 * NG;
    if constexpr (TAIL) {
        if (int(blockIdx.x) >= A.n_slices) {   // the PackTail's blocks follow the slices
            pack_block<64>(P, int(blockIdx.x) - A.n_slices);
            return;
        }
    }
    const int slice = tile_of_block(int(blockIdx.x), TAIL ? A.n_slices : int(gridDim.x), remap);
    if (slice >= A.n_slices) return;
    const int lane = int(threadIdx.x);
    const int r = slice * 64 + lane;
    const auto r_off = rsrc(A.off, A.off_bytes);
    const auto r_val = rsrc(A.val, A.n_alloc * 8u);
    const auto r_x = rsrc(A.x, A.n_x * 8u);
    const int w = A.width, G = A.groups;
    const int voff = slice * 64 * w;
    double s = 0.0;
    for (int g0 = 0; g0 < G; g0 += NG) {
        int32_t d[U];
        double a[U], xv[U];
        // every load is issued unconditionally (out-of-range slots read
        // past the buffer, giving 0) so that the gathers wait only for the
        // offset loads, not for the value loads behind them
#pragma unroll
        for (int h = 0; h < NG; ++h) {
            const bool in = g0 + h < G;
            const auto o = __builtin_amdgcn_raw_buffer_load_b128(
                r_off, in ? uint32_t(((slice * G + g0 + h) * 64 + lane) * 16) : kOff, 0, 0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int32_t lo, hi;
                unpack16(uint32_t(o[k]), lo, hi);
                d[8 * h + 2 * k] = in ? lo : int32_t(kPad16);
                d[8 * h + 2 * k + 1] = in ? hi : int32_t(kPad16);
            }
        }
        // values in pairs: one 16-byte load per two entries of a row, and
        // the odd last entry of an odd-width row on its own
#pragma unroll
        for (int j = 0; j < U / 2; ++j) {
            const int v = g0 * 8 + 2 * j;
            const auto q = __builtin_amdgcn_raw_buffer_load_b128(
                r_val, v + 1 < w ? uint32_t(voff + (v >> 1) * 128 + lane * 2) * 8u : kOff, 0, 2);
            a[2 * j] = __builtin_bit_cast(double, (uint64_t(q[1]) << 32) | q[0]);
            a[2 * j + 1] = __builtin_bit_cast(double, (uint64_t(q[3]) << 32) | q[2]);
        }
        const int tail_u = (w & 1) ? (w - 1) - g0 * 8 : -1;
        const double tail = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
            r_val, tail_u >= 0 && tail_u < U ? uint32_t(voff + (w - 1) * 64 + lane) * 8u : kOff, 0,
            2));
#pragma unroll
        for (int u = 0; u < U; ++u)
            xv[u] = load_x(r_x, d[u] != kPad16 ? uint32_t(r + d[u]) * 8u : kOff);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double av = u == tail_u ? tail : a[u];
            if (d[u] != kPad16) s = fma(av, xv[u], s);
        }
    }
    if (r < A.n_rows) {
        if constexpr (TAIL)
            if (F.mask) s = remote_add(F, r, s);
        A.out[r] = s;
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

template <int LPR, int ROWS>
hipError_t launch_csr_t(const CsrDev &A, const double *x, double *out, double *acc, int remap,
                        bool buf, hipStream_t s)
{
    constexpr int RPB = (kBlock / LPR) * ROWS;
    const int64_t nb = (int64_t(A.n_rows) + RPB - 1) / RPB;
    if (buf) {
        hipLaunchKernelGGL((k_csr_vector_buf<LPR, ROWS>), dim3(unsigned(nb)), dim3(kBlock), 0, s,
                           A.n_rows, A.rp, A.col, A.val, x, out, A.rows, acc, remap,
                           uint32_t(A.nnz_alloc), uint32_t(A.n_x));
    } else {
        hipLaunchKernelGGL((k_csr_vector<LPR, ROWS>), dim3(unsigned(nb)), dim3(kBlock), 0, s,
                           A.n_rows, A.rp, A.col, A.val, x, out, A.rows, acc, remap);
    }
    return hipGetLastError();
}

template <int LPR>
hipError_t launch_csr_l(const CsrDev &A, const double *x, double *out, double *acc, int rows,
                        int remap, bool buf, hipStream_t s)
{
    switch (rows) {
        case 1: return launch_csr_t<LPR, 1>(A, x, out, acc, remap, buf, s);
        case 2: return launch_csr_t<LPR, 2>(A, x, out, acc, remap, buf, s);
        case 4: return launch_csr_t<LPR, 4>(A, x, out, acc, remap, buf, s);
        case 8: return launch_csr_t<LPR, 8>(A, x, out, acc, remap, buf, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NPT, int VW, int SL>
hipError_t launch_stream_t(const CsrDev &A, const double *x, double *out, double *acc, int remap,
                           hipStream_t s, const PackTail &tail, const RemoteFuse &rem)
{
    StreamArgs a;
    a.tile_row = A.tile_row;
    a.tile_k = A.tile_k;
    a.rp = A.rp;
    a.col = A.col;
    a.rows = A.rows;
    a.val = A.val;
    a.x = x;
    a.out = out;
    a.acc = acc;
    a.nnz_alloc = uint32_t(A.nnz_alloc);
    a.n_x = uint32_t(A.n_x);
    static_assert(sizeof(RemoteFuse::xr) / sizeof(int32_t) == kXcds + 1, "one range per XCD");
    const bool coop = rem.mask && rem.tj;
    // with XCD ranges the product's blocks are n_grid, the Pack blocks after them
    const int nt = coop && rem.n_grid ? rem.n_grid : std::max(A.n_tiles, 0);
    const int nb = pack_blocks<kBlock>(tail);
    const unsigned grid = unsigned(nt + nb);
    if (grid == 0) return hipSuccess;
    const bool tl = nb > 0 || rem.mask;   // the resident step's instance
    // remote sums lengthen the boundary tiles: start the last of them first
    if (rem.mask && remap == 1) remap = 3;
    // a tile's remote products go where its window's products were
    if (coop && (rem.tile_cap > NPT * kBlock || rem.tile_cap > kTileRemoteCap ||
                 (rem.n_grid && rem.xr[kXcds] != A.n_tiles)))
        return hipErrorInvalidValue;
    if (A.col16 && coop)
        hipLaunchKernelGGL((k_csr_stream<NPT, VW, SL, true, true, true>), dim3(grid), dim3(kBlock),
                           0, s, a, remap, nt, tail, rem);
    else if (coop)
        hipLaunchKernelGGL((k_csr_stream<NPT, VW, SL, false, true, true>), dim3(grid),
                           dim3(kBlock), 0, s, a, remap, nt, tail, rem);
    else if (A.col16 && tl)
        hipLaunchKernelGGL((k_csr_stream<NPT, VW, SL, true, true>), dim3(grid), dim3(kBlock), 0, s,
                           a, remap, nt, tail, rem);
    else if (A.col16)
        hipLaunchKernelGGL((k_csr_stream<NPT, VW, SL, true, false>), dim3(grid), dim3(kBlock), 0,
                           s, a, remap, nt, tail, rem);
    else if (tl)
        hipLaunchKernelGGL((k_csr_stream<NPT, VW, SL, false, true>), dim3(grid), dim3(kBlock), 0,
                           s, a, remap, nt, tail, rem);
    else
        hipLaunchKernelGGL((k_csr_stream<NPT, VW, SL, false, false>), dim3(grid), dim3(kBlock), 0,
                           s, a, remap, nt, tail, rem);
    return hipGetLastError();
}

template <int NPT, int VW>
hipError_t launch_stream_v(const CsrDev &A, const double *x, double *out, double *acc, int sl,
                           int remap, hipStream_t s, const PackTail &tail, const RemoteFuse &rem)
{
    switch (sl) {
        case 1: return launch_stream_t<NPT, VW, 1>(A, x, out, acc, remap, s, tail, rem);
        case 2: return launch_stream_t<NPT, VW, 2>(A, x, out, acc, remap, s, tail, rem);
        case 4: return launch_stream_t<NPT, VW, 4>(A, x, out, acc, remap, s, tail, rem);
        case 8: return launch_stream_t<NPT, VW, 8>(A, x, out, acc, remap, s, tail, rem);
        case 16: return launch_stream_t<NPT, VW, 16>(A, x, out, acc, remap, s, tail, rem);
        default: return hipErrorInvalidValue;
    }
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

int auto_rows(int lanes, int64_t rows)
{
    // Enough rows per lane group to keep several loads in flight per lane.
    // Four rows per lane group was the best setting for every lane count on
    // the stencil shares; fewer for inputs too small to fill the chip.
    int r = 4;
    while (r > 1 && rows < int64_t(kBlock / lanes) * r * 512) r >>= 1;
    return r;
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

hipError_t launch_sell(const CsrDev &A, const double *x, double *out, double *acc,
                       int xcd_remap, hipStream_t s)
{
    if (A.n_slices <= 0) return hipSuccess;
    SellArgs a;
    a.ptr = A.sell_ptr;
    a.col = A.col;
    a.rows = A.rows;
    a.val = A.val;
    a.x = x;
    a.out = out;
    a.acc = acc;
    a.n_rows = A.n_rows;
    a.n_slices = A.n_slices;
    a.width = A.sell_width;
    a.n_alloc = uint32_t(A.nnz_alloc);
    a.n_x = uint32_t(A.n_x);
    const unsigned grid = unsigned((A.n_slices + kBlock / 64 - 1) / (kBlock / 64));
    const int remap = xcd_remap == 2 ? 0 : 1;
    switch (A.sell_u) {
        case 4: hipLaunchKernelGGL(k_sell<4>, dim3(grid), dim3(kBlock), 0, s, a, remap); break;
        case 8: hipLaunchKernelGGL(k_sell<8>, dim3(grid), dim3(kBlock), 0, s, a, remap); break;
        case 16: hipLaunchKernelGGL(k_sell<16>, dim3(grid), dim3(kBlock), 0, s, a, remap); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sell16(const CsrDev &A, const double *x, double *out, int xcd_remap,
                         hipStream_t s, const PackTail &tail, const RemoteFuse &rem)
{
    if (A.n_slices < 0 || (A.n_slices == 0 && tail.n <= 0)) return hipSuccess;
    if (A.n_slices > 0 && (A.sell_width <= 0 || A.rows)) return hipErrorInvalidValue;
    Sell16Args a;
    a.off = A.col;
    a.val = A.val;
    a.x = x;
    a.out = out;
    a.n_rows = A.n_rows;
    a.n_slices = A.n_slices;
    a.width = A.sell_width;
    a.groups = (A.sell_width + 7) / 8;
    a.off_bytes = A.off_bytes;
    a.n_alloc = uint32_t(A.nnz_alloc);
    a.n_x = uint32_t(A.n_x);
    const int nb = pack_blocks<64>(tail);
    const unsigned grid = unsigned(A.n_slices + nb);
    // remote sums lengthen the boundary slices: start the last of them first
    const int remap = xcd_remap == 2 ? 0 : rem.mask ? 3 : 1;
    switch (A.sell_u * 2 + (nb > 0 || rem.mask ? 1 : 0)) {
        case 16: hipLaunchKernelGGL((k_sell16<1, false>), dim3(grid), dim3(64), 0, s, a, remap, tail, rem); break;
        case 17: hipLaunchKernelGGL((k_sell16<1, true>), dim3(grid), dim3(64), 0, s, a, remap, tail, rem); break;
        case 32: hipLaunchKernelGGL((k_sell16<2, false>), dim3(grid), dim3(64), 0, s, a, remap, tail, rem); break;
        case 33: hipLaunchKernelGGL((k_sell16<2, true>), dim3(grid), dim3(64), 0, s, a, remap, tail, rem); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int stream_cap(int npt) { return kBlock * npt; }
int stream_maxr(int sum_lanes) { return kBlock / sum_lanes; }

hipError_t launch_csr_stream(const CsrDev &A, const double *x, double *out, double *acc, int npt,
                             int vw, int sum_lanes, int xcd_remap, hipStream_t s,
                             const PackTail &tail, const RemoteFuse &rem)
{
    if (A.n_tiles <= 0 && tail.n <= 0) return hipSuccess;
    const int remap = xcd_remap == 2 ? 0 : 1;
    if (vw == 2) {
        switch (npt) {
            case 4: return launch_stream_v<4, 2>(A, x, out, acc, sum_lanes, remap, s, tail, rem);
            case 8: return launch_stream_v<8, 2>(A, x, out, acc, sum_lanes, remap, s, tail, rem);
            case 16: return launch_stream_v<16, 2>(A, x, out, acc, sum_lanes, remap, s, tail, rem);
            default: return hipErrorInvalidValue;
        }
    }
    if (vw == 4) {
        switch (npt) {
            case 4: return launch_stream_v<4, 4>(A, x, out, acc, sum_lanes, remap, s, tail, rem);
            case 8: return launch_stream_v<8, 4>(A, x, out, acc, sum_lanes, remap, s, tail, rem);
            case 16: return launch_stream_v<16, 4>(A, x, out, acc, sum_lanes, remap, s, tail, rem);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_csr(const CsrDev &A, const double *x, double *out, double *acc, int lanes,
                      int rows, int xcd_remap, bool allow_buffer, hipStream_t s)
{
    if (A.n_rows <= 0) return hipSuccess;
    const int remap = xcd_remap == 2 ? 0 : 1;
    // buffer resources address at most 4 GiB - 16 (the out-of-range offset)
    constexpr int64_t kMax = (int64_t(1) << 32) - 64;
    const bool buf = allow_buffer && A.nnz_alloc * 8 < kMax && A.n_x * 8 < kMax &&
                     (int64_t(A.n_rows) + 1) * 4 < kMax;
    switch (lanes) {
        case 1: return launch_csr_l<1>(A, x, out, acc, rows, remap, buf, s);
        case 2: return launch_csr_l<2>(A, x, out, acc, rows, remap, buf, s);
        case 4: return launch_csr_l<4>(A, x, out, acc, rows, remap, buf, s);
        case 8: return launch_csr_l<8>(A, x, out, acc, rows, remap, buf, s);
        case 16: return launch_csr_l<16>(A, x, out, acc, rows, remap, buf, s);
        case 32: return launch_csr_l<32>(A, x, out, acc, rows, remap, buf, s);
        case 64: return launch_csr_l<64>(A, x, out, acc, rows, remap, buf, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {

static_assert(kSlabs == kXcds, "one column slab per XCD");

struct SlabArgs {
    StreamArgs s[kSlabs];
    int32_t n_tiles[kSlabs];
};

// Column slabs: block b works on slab b % kSlabs, which the hardware's
// round-robin dealing of blocks places on XCD b % kSlabs, and takes that
// slab's tile b / kSlabs.  Each slab writes its row sums to its own part of
// the partial-sum array.
template <int NPT, int VW, int SL>
__global__ __launch_bounds__(kBlock) void k_csr_slabs(const SlabArgs a)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[kBlock / SL + 1];
    const int k = int(blockIdx.x) % kSlabs, q = int(blockIdx.x) / kSlabs;
    if (q >= a.n_tiles[k]) return;   // whole block, before any barrier
    stream_tile<NPT, VW, SL, false>(a.s[k], q, s_p, s_rp);
}

// The same with wide tiles: RPT * kBlock rows per tile at most, one thread
// per row.
template <int NPT, int VW, int RPT>
__global__ __launch_bounds__(kBlock) void k_csr_slabs_wide(const SlabArgs a)
{
    __shared__ double s_p[kBlock * NPT];
    __shared__ int32_t s_rp[RPT * kBlock + 1];
    const int k = int(blockIdx.x) % kSlabs, q = int(blockIdx.x) / kSlabs;
    if (q >= a.n_tiles[k]) return;   // whole block, before any barrier
    wide_tile<NPT, VW, RPT>(a.s[k], q, s_p, s_rp);
}

// y_R of row i = the slab partial sums added in slab order; stored, or added
// into y at the row's local index.
__global__ __launch_bounds__(kBlock) void k_slab_sum(const double *__restrict__ part, int64_t n,
                                                     const int32_t *__restrict__ rows,
                                                     double *__restrict__ out,
                                                     double *__restrict__ acc)
{
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        double s = part[i];
#pragma unroll
        for (int k = 1; k < kSlabs; ++k) s += part[k * n + i];
        if (acc)
            acc[rows[i]] += s;
        else
            out[i] = s;
    }
}

template <int NPT, int VW, int SL, int RPT>
hipError_t launch_slabs_t(const SlabDev &A, hipStream_t s)
{
    SlabArgs a;
    int64_t most = 0;
    for (int k = 0; k < kSlabs; ++k) {
        StreamArgs &t = a.s[k];
        t.tile_row = A.tile_row + A.tile_off[k];
        t.tile_k = A.tile_k + A.tile_off[k];
        t.rp = A.rp + int64_t(k) * (A.n_rows + 1);
        t.col = A.col + A.nnz_off[k];
        t.rows = nullptr;
        t.val = A.val + A.nnz_off[k];
        t.x = A.x;
        t.out = A.part + int64_t(k) * A.n_rows;
        t.acc = nullptr;
        t.nnz_alloc = uint32_t(A.nnz_alloc - A.nnz_off[k]);
        t.n_x = uint32_t(A.n_x);
        a.n_tiles[k] = int32_t(A.tile_off[k + 1] - A.tile_off[k] - 1);
        most = std::max<int64_t>(most, a.n_tiles[k]);
    }
    if (most > 0) {
        if constexpr (RPT == 1)
            hipLaunchKernelGGL((k_csr_slabs<NPT, VW, SL>), dim3(unsigned(most * kSlabs)),
                               dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_csr_slabs_wide<NPT, VW, RPT>), dim3(unsigned(most * kSlabs)),
                               dim3(kBlock), 0, s, a);
    }
    hipLaunchKernelGGL(k_slab_sum, dim3(grid_for(A.n_rows)), dim3(kBlock), 0, s, A.part,
                       int64_t(A.n_rows), A.rows, A.out, A.acc);
    return hipGetLastError();
}

template <int NPT, int VW>
hipError_t launch_slabs_v(const SlabDev &A, hipStream_t s)
{
    if (A.rpt > 1) {
        if (A.lanes != 1) return hipErrorInvalidValue;
        switch (A.rpt) {
            case 2: return launch_slabs_t<NPT, VW, 1, 2>(A, s);
            case 4: return launch_slabs_t<NPT, VW, 1, 4>(A, s);
            case 8: return launch_slabs_t<NPT, VW, 1, 8>(A, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (A.lanes) {
        case 1: return launch_slabs_t<NPT, VW, 1, 1>(A, s);
        case 2: return launch_slabs_t<NPT, VW, 2, 1>(A, s);
        case 4: return launch_slabs_t<NPT, VW, 4, 1>(A, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_slabs(const SlabDev &A, hipStream_t s)
{
    if (A.n_rows <= 0) return hipSuccess;
    if (A.width == 2) {
        switch (A.chunk) {
            case 4: return launch_slabs_v<4, 2>(A, s);
            case 8: return launch_slabs_v<8, 2>(A, s);
            case 16: return launch_slabs_v<16, 2>(A, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (A.width == 4) {
        switch (A.chunk) {
            case 4: return launch_slabs_v<4, 4>(A, s);
            case 8: return launch_slabs_v<8, 4>(A, s);
            case 16: return launch_slabs_v<16, 4>(A, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace spmv
