// Device code shared by the single-share and the grouped (batched) kernels:
// buffer-resource loads and the stream-CSR tile body.
//
// Stream CSR: rows are cut on the host into tiles at row boundaries; a tile
// holds at most MAXR = kBlock / SL rows whose entries fit one window of
// CAP = kBlock * NPT entries starting at the tile's first entry rounded down
// to VW (or it is a single row longer than the window).  The block streams
// the window with coalesced VW-wide loads of col/val (no idle lanes, no
// per-row pointer chase before the loads), gathers x, stages the products in
// LDS, and SL lanes per row sum them in a fixed order.  A single row longer
// than the window is summed by the whole block, chunk by chunk, with a
// fixed-order block reduction.  The result of a tile depends only on the
// tile, so a share computes the same bits alone or in any batch.
#pragma once

#include "spmv_device.h"
#include "spmv_internal.h"

namespace spmv {

constexpr int kBlock = 256;                // 4 wave64 per block
constexpr int kRsrcWord3 = 0x00020000;     // raw buffer, gfx9-family data format
constexpr uint32_t kOff = 0xFFFFFFF0u;     // out-of-range offset: the load returns 0
constexpr uint32_t kNoEntry = 0xFFFFFFFFu; // "no vector" marker for load_vec

// Buffer resource over [p, p + bytes): 32-bit offsets against a scalar
// descriptor keep 64-bit addresses out of vector registers, and a load past
// `bytes` returns 0 without touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, int(bytes), kRsrcWord3);
}

// VW consecutive entries (columns and values) starting at entry e; e ==
// kNoEntry loads nothing (zeros).  Device col/val arrays are padded, so a
// vector never straddles the end of its buffer.
template <int VW>
__device__ __forceinline__ void load_vec(__amdgpu_buffer_rsrc_t rc, __amdgpu_buffer_rsrc_t rv,
                                         uint32_t e, int32_t *c, double *a)
{
    const uint32_t oc = e == kNoEntry ? kOff : e * 4u;
    const uint32_t ov = e == kNoEntry ? kOff : e * 8u;
    if constexpr (VW == 1) {
        c[0] = __builtin_amdgcn_raw_buffer_load_b32(rc, oc, 0, 2);
        a[0] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, ov, 0, 2));
    } else if constexpr (VW == 2) {
        const auto cc = __builtin_amdgcn_raw_buffer_load_b64(rc, oc, 0, 2);
        const auto vv = __builtin_amdgcn_raw_buffer_load_b128(rv, ov, 0, 2);
        c[0] = int32_t(cc[0]);
        c[1] = int32_t(cc[1]);
        a[0] = __builtin_bit_cast(double, (uint64_t(vv[1]) << 32) | vv[0]);
        a[1] = __builtin_bit_cast(double, (uint64_t(vv[3]) << 32) | vv[2]);
    } else {
        static_assert(VW == 4, "VW must be 1, 2 or 4");
        const auto cc = __builtin_amdgcn_raw_buffer_load_b128(rc, oc, 0, 2);
        const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rv, ov, 0, 2);
        const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(rv, ov == kOff ? kOff : ov + 16u, 0, 2);
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = int32_t(cc[j]);
        a[0] = __builtin_bit_cast(double, (uint64_t(v0[1]) << 32) | v0[0]);
        a[1] = __builtin_bit_cast(double, (uint64_t(v0[3]) << 32) | v0[2]);
        a[2] = __builtin_bit_cast(double, (uint64_t(v1[1]) << 32) | v1[0]);
        a[3] = __builtin_bit_cast(double, (uint64_t(v1[3]) << 32) | v1[2]);
    }
}

// The two halves of load_vec, so that a caller can issue all columns first.
// Columns are read with the default cache policy, values as streaming
// (non-temporal) data: streaming the columns too measured 3-4% slower on
// the 7- and 27-point shares.
template <int VW>
__device__ __forceinline__ void load_cols(__amdgpu_buffer_rsrc_t rc, uint32_t e, int32_t *c)
{
    const uint32_t oc = e == kNoEntry ? kOff : e * 4u;
    if constexpr (VW == 2) {
        const auto cc = __builtin_amdgcn_raw_buffer_load_b64(rc, oc, 0, 0);
        c[0] = int32_t(cc[0]);
        c[1] = int32_t(cc[1]);
    } else {
        static_assert(VW == 4, "VW must be 2 or 4");
        const auto cc = __builtin_amdgcn_raw_buffer_load_b128(rc, oc, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = int32_t(cc[j]);
    }
}

// The same for 16-bit column offsets from a base row (the tile's first
// row): VW offsets in one 4- or 8-byte load at byte 2e.
template <int VW>
__device__ __forceinline__ void load_cols16(__amdgpu_buffer_rsrc_t rc, uint32_t e, int32_t base_row,
                                            int32_t *c)
{
    const uint32_t oc = e == kNoEntry ? kOff : e * 2u;
    if constexpr (VW == 2) {
        const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rc, oc, 0, 0);
        c[0] = base_row + int32_t(int16_t(uint16_t(w & 0xFFFFu)));
        c[1] = base_row + (int32_t(w) >> 16);
    } else {
        static_assert(VW == 4, "VW must be 2 or 4");
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(rc, oc, 0, 0);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            c[2 * j] = base_row + int32_t(int16_t(uint16_t(uint32_t(w[j]) & 0xFFFFu)));
            c[2 * j + 1] = base_row + (int32_t(w[j]) >> 16);
        }
    }
}

template <int VW>
__device__ __forceinline__ void load_vals(__amdgpu_buffer_rsrc_t rv, uint32_t e, double *a)
{
    const uint32_t ov = e == kNoEntry ? kOff : e * 8u;
    const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rv, ov, 0, 2);
    a[0] = __builtin_bit_cast(double, (uint64_t(v0[1]) << 32) | v0[0]);
    a[1] = __builtin_bit_cast(double, (uint64_t(v0[3]) << 32) | v0[2]);
    if constexpr (VW == 4) {
        const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(rv, ov == kOff ? kOff : ov + 16u, 0, 2);
        a[2] = __builtin_bit_cast(double, (uint64_t(v1[1]) << 32) | v1[0]);
        a[3] = __builtin_bit_cast(double, (uint64_t(v1[3]) << 32) | v1[2]);
    }
}

__device__ __forceinline__ double load_x(__amdgpu_buffer_rsrc_t rx, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, off, 0, 0));
}

// The remote sum of entries [e0, e1), 8 at a time: columns and values of
// the 8 first, then their x values, then the 8 terms in order (FMA: an fma
// chain; else each product rounded, then added).
template <bool FMA>
__device__ __forceinline__ double remote_sum(const RemoteFuse &F, int e0, int e1)
{
#pragma clang fp contract(off)
    double t = 0.0;
    for (int e = e0; e < e1; e += 8) {
        int32_t c[8];
        double a[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool in = e + u < e1;
            c[u] = in ? F.col[e + u] : 0;
            a[u] = in ? F.val[e + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = e + u < e1 ? F.xh[c[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (e + u >= e1) break;
            if constexpr (FMA) {
                t = fma(a[u], xv[u], t);
            } else {
                const double p = a[u] * xv[u];
                t += p;
            }
        }
    }
    return t;
}

// fl(s + s_R(r)) for a local row r with remote entries, else s.
__device__ __forceinline__ double remote_add(const RemoteFuse &F, int r, double s)
{
    const uint64_t m = F.mask[r >> 6];
    const int l = r & 63;
    if (!((m >> l) & 1ull)) return s;
    const int j = F.j0[r >> 6] + __popcll(m & ((1ull << l) - 1ull));
    const int e0 = F.rp[j], e1 = F.rp[j + 1];
    const double t = F.fma_chain ? remote_sum<true>(F, e0, e1) : remote_sum<false>(F, e0, e1);
    return s + t;
}

// The remote part of one packed tile (RemoteFuse tj/te), loaded by the
// whole block beside the tile's own loads: entries [ea, ea + ne) of the
// compressed remote rows [ja, ja + nj), up to NQ per thread, each product
// rounded as soon as its x value is in; the storing lane of each row keeps
// its row group's mask word and first compressed row.
struct RemoteTile {
    static constexpr int NQ = kTileRemoteCap / kBlock;
    int ja, nj, ea, ne;
    int32_t qc[NQ];
    double qa[NQ], qp[NQ];
    int32_t qr;   // rp[ja + tid] - ea, tid < nj
    uint64_t m;
    int32_t j0;
};

template <int SL>
__device__ __forceinline__ void rtile_load(const RemoteFuse &F, int t, int r0, int nr,
                                           RemoteTile &R)
{
    const int tid = int(threadIdx.x);
    R.ja = F.tj[t];
    R.nj = F.tj[t + 1] - R.ja;
    R.ea = F.te[t];
    R.ne = F.te[t + 1] - R.ea;
    R.qr = 0;
    R.m = 0;
    R.j0 = 0;
    if (R.nj == 0) return;   // block-uniform: no remote rows in this tile
#pragma unroll
    for (int u = 0; u < R.NQ; ++u) {
        const int k = u * kBlock + tid;
        const bool in = k < R.ne;
        R.qc[u] = in ? F.col[R.ea + k] : 0;
        R.qa[u] = in ? F.val[R.ea + k] : 0.0;
    }
    if (tid < R.nj) R.qr = F.rp[R.ja + tid] - R.ea;
    const int g = tid / SL;
    if (tid % SL == SL - 1 && g < nr) {
        R.m = F.mask[(r0 + g) >> 6];
        R.j0 = F.j0[(r0 + g) >> 6];
    }
}

__device__ __forceinline__ double product_rn(double a, double b)
{
#pragma clang fp contract(off)
    return a * b;
}

__device__ __forceinline__ void rtile_gather(const RemoteFuse &F, RemoteTile &R)
{
    if (R.nj == 0) return;
    const int tid = int(threadIdx.x);
    double xq[RemoteTile::NQ];
#pragma unroll
    for (int u = 0; u < R.NQ; ++u) xq[u] = u * kBlock + tid < R.ne ? F.xh[R.qc[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < R.NQ; ++u) R.qp[u] = product_rn(R.qa[u], xq[u]);
}

// Operands of one stream-CSR product.  out[r] = row sum (acc == nullptr) or
// acc[rows[r]] += row sum.  nnz_alloc = entries incl. padding, n_x = |x|.
// With 16-bit columns (C16), col holds int16 offsets of each entry's column
// from the first row of its tile.
struct StreamArgs {
    const int32_t *tile_row, *tile_k, *rp, *col, *rows;
    const double *val, *x;
    double *out, *acc;
    uint32_t nnz_alloc, n_x;
};

// Registers of one short-row tile between its stages: window entries,
// gathered x values, row pointers, and the tile's bounds.
template <int NPT, int VW>
struct TileRegs {
    static constexpr int NV = NPT / VW;
    int32_t c[NV][VW];
    double a[NV][VW];
    double xv[NV][VW];
    int32_t rp_a, rp_b;
    int r0, nr, k0, k1, base;
};

// Stage 1: the tile's bounds, its window's columns and values, then its row
// pointers.  The two load groups are independent, so their memory latencies
// overlap (the row pointers wait in registers until the LDS stage).
template <int NPT, int VW, bool C16 = false>
__device__ __forceinline__ void tile_load(const StreamArgs &A, __amdgpu_buffer_rsrc_t r_col,
                                          __amdgpu_buffer_rsrc_t r_val, int t,
                                          TileRegs<NPT, VW> &T)
{
    const int tid = int(threadIdx.x);
    T.r0 = A.tile_row[t];
    T.nr = A.tile_row[t + 1] - T.r0;
    T.k0 = A.tile_k[t];
    T.k1 = A.tile_k[t + 1];
    T.base = T.k0 & ~(VW - 1);
    // columns of the whole window first, then values: the x gathers wait
    // only for the columns
#pragma unroll
    for (int v = 0; v < T.NV; ++v) {
        const int e = T.base + (v * kBlock + tid) * VW;
        if constexpr (C16)
            load_cols16<VW>(r_col, e < T.k1 ? uint32_t(e) : kNoEntry, T.r0, T.c[v]);
        else
            load_cols<VW>(r_col, e < T.k1 ? uint32_t(e) : kNoEntry, T.c[v]);
    }
#pragma unroll
    for (int v = 0; v < T.NV; ++v) {
        const int e = T.base + (v * kBlock + tid) * VW;
        load_vals<VW>(r_val, e < T.k1 ? uint32_t(e) : kNoEntry, T.a[v]);
    }
    // nr + 1 <= kBlock / SL + 1 pointers: one per thread, plus the last one
    // by thread 0 when the tile has kBlock rows
    T.rp_a = tid <= T.nr ? A.rp[T.r0 + tid] : 0;
    T.rp_b = (tid == 0 && T.nr == kBlock) ? A.rp[T.r0 + kBlock] : 0;
}

// Stage 2: gather x for the window's entries (entries outside the tile read
// nothing and give 0).
template <int NPT, int VW>
__device__ __forceinline__ void tile_gather(__amdgpu_buffer_rsrc_t r_x, TileRegs<NPT, VW> &T)
{
    const int tid = int(threadIdx.x);
#pragma unroll
    for (int v = 0; v < T.NV; ++v) {
#pragma unroll
        for (int j = 0; j < VW; ++j) {
            const int k = T.base + (v * kBlock + tid) * VW + j;
            const bool ok = k >= T.k0 && k < T.k1;
            T.xv[v][j] = load_x(r_x, ok ? uint32_t(T.c[v][j]) * 8u : kOff);
        }
    }
}

// Stage 3: products into LDS, row sums by SL lanes per row in a fixed
// order, results stored.  Contains one barrier (three with a remote part
// R, whose products and row pointers then take the place of the local
// ones in LDS: s_p must hold its ne <= kBlock * NPT entries); the caller
// separates consecutive tiles with another (LDS is reused).
template <int NPT, int VW, int SL, bool COOP = false>
__device__ __forceinline__ void tile_reduce(const StreamArgs &A, const TileRegs<NPT, VW> &T,
                                            double *s_p, int32_t *s_rp,
                                            const RemoteFuse *F = nullptr,
                                            const RemoteTile *R = nullptr)
{
    const int tid = int(threadIdx.x);
#pragma unroll
    for (int v = 0; v < T.NV; ++v)
#pragma unroll
        for (int j = 0; j < VW; ++j) s_p[(v * kBlock + tid) * VW + j] = T.a[v][j] * T.xv[v][j];
    if (tid <= T.nr) s_rp[tid] = T.rp_a;
    if (tid == 0 && T.nr == kBlock) s_rp[kBlock] = T.rp_b;
    __syncthreads();

    const int g = tid / SL, lane = tid % SL;
    double s = 0.0;
    if (g < T.nr) {
        // left-to-right sum of the row's products owned by this lane; four
        // LDS reads are issued together, the additions keep their order
        const int b = s_rp[g] - T.base, e = s_rp[g + 1] - T.base;
        int k = b + lane;
        for (; k + 3 * SL < e; k += 4 * SL) {
            const double p0 = s_p[k], p1 = s_p[k + SL], p2 = s_p[k + 2 * SL], p3 = s_p[k + 3 * SL];
            s += p0;
            s += p1;
            s += p2;
            s += p3;
        }
        for (; k < e; k += SL) s += s_p[k];
    }
    s = group_sum<SL>(s);
    if constexpr (COOP) {
        if (R->nj > 0) {   // block-uniform
            __syncthreads();   // every row has read s_p and s_rp
#pragma unroll
            for (int u = 0; u < R->NQ; ++u) {
                const int k = u * kBlock + tid;
                if (k < R->ne) s_p[k] = R->qp[u];
            }
            if (tid < R->nj) s_rp[tid] = R->qr;
            if (tid == 0) s_rp[R->nj] = R->ne;
            __syncthreads();
            const int l = (T.r0 + g) & 63;
            if (lane == SL - 1 && g < T.nr && ((R->m >> l) & 1ull)) {
                // y_R's sum of the row: rounded products, left to right from 0
                const int jr = R->j0 + __popcll(R->m & ((1ull << l) - 1ull)) - R->ja;
                const int qb = s_rp[jr], qe = s_rp[jr + 1];
                double q = 0.0;
                for (int k = qb; k < qe; ++k) q += s_p[k];
                s = s + q;
            }
        }
    } else {
        if (lane == SL - 1 && g < T.nr && F && F->mask) s = remote_add(*F, T.r0 + g, s);
    }
    if (lane == SL - 1 && g < T.nr) {
        if (A.acc)
            A.acc[A.rows[T.r0 + g]] += s;
        else
            A.out[T.r0 + g] = s;
    }
}

// One row longer than the window (a tile of its own): per-thread fma
// chains over all windows, then a fixed-order reduction over the block.
// s_p needs kBlock / 64 doubles.
template <int NPT, int VW, bool C16 = false>
__device__ __forceinline__ void long_row_tile(const StreamArgs &A, __amdgpu_buffer_rsrc_t r_col,
                                              __amdgpu_buffer_rsrc_t r_val,
                                              __amdgpu_buffer_rsrc_t r_x, int r0, int k0, int k1,
                                              double *s_p, const RemoteFuse *F = nullptr)
{
    constexpr int CAP = kBlock * NPT;
    constexpr int NV = NPT / VW;
    const int base = k0 & ~(VW - 1);
    const int tid = int(threadIdx.x);
    double s = 0.0;
    for (int w0 = base; w0 < k1; w0 += CAP) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = w0 + (v * kBlock + tid) * VW;
            int32_t c[VW];
            double a[VW];
            if constexpr (C16) {
                load_cols16<VW>(r_col, e < k1 ? uint32_t(e) : kNoEntry, r0, c);
                load_vals<VW>(r_val, e < k1 ? uint32_t(e) : kNoEntry, a);
            } else {
                load_vec<VW>(r_col, r_val, e < k1 ? uint32_t(e) : kNoEntry, c, a);
            }
#pragma unroll
            for (int j = 0; j < VW; ++j) {
                const bool ok = e + j >= k0 && e + j < k1;
                const double xv = load_x(r_x, ok ? uint32_t(c[j]) * 8u : kOff);
                const double f = fma(a[j], xv, s);
                s = ok ? f : s;
            }
        }
    }
    s = group_sum<64>(s);
    if ((tid & 63) == 63) s_p[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        double tot = (s_p[0] + s_p[1]) + (s_p[2] + s_p[3]);
        if (F && F->mask) tot = remote_add(*F, r0, tot);
        if (A.acc)
            A.acc[A.rows[r0]] += tot;
        else
            A.out[r0] = tot;
    }
}

// One tile.  s_p: LDS[kBlock * NPT] doubles, s_rp: LDS[kBlock / SL + 1] ints.
// Block-uniform control flow; the caller separates consecutive tiles with a
// barrier (LDS is reused).  COOP: F has tj/te, and the tile's remote part
// is loaded by the block (RemoteTile).
template <int NPT, int VW, int SL, bool C16 = false, bool COOP = false>
__device__ __forceinline__ void stream_tile(const StreamArgs &A, int t, double *s_p, int32_t *s_rp,
                                            const RemoteFuse *F = nullptr)
{
    constexpr int CAP = kBlock * NPT;
    static_assert(NPT % VW == 0, "NPT must be a multiple of VW");
    const auto r_col = rsrc(A.col, A.nnz_alloc * (C16 ? 2u : 4u));
    const auto r_val = rsrc(A.val, A.nnz_alloc * 8u);
    const auto r_x = rsrc(A.x, A.n_x * 8u);
    const int r0 = A.tile_row[t], r1 = A.tile_row[t + 1];
    const int k0 = A.tile_k[t], k1 = A.tile_k[t + 1];
    const int base = k0 & ~(VW - 1);

    if (r1 - r0 == 1 && k1 - base > CAP) {
        long_row_tile<NPT, VW, C16>(A, r_col, r_val, r_x, r0, k0, k1, s_p, F);
        return;
    }

    TileRegs<NPT, VW> T;
    tile_load<NPT, VW, C16>(A, r_col, r_val, t, T);
    if constexpr (COOP) {
        RemoteTile R;
        rtile_load<SL>(*F, t, T.r0, T.nr, R);
        tile_gather<NPT, VW>(r_x, T);
        rtile_gather(*F, R);
        tile_reduce<NPT, VW, SL, true>(A, T, s_p, s_rp, F, &R);
    } else {
        tile_gather<NPT, VW>(r_x, T);
        tile_reduce<NPT, VW, SL>(A, T, s_p, s_rp, F);
    }
}

// Wide tile: up to RPT * kBlock short rows whose entries fit one window of
// kBlock * NPT entries, each row summed left to right by one thread (thread
// t takes rows t, t + kBlock, ...), so a tile of rows with one or two
// entries still fills its window and every thread keeps NPT gathers in
// flight.  A row's sum is the same as with one summing lane in a tile of
// kBlock rows.  s_p: LDS[kBlock * NPT] doubles, s_rp: LDS[RPT * kBlock + 1]
// ints.  Stores out[r0 + g] (acc is not used).
template <int NPT, int VW, int RPT>
__device__ __forceinline__ void wide_tile(const StreamArgs &A, int t, double *s_p, int32_t *s_rp)
{
    constexpr int CAP = kBlock * NPT;
    constexpr int NV = NPT / VW;
    static_assert(NPT % VW == 0, "NPT must be a multiple of VW");
    const auto r_col = rsrc(A.col, A.nnz_alloc * 4u);
    const auto r_val = rsrc(A.val, A.nnz_alloc * 8u);
    const auto r_x = rsrc(A.x, A.n_x * 8u);
    const int r0 = A.tile_row[t], nr = A.tile_row[t + 1] - r0;
    const int k0 = A.tile_k[t], k1 = A.tile_k[t + 1];
    const int base = k0 & ~(VW - 1);
    const int tid = int(threadIdx.x);

    if (nr == 1 && k1 - base > CAP) {
        long_row_tile<NPT, VW, false>(A, r_col, r_val, r_x, r0, k0, k1, s_p);
        return;
    }

    // columns of the whole window, then values, then the row pointers: the
    // three load groups are independent
    int32_t c[NV][VW];
    double a[NV][VW], xv[NV][VW];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int e = base + (v * kBlock + tid) * VW;
        load_cols<VW>(r_col, e < k1 ? uint32_t(e) : kNoEntry, c[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int e = base + (v * kBlock + tid) * VW;
        load_vals<VW>(r_val, e < k1 ? uint32_t(e) : kNoEntry, a[v]);
    }
    // nr + 1 <= RPT * kBlock + 1 pointers: RPT per thread, plus the last
    // one by thread 0 when the tile is full
    int32_t rp[RPT + 1];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = j * kBlock + tid;
        rp[j] = i <= nr ? A.rp[r0 + i] : 0;
    }
    rp[RPT] = (tid == 0 && nr == RPT * kBlock) ? A.rp[r0 + RPT * kBlock] : 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int j = 0; j < VW; ++j) {
            const int k = base + (v * kBlock + tid) * VW + j;
            const bool ok = k >= k0 && k < k1;
            xv[v][j] = load_x(r_x, ok ? uint32_t(c[v][j]) * 8u : kOff);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int j = 0; j < VW; ++j) s_p[(v * kBlock + tid) * VW + j] = a[v][j] * xv[v][j];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = j * kBlock + tid;
        if (i <= nr) s_rp[i] = rp[j];
    }
    if (tid == 0 && nr == RPT * kBlock) s_rp[RPT * kBlock] = rp[RPT];
    __syncthreads();

#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int g = j * kBlock + tid;
        if (g < nr) {
            const int b = s_rp[g] - base, e = s_rp[g + 1] - base;
            double s = 0.0;
            int k = b;
            for (; k + 3 < e; k += 4) {
                const double p0 = s_p[k], p1 = s_p[k + 1], p2 = s_p[k + 2], p3 = s_p[k + 3];
                s += p0;
                s += p1;
                s += p2;
                s += p3;
            }
            for (; k < e; ++k) s += s_p[k];
            A.out[r0 + g] = s;
        }
    }
}

}  // namespace spmv
