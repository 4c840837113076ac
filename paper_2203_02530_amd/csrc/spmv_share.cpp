// Host side of the rank share: CSR validation, the contiguous row-block
// partition, the A = A_L + A_R split, the halo x_R and the send lists
// (Sec. III-A of the paper).  Runs once per plan: A is static, only the
// values of x change between products.
#include <algorithm>
#include <cstring>

#include "spmv_internal.h"

namespace spmv {

int validate_csr(const spmv_csr_t *csr)
{
    if (!csr) return set_error(SPMV_EINVAL, "csr is NULL");
    if (csr->n_rows < 0 || csr->n_cols < 0 || csr->nnz < 0)
        return set_error(SPMV_EINVAL, "negative CSR size");
    if (csr->n_rows != csr->n_cols)
        return set_error(SPMV_EINVAL, "matrix must be square: rows, x and y share one partition");
    if (csr->nnz >= (int64_t(1) << 31))
        return set_error(SPMV_EINVAL, "nnz does not fit int32 indexing");
    if (!csr->row_ptr) return set_error(SPMV_EINVAL, "row_ptr is NULL");
    if (csr->nnz > 0 && (!csr->col_idx || !csr->val))
        return set_error(SPMV_EINVAL, "col_idx/val is NULL");
    const int32_t *rp = csr->row_ptr;
    if (rp[0] != 0) return set_error(SPMV_ECSR, "row_ptr[0] != 0");
    if (rp[csr->n_rows] != csr->nnz)
        return set_error(SPMV_ECSR, "row_ptr[n_rows] != nnz");
    for (int32_t i = 0; i < csr->n_rows; ++i) {
        if (rp[i + 1] < rp[i])
            return set_error(SPMV_ECSR, "row_ptr decreases at row " + std::to_string(i));
        int32_t prev = -1;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            int32_t c = csr->col_idx[k];
            if (c < 0 || c >= csr->n_cols)
                return set_error(SPMV_ECSR, "column out of range in row " + std::to_string(i));
            if (c <= prev)
                return set_error(SPMV_ECSR, "columns not strictly ascending in row " +
                                                std::to_string(i));
            prev = c;
        }
    }
    return SPMV_OK;
}

// Rank q owns rows [block_lo(q), block_lo(q+1)): the rows are divided evenly,
// and when P does not divide n the first n mod P ranks take one extra row.
int64_t block_lo(int64_t n, int32_t P, int32_t q)
{
    return int64_t(q) * (n / P) + std::min<int64_t>(q, n % P);
}

namespace {

// The rank's own rows: rp[0..nl] indexes col/val (rp[0] may be non-zero when
// the rows sit inside a global matrix).  Splits them into A_L / A_R and
// derives the halo and its owners (Sec. III-A).
void split_rows(const int32_t *rp, const int32_t *ci, const double *va, int64_t nl, int64_t n,
                int32_t P, int64_t lo, int64_t hi, Share &S)
{
    std::vector<uint8_t> remote_mark(size_t(n), 0);
    S.L_ptr.assign(size_t(nl) + 1, 0);
    int64_t nnz_rem = 0;
    for (int64_t i = 0; i < nl; ++i) {
        int32_t cnt = 0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t c = ci[k];
            if (c >= lo && c < hi) {
                ++cnt;
            } else {
                remote_mark[size_t(c)] = 1;
                ++nnz_rem;
            }
        }
        S.L_ptr[size_t(i) + 1] = S.L_ptr[size_t(i)] + cnt;
    }
    const int64_t nnz_loc = S.L_ptr[size_t(nl)];
    S.L_col.resize(size_t(nnz_loc));
    S.L_val.resize(size_t(nnz_loc));

    // Halo in ascending global column order; owners are contiguous blocks,
    // so the halo is grouped by owner rank in ascending order.
    std::vector<int32_t> halo_index(size_t(n), -1);
    for (int64_t c = 0; c < n; ++c)
        if (remote_mark[size_t(c)]) {
            halo_index[size_t(c)] = int32_t(S.halo.size());
            S.halo.push_back(int32_t(c));
        }
    S.recv_off.resize(size_t(P) + 1);
    for (int32_t q = 0; q <= P; ++q)
        S.recv_off[size_t(q)] = int32_t(
            std::lower_bound(S.halo.begin(), S.halo.end(), block_lo(n, P, q)) - S.halo.begin());

    // Fill A_L values and A_R over the rows that touch the halo.
    S.R_ptr.assign(1, 0);
    S.R_col.reserve(size_t(nnz_rem));
    S.R_val.reserve(size_t(nnz_rem));
    for (int64_t i = 0; i < nl; ++i) {
        int32_t w = S.L_ptr[size_t(i)];
        int32_t rcount = 0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t c = ci[k];
            if (c >= lo && c < hi) {
                S.L_col[size_t(w)] = int32_t(c - lo);
                S.L_val[size_t(w)] = va[k];
                ++w;
            } else {
                S.R_col.push_back(halo_index[size_t(c)]);
                S.R_val.push_back(va[k]);
                ++rcount;
            }
        }
        if (rcount) {
            S.R_rows.push_back(int32_t(i));
            S.R_ptr.push_back(S.R_ptr.back() + rcount);
        }
    }
    S.unpack_perm.resize(S.halo.size());
    for (size_t p = 0; p < S.halo.size(); ++p) S.unpack_perm[p] = int32_t(p);
}

void init_share(Share &S, int64_t n, int32_t P, int32_t r)
{
    S = Share();
    S.n_global = n;
    S.lo = block_lo(n, P, r);
    S.n_loc = block_lo(n, P, r + 1) - S.lo;
    S.nranks = P;
    S.rank = r;
}

}  // namespace

int build_share(const spmv_csr_t *csr, int32_t P, int32_t r, Share &S)
{
    if (int rc = validate_csr(csr)) return rc;
    if (P < 1) return set_error(SPMV_EINVAL, "nranks < 1");
    if (r < 0 || r >= P) return set_error(SPMV_EINVAL, "rank out of range");
    const int64_t n = csr->n_rows;
    const int32_t *rp = csr->row_ptr, *ci = csr->col_idx;
    init_share(S, n, P, r);
    const int64_t lo = S.lo, hi = S.lo + S.n_loc, nl = S.n_loc;
    split_rows(rp + lo, ci, csr->val, nl, n, P, lo, hi, S);

    // Send lists: for each other rank q, the owned columns appearing in q's
    // rows, as local indices, ascending.  A stamp per local index avoids
    // clearing a marker between destinations.
    std::vector<int32_t> stamp(size_t(nl), -1);
    S.send_off.assign(size_t(P) + 1, 0);
    for (int32_t q = 0; q < P; ++q) {
        S.send_off[size_t(q) + 1] = S.send_off[size_t(q)];
        if (q == r) continue;
        const int64_t qlo = block_lo(n, P, q), qhi = block_lo(n, P, q + 1);
        int64_t found = 0;
        for (int32_t k = rp[qlo]; k < rp[qhi]; ++k) {
            const int32_t c = ci[k];
            if (c >= lo && c < hi && stamp[size_t(c - lo)] != q) {
                stamp[size_t(c - lo)] = q;
                ++found;
            }
        }
        if (!found) continue;
        const size_t base = S.send_idx.size();
        if (found * 8 < nl) {
            // few entries: collect and sort
            for (int32_t k = rp[qlo]; k < rp[qhi]; ++k) {
                const int32_t c = ci[k];
                if (c >= lo && c < hi && stamp[size_t(c - lo)] == q) {
                    stamp[size_t(c - lo)] = P + q;  // collected
                    S.send_idx.push_back(int32_t(c - lo));
                }
            }
            std::sort(S.send_idx.begin() + long(base), S.send_idx.end());
        } else {
            for (int64_t j = 0; j < nl; ++j)
                if (stamp[size_t(j)] == q) {
                    S.send_idx.push_back(int32_t(j));
                    stamp[size_t(j)] = P + q;
                }
        }
        S.send_off[size_t(q) + 1] = int32_t(S.send_idx.size());
    }
    return SPMV_OK;
}

int build_share_local(const spmv_csr_t *local, int64_t n, int32_t P, int32_t r,
                      const int32_t *send_idx, const int32_t *send_off, Share &S)
{
    if (!local) return set_error(SPMV_EINVAL, "local rows are NULL");
    if (P < 1) return set_error(SPMV_EINVAL, "nranks < 1");
    if (r < 0 || r >= P) return set_error(SPMV_EINVAL, "rank out of range");
    if (n < 0 || n >= (int64_t(1) << 31)) return set_error(SPMV_EINVAL, "n_global out of range");
    if (local->n_cols != n)
        return set_error(SPMV_EINVAL, "local rows must carry global columns (n_cols = n_global)");
    init_share(S, n, P, r);
    if (local->n_rows != S.n_loc)
        return set_error(SPMV_EINVAL, "local rows do not match the rank's row block (" +
                                          std::to_string(S.n_loc) + " rows)");
    // same structural checks as a global matrix, minus squareness
    {
        const int32_t *rp = local->row_ptr;
        if (!rp || rp[0] != 0 || rp[local->n_rows] != local->nnz)
            return set_error(SPMV_ECSR, "local row_ptr malformed");
        for (int32_t i = 0; i < local->n_rows; ++i) {
            if (rp[i + 1] < rp[i]) return set_error(SPMV_ECSR, "row_ptr decreases");
            int32_t prev = -1;
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t c = local->col_idx[k];
                if (c < 0 || c >= n) return set_error(SPMV_ECSR, "column out of range");
                if (c <= prev) return set_error(SPMV_ECSR, "columns not strictly ascending");
                prev = c;
            }
        }
    }
    if (!send_off) return set_error(SPMV_EINVAL, "send_off is NULL");
    if (send_off[0] != 0) return set_error(SPMV_EINVAL, "send_off[0] != 0");
    for (int32_t q = 0; q < P; ++q) {
        if (send_off[q + 1] < send_off[q]) return set_error(SPMV_EINVAL, "send_off decreases");
        if (q == r && send_off[q + 1] != send_off[q])
            return set_error(SPMV_EINVAL, "a rank sends nothing to itself");
        if (send_off[q + 1] > send_off[q] && !send_idx)
            return set_error(SPMV_EINVAL, "send_idx is NULL");
        for (int32_t k = send_off[q]; k < send_off[q + 1]; ++k) {
            if (send_idx[k] < 0 || send_idx[k] >= S.n_loc)
                return set_error(SPMV_EINVAL, "send index out of the rank's rows");
            if (k > send_off[q] && send_idx[k] <= send_idx[k - 1])
                return set_error(SPMV_EINVAL, "send indices must ascend per destination");
        }
    }
    split_rows(local->row_ptr, local->col_idx, local->val, S.n_loc, n, P, S.lo,
               S.lo + S.n_loc, S);
    S.send_off.assign(send_off, send_off + P + 1);
    if (send_off[P] > 0) S.send_idx.assign(send_idx, send_idx + send_off[P]);
    return SPMV_OK;
}

// Tiles of the CSR-stream kernel: consecutive rows, at most `maxr` of them,
// whose entries fit the window [rp[r0] rounded down to vw, + cap); a row
// whose entries alone overflow the window is a tile of its own.
void build_tiles(const std::vector<int32_t> &rp, int64_t n_rows, int cap, int maxr, int vw,
                 std::vector<int32_t> &tile_row, std::vector<int32_t> &tile_k)
{
    tile_row.clear();
    tile_k.clear();
    int64_t r = 0;
    while (r < n_rows) {
        tile_row.push_back(int32_t(r));
        tile_k.push_back(rp[size_t(r)]);
        const int64_t base = rp[size_t(r)] & ~int64_t(vw - 1);
        int64_t e = r + 1;
        if (rp[size_t(e)] - base <= cap)
            while (e < n_rows && e - r < maxr && rp[size_t(e) + 1] - base <= cap) ++e;
        r = e;
    }
    tile_row.push_back(int32_t(n_rows));
    tile_k.push_back(n_rows > 0 ? rp[size_t(n_rows)] : (rp.empty() ? 0 : rp[0]));
}

void build_slabs(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                 const std::vector<double> &val, int64_t n_rows, int64_t n_x, int cap, int maxr,
                 int vw, std::vector<int32_t> &s_rp, std::vector<int32_t> &s_col,
                 std::vector<double> &s_val, std::vector<int32_t> &tile_row,
                 std::vector<int32_t> &tile_k, int64_t *nnz_off, int64_t *tile_off)
{
    const int64_t w = std::max<int64_t>((n_x + kSlabs - 1) / kSlabs, 1);
    s_rp.assign(size_t(kSlabs * (n_rows + 1)), 0);
    s_col.clear();
    s_val.clear();
    tile_row.clear();
    tile_k.clear();
    std::vector<int32_t> rk, tr, tk;
    for (int k = 0; k < kSlabs; ++k) {
        while (s_col.size() % 4) {   // each slab starts 16-byte aligned
            s_col.push_back(0);
            s_val.push_back(0.0);
        }
        nnz_off[k] = int64_t(s_col.size());
        tile_off[k] = int64_t(tile_row.size());
        // a row's entries in slab k are contiguous: its columns ascend
        rk.assign(size_t(n_rows + 1), 0);
        for (int64_t r = 0; r < n_rows; ++r) {
            for (int64_t j = rp[size_t(r)]; j < rp[size_t(r) + 1]; ++j)
                if (col[size_t(j)] / w == k) {
                    s_col.push_back(col[size_t(j)]);
                    s_val.push_back(val[size_t(j)]);
                }
            rk[size_t(r) + 1] = int32_t(int64_t(s_col.size()) - nnz_off[k]);
        }
        std::copy(rk.begin(), rk.end(), s_rp.begin() + k * (n_rows + 1));
        build_tiles(rk, n_rows, cap, maxr, vw, tr, tk);
        tile_row.insert(tile_row.end(), tr.begin(), tr.end());
        tile_k.insert(tile_k.end(), tk.begin(), tk.end());
    }
    nnz_off[kSlabs] = int64_t(s_col.size());
    tile_off[kSlabs] = int64_t(tile_row.size());
}

bool build_sell(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                const std::vector<double> &val, int64_t n_rows, double max_ratio,
                std::vector<int32_t> &ptr, std::vector<int32_t> &scol, std::vector<double> &sval,
                int32_t &max_width, bool &uniform)
{
    ptr.clear();
    scol.clear();
    sval.clear();
    max_width = 0;
    uniform = false;
    const int64_t n_slices = (n_rows + 63) / 64;
    const int64_t nnz = n_rows > 0 ? rp[size_t(n_rows)] : 0;
    std::vector<int64_t> width(size_t(n_slices), 0);
    for (int64_t sl = 0; sl < n_slices; ++sl) {
        for (int64_t r = sl * 64; r < std::min(n_rows, sl * 64 + 64); ++r)
            width[size_t(sl)] = std::max<int64_t>(width[size_t(sl)], rp[size_t(r) + 1] - rp[size_t(r)]);
        max_width = int32_t(std::max<int64_t>(max_width, width[size_t(sl)]));
    }
    const double budget = max_ratio * double(std::max<int64_t>(nnz, 1));
    // one width for every slice (no per-slice offsets to read) when that
    // padding fits too
    uniform = double(64 * max_width) * double(n_slices) <= budget;
    if (uniform) std::fill(width.begin(), width.end(), int64_t(max_width));
    std::vector<int64_t> off(size_t(n_slices) + 1, 0);
    for (int64_t sl = 0; sl < n_slices; ++sl) off[size_t(sl) + 1] = off[size_t(sl)] + 64 * width[size_t(sl)];
    const int64_t total = off[size_t(n_slices)];
    if (double(total) > budget || (total + 64) * 8 >= (int64_t(1) << 32)) {
        uniform = false;
        return false;
    }
    ptr.assign(off.begin(), off.end());
    scol.assign(size_t(total), -1);
    sval.assign(size_t(total), 0.0);
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t sl = r / 64, l = r % 64;
        for (int64_t k = rp[size_t(r)]; k < rp[size_t(r) + 1]; ++k) {
            const int64_t v = k - rp[size_t(r)];
            scol[size_t(off[size_t(sl)] + 64 * v + l)] = col[size_t(k)];
            sval[size_t(off[size_t(sl)] + 64 * v + l)] = val[size_t(k)];
        }
    }
    return true;
}

bool build_sell16(const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                  int64_t n_rows, int32_t width, std::vector<int16_t> &off)
{
    off.clear();
    const int64_t n_slices = (n_rows + 63) / 64, G = (int64_t(width) + 7) / 8;
    const int64_t total = n_slices * G * 512;
    if ((total + 64) * 2 >= (int64_t(1) << 32)) return false;
    off.assign(size_t(total), kPad16);
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t s = r / 64, l = r % 64;
        if (rp[size_t(r) + 1] - rp[size_t(r)] > width) {
            off.clear();
            return false;
        }
        for (int64_t k = rp[size_t(r)]; k < rp[size_t(r) + 1]; ++k) {
            const int64_t v = k - rp[size_t(r)], d = int64_t(col[size_t(k)]) - r;
            if (d <= int64_t(kPad16) || d > 32767) {
                off.clear();
                return false;
            }
            off[size_t(((s * G + v / 8) * 64 + l) * 8 + v % 8)] = int16_t(d);
        }
    }
    return true;
}

void pair_values(std::vector<double> &val, int64_t n_slices, int32_t width)
{
    const int64_t w = width, even = w & ~int64_t(1);
    std::vector<double> out(val.size(), 0.0);
    for (int64_t sl = 0; sl < n_slices; ++sl) {
        const int64_t base = sl * 64 * w;
        for (int64_t v = 0; v < w; ++v)
            for (int64_t l = 0; l < 64; ++l) {
                const int64_t dst = v < even ? base + (v >> 1) * 128 + 2 * l + (v & 1)
                                             : base + (w - 1) * 64 + l;
                out[size_t(dst)] = val[size_t(base + v * 64 + l)];
            }
    }
    val.swap(out);
}

bool build_tile16(const std::vector<int32_t> &col, const std::vector<int32_t> &tile_row,
                  const std::vector<int32_t> &tile_k, std::vector<int16_t> &off)
{
    off.assign(col.size(), 0);
    for (size_t t = 0; t + 1 < tile_row.size(); ++t) {
        for (int64_t k = tile_k[t]; k < tile_k[t + 1]; ++k) {
            const int64_t d = int64_t(col[size_t(k)]) - tile_row[t];
            if (d < -32767 || d > 32767) {
                off.clear();
                return false;
            }
            off[size_t(k)] = int16_t(d);
        }
    }
    return true;
}

}  // namespace spmv
