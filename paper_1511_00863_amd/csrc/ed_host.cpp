// Host side of the library: per-spin basis and ranking, hopping tables in ELL
// form, the device table packer, and the tridiagonal eigensolver.
//
// Basis and ELL: Sec. 2.1 and Fig. 2.  Tridiagonal T: Sec. 2.2.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <set>
#include <string>
#include <utility>
#include <tuple>
#include <vector>

#include "../../include/ed.h"
#include "ed_internal.h"

namespace ed {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

struct BinomTable {
    uint64_t c[65][66];
    BinomTable() {
        std::memset(c, 0, sizeof c);
        for (int n = 0; n <= 64; ++n) {
            c[n][0] = 1;
            for (int k = 1; k <= n; ++k) c[n][k] = c[n - 1][k - 1] + (k <= n - 1 ? c[n - 1][k] : 0);
        }
    }
};
static const BinomTable g_binom;

uint64_t binom(int n, int k) {
    if (n < 0 || n > 64 || k < 0 || k > n) return 0;
    return g_binom.c[n][k];
}

// Colex rank of a bitmask with set bits p_0 < p_1 < ...: sum_k C(p_k, k+1).
static inline int64_t colex_rank(uint64_t s) {
    int64_t r = 0;
    int k = 0;
    while (s) {
        int p = __builtin_ctzll(s);
        r += (int64_t)g_binom.c[p][k + 1];
        ++k;
        s &= s - 1;
    }
    return r;
}

// Number of negative pivots of T - x I (= eigenvalues below x).
static int sturm_count(const double *a, const double *b2, int m, double x, double pivmin) {
    int cnt = 0;
    double d = a[0] - x;
    if (std::fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
    for (int k = 1; k < m; ++k) {
        d = (a[k] - x) - b2[k - 1] / d;
        if (std::fabs(d) < pivmin) d = -pivmin;
        if (d < 0) ++cnt;
    }
    return cnt;
}

double tridiag_lowest(const double *a, const double *b, int m) {
    if (m == 1) return a[0];
    std::vector<double> b2(m - 1);
    double lo = INFINITY, hi = -INFINITY, bmax2 = 0.0;
    for (int k = 0; k < m; ++k) {
        double r = (k > 0 ? std::fabs(b[k - 1]) : 0.0) + (k < m - 1 ? std::fabs(b[k]) : 0.0);
        lo = std::min(lo, a[k] - r);
        hi = std::max(hi, a[k] + r);
        if (k < m - 1) {
            b2[k] = b[k] * b[k];
            bmax2 = std::max(bmax2, b2[k]);
        }
    }
    const double eps = std::ldexp(1.0, -53);
    const double pivmin = std::max(std::numeric_limits<double>::min() * std::max(1.0, bmax2), 1e-300);
    double scale = std::max(std::fabs(lo), std::fabs(hi));
    lo -= 2.0 * eps * scale + pivmin;
    hi += 2.0 * eps * scale + pivmin;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b2.data(), m, mid, pivmin) >= 1) hi = mid; else lo = mid;
        if (hi - lo <= 2.0 * eps * std::max(std::fabs(lo), std::fabs(hi))) break;
    }
    return 0.5 * (lo + hi);
}

constexpr int kComplexMaxAmps = 64;                 // distinct values of a complex table (6-bit index)
constexpr int kComplexMaxDim = (1 << 26) - 1;       // columns in 26 bits; the largest entry stays below padding

// The two device table formats differ only in the entry type.
template <typename E>
static int pack_tables_impl(const char *who, const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                     int32_t width, int layout, int64_t max_dim, E *packed) {
    if (!cols || !vals || !nnz || !packed || dim < 1 || width < 0)
        return set_error(ED_EINVAL, "%s: bad arguments", who);
    if (dim > max_dim) return set_error(ED_EOVERFLOW, "%s: dim %lld > %lld", who, (long long)dim, (long long)max_dim);
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR) return set_error(ED_EINVAL, "%s: bad layout %d", who, layout);
    const int64_t stride = (width + 7) & ~7;
    const E pad = static_cast<E>(~E(0));
    for (int64_t r = 0; r < dim; ++r) {
        if (nnz[r] < 0 || nnz[r] > width)
            return set_error(ED_EINVAL, "%s: nnz[%lld] = %d out of range", who, (long long)r, nnz[r]);
        int64_t last = -1;
        for (int64_t k = 0; k < stride; ++k) {
            E e = pad;
            if (k < nnz[r]) {
                int64_t at = layout == ED_ROW_MAJOR ? r * width + k : k * dim + r;
                if (cols[at] < 0 || cols[at] >= dim) return set_error(ED_EINVAL, "%s: column %d out of range", who, cols[at]);
                if (cols[at] <= last)
                    return set_error(ED_EINVAL, "%s: row %lld not in ascending column order", who, (long long)r);
                if (vals[at] != 1.0 && vals[at] != -1.0) return set_error(ED_EINVAL, "%s: value %g is not +-1", who, vals[at]);
                last = cols[at];
                e = static_cast<E>(((uint64_t)cols[at] << 1) | (vals[at] < 0 ? 1u : 0u));
            }
            packed[r * stride + k] = e;                                   // row-major part
            packed[dim * stride + ((k >> 3) * dim + r) * 8 + (k & 7)] = e;  // 8-interleaved part
        }
    }
    return ED_OK;
}

}  // namespace ed

using namespace ed;

extern "C" {

const char *ed_last_error(void) { return g_last_error.c_str(); }

const char *ed_version(void) { return "ed-mi355x 0.1 (gfx950)"; }

int ed_build_basis(int n_sites, int n_part, uint64_t *states, int64_t cap, int64_t *dim) {
    clear_error();
    if (!dim) return set_error(ED_EINVAL, "ed_build_basis: dim is NULL");
    if (n_sites > 64) return set_error(ED_EOVERFLOW, "ed_build_basis: n_sites=%d > 64", n_sites);
    if (n_sites < 1 || n_part < 0 || n_part > n_sites)
        return set_error(ED_EINVAL, "ed_build_basis: need 0 <= n_part (%d) <= n_sites (%d), n_sites >= 1",
                         n_part, n_sites);
    uint64_t d = binom(n_sites, n_part);
    if (d > 0x7fffffffULL) return set_error(ED_EOVERFLOW, "ed_build_basis: dim %llu > 2^31-1",
                                            (unsigned long long)d);
    *dim = (int64_t)d;
    if (states == nullptr && cap == 0) return ED_OK;
    if (!states) return set_error(ED_EINVAL, "ed_build_basis: states is NULL");
    if (cap < (int64_t)d) return set_error(ED_ECAPACITY, "ed_build_basis: cap %lld < dim %llu",
                                           (long long)cap, (unsigned long long)d);
    // Ascending integers with n_part set bits (next-larger-same-popcount step).
    uint64_t s = n_part == 0 ? 0ULL : (n_part == 64 ? ~0ULL : ((1ULL << n_part) - 1ULL));
    for (uint64_t k = 0; k < d; ++k) {
        states[k] = s;
        if (n_part == 0 || k + 1 == d) break;
        uint64_t c = s & (~s + 1ULL);
        uint64_t r = s + c;
        s = (((r ^ s) >> 2) / c) | r;
    }
    return ED_OK;
}

int ed_state_rank(int n_sites, int n_part, const uint64_t *states, int64_t n, int64_t *ranks) {
    clear_error();
    if (n_sites < 1 || n_sites > 64 || n_part < 0 || n_part > n_sites)
        return set_error(ED_EINVAL, "ed_state_rank: bad n_sites/n_part");
    if (n < 0 || (n > 0 && (!states || !ranks))) return set_error(ED_EINVAL, "ed_state_rank: bad buffers");
    const uint64_t allowed = n_sites == 64 ? ~0ULL : ((1ULL << n_sites) - 1ULL);
    for (int64_t k = 0; k < n; ++k) {
        uint64_t s = states[k];
        if ((s & ~allowed) || __builtin_popcountll(s) != n_part)
            return set_error(ED_EINVAL, "ed_state_rank: state %lld (0x%llx) not in the basis",
                             (long long)k, (unsigned long long)s);
        ranks[k] = colex_rank(s);
    }
    return ED_OK;
}

// One species' hopping rows (real values -sign, or with amps the complex amplitude of the term that
// connects the row state to the column state times the sign); vals has 1 or 2 doubles per entry.
static int build_hopping_impl(int n_sites, const int32_t *bonds, int n_bonds, const double *amps,
                              const uint64_t *states, int64_t dim, int layout, int32_t cap_width, int32_t *cols,
                              double *vals, int32_t *nnz, int32_t *width) {
    if (!width) return set_error(ED_EINVAL, "ed_build_hopping: width is NULL");
    if (n_sites < 1 || n_sites > 64) return set_error(ED_EINVAL, "ed_build_hopping: n_sites=%d", n_sites);
    if (n_bonds < 0 || (n_bonds > 0 && !bonds)) return set_error(ED_EINVAL, "ed_build_hopping: bad bonds");
    if (dim < 1 || !states) return set_error(ED_EINVAL, "ed_build_hopping: bad states/dim");
    if (dim > 0x3fffffffLL) return set_error(ED_EOVERFLOW, "ed_build_hopping: dim too large");
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR)
        return set_error(ED_EINVAL, "ed_build_hopping: bad layout %d", layout);
    std::set<std::pair<int, int>> seen;
    std::vector<uint64_t> bmask(n_bonds), between(n_bonds);
    for (int k = 0; k < n_bonds; ++k) {
        int i = bonds[2 * k], j = bonds[2 * k + 1];
        if (i < 0 || j < 0 || i >= n_sites || j >= n_sites || i == j)
            return set_error(ED_EINVAL, "ed_build_hopping: bond %d = (%d, %d) invalid", k, i, j);
        int lo = std::min(i, j), hi = std::max(i, j);
        if (!seen.insert({lo, hi}).second)
            return set_error(ED_EINVAL, "ed_build_hopping: duplicate bond (%d, %d)", lo, hi);
        bmask[k] = (1ULL << lo) | (1ULL << hi);
        // sites strictly between lo and hi
        uint64_t below_hi = (1ULL << hi) - 1ULL;
        uint64_t upto_lo = (lo == 63) ? ~0ULL : ((1ULL << (lo + 1)) - 1ULL);
        between[k] = below_hi & ~upto_lo;
    }
    const int popc = __builtin_popcountll(states[0]);
    // first pass: width and validation
    int32_t w = 0;
    for (int64_t r = 0; r < dim; ++r) {
        uint64_t s = states[r];
        if (__builtin_popcountll(s) != popc || (n_sites < 64 && (s >> n_sites)))
            return set_error(ED_EINVAL, "ed_build_hopping: state %lld not in a fixed-N basis", (long long)r);
        if (r > 0 && states[r] <= states[r - 1])
            return set_error(ED_EINVAL, "ed_build_hopping: states not strictly ascending at %lld", (long long)r);
        int c = 0;
        for (int k = 0; k < n_bonds; ++k) {
            uint64_t m = s & bmask[k];
            if (m && m != bmask[k]) ++c;
        }
        w = std::max(w, c);
    }
    if ((int64_t)binom(n_sites, popc) != dim)
        return set_error(ED_EINVAL, "ed_build_hopping: dim %lld is not C(%d,%d)", (long long)dim, n_sites, popc);
    *width = w;
    if (cols == nullptr && vals == nullptr && nnz == nullptr && cap_width == 0) return ED_OK;
    if (!cols || !vals || !nnz) return set_error(ED_EINVAL, "ed_build_hopping: NULL output buffer");
    if (cap_width < w) return set_error(ED_ECAPACITY, "ed_build_hopping: cap_width %d < width %d", cap_width, w);
    // (column, value re, value im) of each nonzero of a row
    std::vector<std::tuple<int32_t, double, double>> row;
    row.reserve(n_bonds);
    const int64_t W = cap_width;
    const int nv = amps ? 2 : 1;
    for (int64_t r = 0; r < dim; ++r) {
        uint64_t s = states[r];
        row.clear();
        for (int k = 0; k < n_bonds; ++k) {
            uint64_t m = s & bmask[k];
            if (!m || m == bmask[k]) continue;      // both empty or both occupied: no hop
            uint64_t t = s ^ bmask[k];
            int sign = (__builtin_popcountll(s & between[k]) & 1) ? -1 : 1;
            double re = -1.0, im = 0.0;
            if (amps) {
                // term a c+_i c_j + conj(a) c+_j c_i of bond (i, j): the row state holds the particle at i
                // for a (it came from j), at j for conj(a)
                const int i = bonds[2 * k];
                re = amps[2 * k];
                im = ((s >> i) & 1ULL) ? amps[2 * k + 1] : -amps[2 * k + 1];
            }
            row.emplace_back((int32_t)colex_rank(t), re * sign, im * sign);
        }
        std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return std::get<0>(a) < std::get<0>(b); });
        nnz[r] = (int32_t)row.size();
        for (int64_t k = 0; k < W; ++k) {
            const bool live = k < (int64_t)row.size();
            int64_t at = layout == ED_ROW_MAJOR ? r * W + k : k * dim + r;
            cols[at] = live ? std::get<0>(row[k]) : 0;
            vals[nv * at] = live ? std::get<1>(row[k]) : 0.0;
            if (amps) vals[nv * at + 1] = live ? std::get<2>(row[k]) : 0.0;
        }
    }
    return ED_OK;
}

int ed_build_hopping(int n_sites, const int32_t *bonds, int n_bonds, const uint64_t *states,
                     int64_t dim, int layout, int32_t cap_width, int32_t *cols, double *vals,
                     int32_t *nnz, int32_t *width) {
    clear_error();
    return build_hopping_impl(n_sites, bonds, n_bonds, nullptr, states, dim, layout, cap_width, cols, vals, nnz,
                              width);
}

int ed_build_hopping_complex(int n_sites, const int32_t *bonds, int n_bonds, const double *amps,
                             const uint64_t *states, int64_t dim, int layout, int32_t cap_width, int32_t *cols,
                             double *vals, int32_t *nnz, int32_t *width) {
    clear_error();
    if (n_bonds > 0 && !amps) return set_error(ED_EINVAL, "ed_build_hopping_complex: amps is NULL");
    for (int k = 0; k < 2 * n_bonds; ++k)
        if (!std::isfinite(amps[k])) return set_error(ED_EINVAL, "ed_build_hopping_complex: non-finite amplitude");
    return build_hopping_impl(n_sites, bonds, n_bonds, amps, states, dim, layout, cap_width, cols, vals, nnz,
                              width);
}

int ed_pack_tables(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                   int32_t width, int layout, uint16_t *packed) {
    clear_error();
    return pack_tables_impl<uint16_t>("ed_pack_tables", cols, vals, nnz, dim, width, layout, 32767, packed);
}

int ed_pack_tables32(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                     int32_t width, int layout, uint32_t *packed) {
    clear_error();
    return pack_tables_impl<uint32_t>("ed_pack_tables32", cols, vals, nnz, dim, width, layout, int64_t(1) << 30,
                                      packed);
}

int ed_pack_tables_complex(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                           int32_t width, int layout, uint32_t *packed, double *amps, int32_t *n_amps) {
    clear_error();
    const char *who = "ed_pack_tables_complex";
    if (!cols || !vals || !nnz || !packed || !amps || !n_amps || dim < 1 || width < 0)
        return set_error(ED_EINVAL, "%s: bad arguments", who);
    if (dim > kComplexMaxDim) return set_error(ED_EOVERFLOW, "%s: dim %lld > %d", who, (long long)dim, kComplexMaxDim);
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR) return set_error(ED_EINVAL, "%s: bad layout %d", who, layout);
    const int64_t stride = (width + 7) & ~7;
    int n = 0;
    for (int64_t r = 0; r < dim; ++r) {
        if (nnz[r] < 0 || nnz[r] > width)
            return set_error(ED_EINVAL, "%s: nnz[%lld] = %d out of range", who, (long long)r, nnz[r]);
        int64_t last = -1;
        for (int64_t k = 0; k < stride; ++k) {
            uint32_t e = 0xFFFFFFFFu;
            if (k < nnz[r]) {
                const int64_t at = layout == ED_ROW_MAJOR ? r * width + k : k * dim + r;
                const int32_t c = cols[at];
                if (c < 0 || c >= dim) return set_error(ED_EINVAL, "%s: column %d out of range", who, c);
                if (c <= last) return set_error(ED_EINVAL, "%s: row %lld not in ascending column order", who, (long long)r);
                last = c;
                const double re = vals[2 * at], im = vals[2 * at + 1];
                if (!std::isfinite(re) || !std::isfinite(im)) return set_error(ED_EINVAL, "%s: non-finite value", who);
                int idx = 0;
                while (idx < n && !(amps[2 * idx] == re && amps[2 * idx + 1] == im)) ++idx;
                if (idx == n) {
                    if (n == kComplexMaxAmps)
                        return set_error(ED_EOVERFLOW, "%s: more than %d distinct values", who, kComplexMaxAmps);
                    amps[2 * n] = re;
                    amps[2 * n + 1] = im;
                    ++n;
                }
                e = ((uint32_t)c << 6) | (uint32_t)idx;
            }
            packed[r * stride + k] = e;                                   // row-major part
            packed[dim * stride + ((k >> 3) * dim + r) * 8 + (k & 7)] = e;  // 8-interleaved part
        }
    }
    *n_amps = n;
    return ED_OK;
}

int ed_hop_order(const int32_t *nnz, int64_t dim, int64_t *perm) {
    clear_error();
    if (!nnz || !perm || dim < 1) return set_error(ED_EINVAL, "ed_hop_order: bad arguments");
    int32_t most = 0;
    for (int64_t r = 0; r < dim; ++r) {
        if (nnz[r] < 0) return set_error(ED_EINVAL, "ed_hop_order: nnz[%lld] = %d", (long long)r, nnz[r]);
        most = std::max(most, nnz[r]);
    }
    // counting sort on (most - nnz): more hops first, ascending index among equals
    std::vector<int64_t> at(most + 2, 0);
    for (int64_t r = 0; r < dim; ++r) ++at[most - nnz[r] + 1];
    for (int32_t b = 1; b <= most + 1; ++b) at[b] += at[b - 1];
    for (int64_t r = 0; r < dim; ++r) perm[at[most - nnz[r]]++] = r;
    return ED_OK;
}

int ed_wave_chunks(const int32_t *nnz, int64_t dim, uint32_t *out) {
    clear_error();
    if (!nnz || !out || dim < 1) return set_error(ED_EINVAL, "ed_wave_chunks: bad arguments");
    for (int64_t g = 0; g * 64 < dim; ++g) {
        uint32_t most = 0;
        for (int64_t r = g * 64; r < std::min(dim, g * 64 + 64); ++r) {
            if (nnz[r] < 0) return set_error(ED_EINVAL, "ed_wave_chunks: nnz[%lld] = %d", (long long)r, nnz[r]);
            most = std::max(most, (uint32_t)(nnz[r] + 7) / 8);
        }
        out[g] = most;
    }
    return ED_OK;
}

int ed_pack_tables_windowed(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim, int32_t width,
                            int layout, int32_t block_cols, const int32_t *lo_hi, uint16_t *packed) {
    clear_error();
    const char *who = "ed_pack_tables_windowed";
    if (!cols || !vals || !nnz || !lo_hi || !packed || dim < 1 || width < 0 || block_cols <= 0 || (block_cols & 63))
        return set_error(ED_EINVAL, "%s: bad arguments", who);
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR) return set_error(ED_EINVAL, "%s: bad layout %d", who, layout);
    const int64_t stride = (width + 7) & ~7;
    const uint16_t pad = 0xFFFFu;
    for (int64_t r = 0; r < dim; ++r) {
        if (nnz[r] < 0 || nnz[r] > width)
            return set_error(ED_EINVAL, "%s: nnz[%lld] = %d out of range", who, (long long)r, nnz[r]);
        const int64_t b = r / block_cols;
        const int64_t lo = lo_hi[2 * b], hi = lo_hi[2 * b + 1];
        if (lo < 0 || lo > r || hi <= r || hi > dim || hi - lo > 32767)
            return set_error(ED_EINVAL, "%s: window %lld [%lld, %lld) does not hold row %lld in 15 bits", who,
                             (long long)b, (long long)lo, (long long)hi, (long long)r);
        for (int64_t k = 0; k < stride; ++k) {
            uint16_t e = pad;
            if (k < nnz[r]) {
                const int64_t at = layout == ED_ROW_MAJOR ? r * width + k : k * dim + r;
                const int64_t c = cols[at];
                if (c < lo || c >= hi)
                    return set_error(ED_EINVAL, "%s: column %lld of row %lld outside its window", who, (long long)c,
                                     (long long)r);
                if (vals[at] != 1.0 && vals[at] != -1.0) return set_error(ED_EINVAL, "%s: value %g is not +-1", who, vals[at]);
                e = static_cast<uint16_t>(((uint32_t)(c - lo) << 1) | (vals[at] < 0 ? 1u : 0u));
            }
            packed[r * stride + k] = pad;                                   // row-major part: unused
            packed[dim * stride + ((k >> 3) * dim + r) * 8 + (k & 7)] = e;  // 8-interleaved part
        }
    }
    return ED_OK;
}

int ed_row_windows(const int32_t *cols, const int32_t *nnz, int64_t dim, int32_t width, int layout,
                   int32_t block_cols, int32_t *lo_hi, int32_t *max_window) {
    clear_error();
    const char *who = "ed_row_windows";
    if (!nnz || !lo_hi || !max_window || dim < 1 || width < 0 || (width > 0 && !cols) || block_cols <= 0 ||
        (block_cols & 63))
        return set_error(ED_EINVAL, "%s: bad arguments", who);
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR) return set_error(ED_EINVAL, "%s: bad layout %d", who, layout);
    if (dim > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "%s: dim too large", who);
    const int64_t nblk = (dim + block_cols - 1) / block_cols;
    int64_t widest = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t c0 = b * block_cols, c1 = std::min<int64_t>(dim, c0 + block_cols);
        int64_t lo = c0, hi = c1;
        for (int64_t r = c0; r < c1; ++r) {
            if (nnz[r] < 0 || nnz[r] > width) return set_error(ED_EINVAL, "%s: nnz[%lld] = %d", who, (long long)r, nnz[r]);
            for (int k = 0; k < nnz[r]; ++k) {
                const int64_t c = layout == ED_ROW_MAJOR ? cols[r * width + k] : cols[(int64_t)k * dim + r];
                if (c < 0 || c >= dim)
                    return set_error(ED_EINVAL, "%s: column %lld of row %lld out of range", who, (long long)c, (long long)r);
                lo = std::min(lo, c);
                hi = std::max(hi, c + 1);
            }
        }
        lo &= ~int64_t(3);
        hi = std::min<int64_t>(dim, (hi + 3) & ~int64_t(3));
        lo_hi[2 * b] = (int32_t)lo;
        lo_hi[2 * b + 1] = (int32_t)hi;
        widest = std::max(widest, hi - lo);
    }
    *max_window = (int32_t)widest;
    return ED_OK;
}

int ed_band_order(const int32_t *cols, const int32_t *nnz, int64_t dim, int32_t width, int layout, int64_t *perm) {
    clear_error();
    const char *who = "ed_band_order";
    if (!nnz || !perm || dim < 1 || width < 0 || (width > 0 && !cols)) return set_error(ED_EINVAL, "%s: bad arguments", who);
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR) return set_error(ED_EINVAL, "%s: bad layout %d", who, layout);
    if (dim > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "%s: dim too large", who);
    const int n = (int)dim;
    // adjacency as compressed rows (the hopping graph is symmetric: a column of row r is a neighbour of r)
    std::vector<int64_t> start(n + 1, 0);
    for (int r = 0; r < n; ++r) {
        if (nnz[r] < 0 || nnz[r] > width) return set_error(ED_EINVAL, "%s: nnz[%d] = %d", who, r, nnz[r]);
        start[r + 1] = start[r] + nnz[r];
    }
    std::vector<int> adj(start[n]);
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < nnz[r]; ++k) {
            const int c = layout == ED_ROW_MAJOR ? cols[(int64_t)r * width + k] : cols[(int64_t)k * dim + r];
            if (c < 0 || c >= n) return set_error(ED_EINVAL, "%s: column %d of row %d out of range", who, c, r);
            adj[start[r] + k] = c;
        }
    // neighbours in the order the breadth-first sweep appends them: fewest neighbours first, then index
    for (int r = 0; r < n; ++r)
        std::sort(adj.begin() + start[r], adj.begin() + start[r + 1],
                  [&](int a, int b) { return nnz[a] != nnz[b] ? nnz[a] < nnz[b] : a < b; });
    std::vector<int> mark(n, -1), order;   // mark: the sweep that reached a vertex (-1: none yet)
    order.reserve(n);
    std::vector<int> level, next;
    int sweep = 0;
    // one breadth-first sweep over the unordered vertices from s: its levels, the last one kept in `level`;
    // returns the number of levels.  Marks the vertices it reaches with `sweep`.
    auto levels = [&](int s, std::vector<int> *out) {
        ++sweep;
        level.assign(1, s);
        mark[s] = sweep;
        if (out) out->push_back(s);
        int depth = 1;
        while (true) {
            next.clear();
            for (int v : level)
                for (int64_t k = start[v]; k < start[v + 1]; ++k) {
                    const int w = adj[k];
                    if (mark[w] >= 0 && (mark[w] == sweep || mark[w] == 0)) continue;
                    mark[w] = sweep;
                    next.push_back(w);
                    if (out) out->push_back(w);
                }
            if (next.empty()) return depth;
            level.swap(next);
            ++depth;
        }
    };
    // mark 0: already placed in `order`.  Vertices of a sweep that were not placed get unmarked again.
    std::vector<int> comp;
    for (int seed = 0; seed < n; ++seed) {
        if (mark[seed] == 0) continue;
        // the component's vertices, and its vertex of fewest neighbours (lowest index among equals)
        comp.clear();
        levels(seed, &comp);
        int s = seed;
        for (int v : comp)
            if (nnz[v] < nnz[s] || (nnz[v] == nnz[s] && v < s)) s = v;
        // a pseudo-peripheral start (George and Liu): move to the last level's vertex of fewest neighbours
        // while that lengthens the level structure
        int depth = levels(s, nullptr);
        for (int it = 0; it < 32; ++it) {
            int c = level[0];
            for (int v : level)
                if (nnz[v] < nnz[c] || (nnz[v] == nnz[c] && v < c)) c = v;
            const int d = levels(c, nullptr);
            if (d <= depth) break;
            s = c;
            depth = d;
        }
        // Cuthill-McKee: breadth-first from s, each vertex's new neighbours in the sorted order
        for (int v : comp) mark[v] = -1;
        const size_t first = order.size();
        order.push_back(s);
        mark[s] = 0;
        for (size_t i = first; i < order.size(); ++i) {
            const int v = order[i];
            for (int64_t k = start[v]; k < start[v + 1]; ++k) {
                const int w = adj[k];
                if (mark[w] == 0) continue;
                mark[w] = 0;
                order.push_back(w);
            }
        }
    }
    if ((int)order.size() != n) return set_error(ED_EINVAL, "%s: the table is not symmetric", who);
    // reversed (reverse Cuthill-McKee)
    for (int q = 0; q < n; ++q) perm[q] = order[n - 1 - q];
    return ED_OK;
}

int ed_permute_basis(const uint64_t *states, const int32_t *cols, const double *vals, const int32_t *nnz,
                     int64_t dim, int32_t width, int layout, int32_t n_vals, const int64_t *perm,
                     uint64_t *states_out, int32_t *cols_out, double *vals_out, int32_t *nnz_out) {
    clear_error();
    const char *who = "ed_permute_basis";
    if (!states || !nnz || !perm || !states_out || !nnz_out || dim < 1 || width < 0 || (n_vals != 1 && n_vals != 2))
        return set_error(ED_EINVAL, "%s: bad arguments", who);
    if (width > 0 && (!cols || !vals || !cols_out || !vals_out)) return set_error(ED_EINVAL, "%s: NULL table", who);
    if (layout != ED_ROW_MAJOR && layout != ED_COL_MAJOR) return set_error(ED_EINVAL, "%s: bad layout %d", who, layout);
    if (dim > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "%s: dim too large", who);
    // inverse permutation; a repeated or out-of-range entry is an error
    std::vector<int64_t> inv(dim, -1);
    for (int64_t q = 0; q < dim; ++q) {
        const int64_t o = perm[q];
        if (o < 0 || o >= dim || inv[o] >= 0) return set_error(ED_EINVAL, "%s: perm is not a permutation (entry %lld)", who, (long long)q);
        inv[o] = q;
    }
    std::vector<std::pair<int32_t, int64_t>> row;   // (new column, source slot)
    row.reserve(width);
    for (int64_t q = 0; q < dim; ++q) {
        const int64_t o = perm[q];
        states_out[q] = states[o];
        const int32_t n = nnz[o];
        if (n < 0 || n > width) return set_error(ED_EINVAL, "%s: nnz[%lld] = %d out of range", who, (long long)o, n);
        nnz_out[q] = n;
        row.clear();
        for (int32_t k = 0; k < n; ++k) {
            const int64_t src = layout == ED_ROW_MAJOR ? o * width + k : (int64_t)k * dim + o;
            const int32_t c = cols[src];
            if (c < 0 || c >= dim) return set_error(ED_EINVAL, "%s: column %d out of range", who, c);
            row.emplace_back((int32_t)inv[c], src);
        }
        std::sort(row.begin(), row.end());
        for (int32_t k = 0; k < width; ++k) {
            const int64_t dst = layout == ED_ROW_MAJOR ? q * width + k : (int64_t)k * dim + q;
            const bool live = k < n;
            cols_out[dst] = live ? row[k].first : 0;
            for (int v = 0; v < n_vals; ++v) vals_out[n_vals * dst + v] = live ? vals[n_vals * row[k].second + v] : 0.0;
        }
    }
    return ED_OK;
}

int ed_occupation_correlations(const double *g, int32_t n_sites, double *docc, double *nn, double *szsz) {
    clear_error();
    if (!g || n_sites < 1 || n_sites > 32) return set_error(ED_EINVAL, "ed_occupation_correlations: bad arguments");
    const int ns = n_sites, n2 = 2 * n_sites;
    auto G = [&](int a, int b) { return g[a * n2 + b]; };
    for (int i = 0; i < ns; ++i) {
        if (docc) docc[i] = G(i, ns + i);
        for (int j = 0; j < ns; ++j) {
            const double uu = G(i, j), ud = G(i, ns + j), du = G(ns + i, j), dd = G(ns + i, ns + j);
            if (nn) nn[i * ns + j] = uu + ud + du + dd;
            if (szsz) szsz[i * ns + j] = 0.25 * (uu - ud - du + dd);
        }
    }
    return ED_OK;
}

int ed_spin_correlations(const double *g, const double *c, int32_t n_sites, double *ss) {
    clear_error();
    if (!g || !c || !ss || n_sites < 1 || n_sites > 32) return set_error(ED_EINVAL, "ed_spin_correlations: bad arguments");
    const int ns = n_sites, n2 = 2 * n_sites;
    auto G = [&](int a, int b) { return g[a * n2 + b]; };
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) {
            if (i == j) {
                ss[i * ns + i] = 0.75 * (G(i, i) + G(ns + i, ns + i) - 2.0 * G(i, ns + i));
            } else {
                const double zz = 0.25 * (G(i, j) - G(i, ns + j) - G(ns + i, j) + G(ns + i, ns + j));
                ss[i * ns + j] = zz + 0.5 * (c[i * ns + j] + c[j * ns + i]);
            }
        }
    return ED_OK;
}

int ed_tridiag_lowest(const double *a, const double *b, int m, double *e0) {
    clear_error();
    if (!a || !e0 || m < 1 || (m > 1 && !b)) return set_error(ED_EINVAL, "ed_tridiag_lowest: bad arguments");
    for (int k = 0; k < m; ++k)
        if (!std::isfinite(a[k]) || (k < m - 1 && !std::isfinite(b[k])))
            return set_error(ED_EINVAL, "ed_tridiag_lowest: non-finite entry at %d", k);
    *e0 = tridiag_lowest(a, b, m);
    return ED_OK;
}

int ed_tridiag_lowest_vector(const double *a, const double *b, int m, double *e0, double *y) {
    int rc = ed_tridiag_lowest(a, b, m, e0);
    if (rc) return rc;
    if (!y) return set_error(ED_EINVAL, "ed_tridiag_lowest_vector: y is NULL");
    if (m == 1) { y[0] = 1.0; return ED_OK; }
    // Inverse iteration on (T - lambda I) with partial pivoting (tridiagonal
    // elimination with row swaps, so the factor has two super-diagonals).
    double tn = 0.0;
    for (int k = 0; k < m; ++k) tn = std::max(tn, std::fabs(a[k]) + (k ? std::fabs(b[k - 1]) : 0) + (k < m - 1 ? std::fabs(b[k]) : 0));
    const double tiny = std::ldexp(1.0, -52) * std::max(tn, 1e-300);
    const double lam = *e0;
    std::vector<double> d(m), du(m), du2(m), dl(m), x(m);
    std::vector<int> swp(m, 0);
    for (int k = 0; k < m; ++k) { d[k] = a[k] - lam; du[k] = k < m - 1 ? b[k] : 0.0; dl[k] = k < m - 1 ? b[k] : 0.0; du2[k] = 0.0; }
    for (int k = 0; k < m - 1; ++k) {
        if (std::fabs(d[k]) >= std::fabs(dl[k])) {
            if (d[k] == 0.0) d[k] = tiny;
            double f = dl[k] / d[k];
            dl[k] = f;
            d[k + 1] -= f * du[k];
            swp[k] = 0;
        } else {
            double f = d[k] / dl[k];
            d[k] = dl[k];
            dl[k] = f;
            double tmp = du[k];
            du[k] = d[k + 1];
            d[k + 1] = tmp - f * d[k + 1];
            if (k < m - 2) { du2[k] = du[k + 1]; du[k + 1] = -f * du[k + 1]; }
            swp[k] = 1;
        }
    }
    if (d[m - 1] == 0.0) d[m - 1] = tiny;
    for (int k = 0; k < m; ++k) x[k] = 1.0 / std::sqrt((double)m);
    for (int it = 0; it < 4; ++it) {
        // forward: apply L^{-1} with the recorded swaps
        for (int k = 0; k < m - 1; ++k) {
            if (swp[k]) { double t = x[k]; x[k] = x[k + 1]; x[k + 1] = t - dl[k] * x[k]; }
            else x[k + 1] -= dl[k] * x[k];
        }
        // back substitution with U (diag d, super du, second super du2)
        for (int k = m - 1; k >= 0; --k) {
            double s = x[k];
            if (k + 1 < m) s -= du[k] * x[k + 1];
            if (k + 2 < m) s -= du2[k] * x[k + 2];
            if (std::fabs(d[k]) < tiny) d[k] = d[k] < 0 ? -tiny : tiny;
            x[k] = s / d[k];
        }
        double nrm = 0.0;
        for (int k = 0; k < m; ++k) nrm += x[k] * x[k];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return set_error(ED_EINVAL, "ed_tridiag_lowest_vector: inverse iteration failed");
        for (int k = 0; k < m; ++k) x[k] /= nrm;
    }
    double sgn = x[0] < 0 ? -1.0 : 1.0;
    for (int k = 0; k < m; ++k) y[k] = sgn * x[k];
    return ED_OK;
}

}  // extern "C"
