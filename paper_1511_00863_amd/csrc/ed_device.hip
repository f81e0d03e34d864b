// Device side of the library for gfx950 (CDNA4, wave64): matrix-free H.v over
// the two-species occupation basis and the Lanczos iteration built on it.
//
// H x = (H_up x I) x + (I x H_dn) x + U Docc o x   (Eq. 3, 4, 5 and the on-site
// term).  With X the dim_up-by-dim_dn view of x:
//   up part   (Eq. 4): row r of the result is a signed sum of whole rows
//                      X[J_up[r,k], :]  -> coalesced row-segment reads;
//   down part (Eq. 5): every row X[r, :] is multiplied by H_dn
//                      -> the row is staged in LDS and gathered from there.
// The two parts want opposite traversals once X is larger than any cache, so
// they are two kernels:
//   k_up   -- tiles are (column stripe, row chunk).  Every tile of a stripe runs
//             on the same XCD, back to back, so the stripe X[:, cs] is read
//             from HBM once and the ~nnz_up re-reads per element hit that
//             XCD's L2.
//   k_down -- one workgroup per row block: stage X[r, :] in LDS, gather the
//             down neighbours, add the up part written by k_up, the U term
//             and the Lanczos recurrence term, and emit float64 partial dot
//             products for the step (fixed slots, reduced in fixed order).
// A Lanczos step (Alg. 1) is k_up, k_down, k_reduce (one workgroup, scalars
// stay on the device) and k_update (f_{j+1} in place).  No floating-point
// atomics anywhere: results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/ed.h"
#include "ed_internal.h"

namespace ed {

// ---------------------------------------------------------------------------
// Vectors are stored unnormalised ("deferred normalisation"): the buffer of
// Lanczos vector f_j holds s_j f_j with s_1 = |f1| and s_j = b_j, and the
// kernels apply sigma_j = 1/s_j on the fly.  A step is
//   k_up     T  = t * up-part(F_j)                                   (Eq. 4)
//   k_down   q  = sigma_j (T + down-part(F_j) + U Docc F_j) - b_j sigma_{j-1} F_{j-1}
//               = H f_j - b_j f_{j-1}                  (Eq. 5, Alg. 1 line 4)
//            + partial dots of q with F_j (and F_{j-1} in the mixed form)
//   k_reduce a_j = q.f_j (Alg. 1 line 5); mixed form: q's projection onto
//            span{f_j, f_{j-1}} from their 2x2 Gram matrix
//   k_update F_{j+1} = q - a_j f_j (- beta f_{j-1})  in place (line 6)
//            + partial sums of |F_{j+1}|^2 of the stored values
//   k_norm   b_{j+1} = |F_{j+1}| (line 7), breakdown test (line 8)
// so b_{j+1} is the norm of the vector actually stored, with no cancellation.
//
// workspace layout: [Hdr: 256 B][y: max_steps doubles][part: P x 8][part2: 8192]
struct Hdr {
    double sig_cur;    // 1 / s_j of the current vector
    double sig_prev;   // 1 / s_{j-1}
    double cx, cp;     // update coefficients on the stored F_j and F_{j-1}
    double scale;      // max_k(|a_k|, b_k) so far (breakdown threshold)
    double vinv;       // 1 / |v| for the two-pass ground state
    double norm2;      // |f1|^2 of the last init
    int32_t jdev;      // completed steps
    int32_t status;    // 0 running, ED_BREAKDOWN, or kInitBad
};
static_assert(sizeof(Hdr) <= 256, "header too large");
constexpr int32_t kInitBad = 100;
constexpr int kPartStride = 8;   // doubles per k_down partial slot
constexpr int kUpdBlocks = 8192; // k_update / k_sumsq grid cap = part2 slots

static inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

struct WsLayout {
    Hdr *hdr;
    double *y;
    double *part;
    double *part2;
};

static int64_t n_partial_slots(const ed_ham *h) { return std::max<int64_t>(h->dim_up, 1); }

static int64_t ws_bytes(const ed_ham *h, int32_t max_steps) {
    return 256 + align256(8 * (int64_t)std::max(max_steps, 1)) + align256(8 * kPartStride * n_partial_slots(h)) +
           8 * kUpdBlocks;
}

static WsLayout ws_layout(const ed_ham *h, void *ws, int32_t max_steps) {
    char *p = static_cast<char *>(ws);
    WsLayout l;
    l.hdr = reinterpret_cast<Hdr *>(p);
    p += 256;
    l.y = reinterpret_cast<double *>(p);
    p += align256(8 * (int64_t)std::max(max_steps, 1));
    l.part = reinterpret_cast<double *>(p);
    p += align256(8 * kPartStride * n_partial_slots(h));
    l.part2 = reinterpret_cast<double *>(p);
    return l;
}

// ---------------------------------------------------------------------------
// reductions: wave64 butterfly, then a fixed-order sum over waves.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
    __shared__ double red[16][NV];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[w][k];
            out[k] = s;
        }
    }
}

__device__ __forceinline__ bool frozen(const Hdr *hdr, int max_steps) {
    return hdr->status != 0 || hdr->jdev >= max_steps;
}

// ---------------------------------------------------------------------------
// k_up: out[r, c] = t * sum_k sgn_k * x[J_up[r,k], c]   (Eq. 4)
// Workgroup g runs on XCD g % 8 (round-robin dispatch).  Stripe s belongs to
// XCD s % 8; the n_rc row chunks of a stripe are consecutive workgroups of
// that XCD.  A wave covers 64/w rows x w columns of a stripe.
template <typename T>
__global__ __launch_bounds__(256) void k_up(const T *__restrict__ x, T *__restrict__ out,
                                            const uint16_t *__restrict__ tab, int Dup, int Ddn, int Wup,
                                            int w_log2, int rc, int n_stripes, int n_rc, T t,
                                            const Hdr *__restrict__ hdr, int gate, int max_steps) {
    if (gate && frozen(hdr, max_steps)) return;
    const int g = blockIdx.x, xcd = g & 7, local = g >> 3;
    const int sl = local / n_rc, rci = local - sl * n_rc;
    const int s = sl * 8 + xcd;
    if (s >= n_stripes) return;
    const int w = 1 << w_log2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int rpw = 64 >> w_log2;
    const int c = s * w + (lane & (w - 1));
    if (c >= Ddn) return;
    const int r1 = min(Dup, (rci + 1) * rc);
    for (int r = rci * rc + wave * rpw + (lane >> w_log2); r < r1; r += nwave * rpw) {
        T acc = T(0);
        for (int k = 0; k < Wup; ++k) {
            const unsigned e = tab[(int64_t)k * Dup + r];
            if (e == 0xFFFFu) break;
            const T v = x[(int64_t)(e >> 1) * Ddn + c];
            acc += (e & 1u) ? -v : v;
        }
        out[(int64_t)r * Ddn + c] = t * acc;
    }
}

// ---------------------------------------------------------------------------
// k_down: q[r, c] = sig * (io[r, c] + t * sum_k sgn_k x[r, J_dn[c,k]] + U*Docc[r,c]*x[r,c])
//                   (- b_j sig_prev p[r, c] in a Lanczos step)          (Eq. 5)
// io holds the up part on entry and q on exit.
// MODE 0: plain H.v (sig = 1).  MODE 1: Lanczos, partial q.x.
// MODE 2: Lanczos mixed form, partials (q.x, q.p, x.x, x.p, p.p).
template <typename T, int MODE, bool LDS>
__global__ __launch_bounds__(1024) void k_down(const T *__restrict__ x, T *__restrict__ io, const T *__restrict__ p,
                                               const uint16_t *__restrict__ tab,
                                               const uint64_t *__restrict__ st_up,
                                               const uint64_t *__restrict__ st_dn, int Dup, int Ddn, int Wdn,
                                               int rpb, T t, T U, const double *__restrict__ bvec,
                                               const Hdr *__restrict__ hdr, double *__restrict__ partials,
                                               int max_steps) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *xs = reinterpret_cast<T *>(smem);
    bool has_prev = false;
    T sig = T(1), cprev = T(0);
    if (MODE != 0) {
        if (frozen(hdr, max_steps)) return;
        const int j = hdr->jdev;
        has_prev = j > 0;
        sig = static_cast<T>(hdr->sig_cur);
        cprev = static_cast<T>(bvec[j] * hdr->sig_prev);
    }
    const int r0 = blockIdx.x * rpb;
    const int nr = min(rpb, Dup - r0);
    const int64_t base = (int64_t)r0 * Ddn;
    const int n = nr * Ddn;
    if (LDS) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = x[base + i];
        __syncthreads();
    }
    constexpr int NV = MODE == 2 ? 5 : 1;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int rr = 0, c = i;
        if (rpb > 1) { rr = i / Ddn; c = i - rr * Ddn; }
        const T *xrow = LDS ? xs + rr * Ddn : x + base + (int64_t)rr * Ddn;
        T acc = T(0);
        for (int k = 0; k < Wdn; ++k) {
            const unsigned e = tab[(int64_t)k * Ddn + c];
            if (e == 0xFFFFu) break;
            const T v = xrow[e >> 1];
            acc += (e & 1u) ? -v : v;
        }
        const T xv = xrow[c];
        const T nd = static_cast<T>(__popcll(st_up[r0 + rr] & st_dn[c]));
        T q = io[base + i] + t * acc + U * nd * xv;
        T pv = T(0);
        if (MODE != 0) {
            q *= sig;
            if (has_prev) {
                pv = p[base + i];
                q -= cprev * pv;
            }
        }
        io[base + i] = q;
        if (MODE != 0) {
            const double qd = q, xd = xv;
            s[0] += qd * xd;
            if (MODE == 2) {
                const double pd = pv;
                s[1] += qd * pd;
                s[2] += xd * xd;
                s[3] += xd * pd;
                s[4] += pd * pd;
            }
        }
    }
    if (MODE != 0) {
        double tot[NV];
        block_sum<NV>(s, tot);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NV; ++k) partials[(int64_t)blockIdx.x * kPartStride + k] = tot[k];
    }
}

// ---------------------------------------------------------------------------
// k_reduce: fixed-order sum of the partial dots, then a_j and the update
// coefficients.  MODE 1 (Alg. 1, float64): a_j = q.f_j, remove a_j f_j.
// MODE 2 (mixed, local re-orthogonalisation): remove q's projection onto
// span{f_j, f_{j-1}} computed with the Gram matrix of the stored vectors; a_j
// is the f_j coefficient (the f_{j-1} coefficient corrects b_j's rounding).
template <int MODE>
__global__ __launch_bounds__(1024) void k_reduce(const double *__restrict__ partials, int n, Hdr *hdr,
                                                 double *a, int max_steps) {
    if (frozen(hdr, max_steps)) return;
    constexpr int NV = MODE == 2 ? 5 : 1;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += partials[(int64_t)i * kPartStride + k];
    double tot[NV];
    block_sum<NV>(s, tot);
    if (threadIdx.x != 0) return;
    const int j = hdr->jdev;
    const double sx = hdr->sig_cur, sp = hdr->sig_prev;
    double alpha, beta = 0.0;
    if (MODE == 1) {
        alpha = sx * tot[0];
    } else {
        const double qx = sx * tot[0], qp = sp * tot[1];
        const double xx = sx * sx * tot[2], xp = sx * sp * tot[3], pp = sp * sp * tot[4];
        if (j > 0) {
            const double det = xx * pp - xp * xp;
            alpha = (pp * qx - xp * qp) / det;
            beta = (xx * qp - xp * qx) / det;
        } else {
            alpha = qx / xx;
        }
    }
    a[j] = alpha;
    hdr->cx = alpha * sx;
    hdr->cp = j > 0 ? beta * sp : 0.0;
}

// k_update: F_{j+1} = q - cx F_j - cp F_{j-1} in place on q (arithmetic in
// float64, one rounding to T), partial sums of the stored values' squares,
// and for the two-pass ground state v += y_j f_j.
template <typename T>
__global__ __launch_bounds__(256) void k_update(T *__restrict__ q, const T *__restrict__ x,
                                                const T *__restrict__ p, T *__restrict__ v,
                                                const double *__restrict__ y, const Hdr *__restrict__ hdr,
                                                double *__restrict__ part2, int64_t n, int max_steps) {
    if (frozen(hdr, max_steps)) return;
    const double cx = hdr->cx, cp = hdr->cp;
    const double yj = v ? y[hdr->jdev] * hdr->sig_cur : 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double s[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xv = x[i];
        double qv = (double)q[i] - cx * xv;
        if (cp != 0.0) qv -= cp * (double)p[i];
        const T st = static_cast<T>(qv);
        q[i] = st;
        const double sd = st;
        s[0] += sd * sd;
        if (v) v[i] = static_cast<T>((double)v[i] + yj * xv);
    }
    double tot[1];
    block_sum<1>(s, tot);
    if (threadIdx.x == 0) part2[blockIdx.x] = tot[0];
}

// k_norm: b_{j+1} = |F_{j+1}|, breakdown test, advance the step counter.
__global__ __launch_bounds__(1024) void k_norm(const double *__restrict__ part2, int n, Hdr *hdr,
                                               const double *a, double *b, int max_steps, double eps) {
    if (frozen(hdr, max_steps)) return;
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[0] += part2[i];
    double tot[1];
    block_sum<1>(s, tot);
    if (threadIdx.x != 0) return;
    const int j = hdr->jdev;
    const double bn = sqrt(tot[0]);
    const double scale = fmax(hdr->scale, fmax(fabs(a[j]), bn));
    b[j + 1] = bn;
    hdr->scale = scale;
    const bool brk = !(bn > 64.0 * eps * scale);   // also true for NaN
    hdr->sig_prev = hdr->sig_cur;
    hdr->sig_cur = brk ? 0.0 : 1.0 / bn;
    hdr->jdev = j + 1;
    if (brk) hdr->status = ED_BREAKDOWN;
}

// ---------------------------------------------------------------------------
// start vector and two-pass normalisation
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T *__restrict__ x, int64_t n, double *__restrict__ part2) {
    double s[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = x[i];
        s[0] += v * v;
    }
    double tot[1];
    block_sum<1>(s, tot);
    if (threadIdx.x == 0) part2[blockIdx.x] = tot[0];
}

// mode 0: start a Lanczos run: sigma_1 = 1/|f1|, b_1 = 0, counters reset.
// mode 1: vinv = 1/|v|.
__global__ __launch_bounds__(1024) void k_init_norm(const double *__restrict__ part2, int n, Hdr *hdr, double *b,
                                                    int mode) {
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[0] += part2[i];
    double tot[1];
    block_sum<1>(s, tot);
    if (threadIdx.x != 0) return;
    const double n2 = tot[0];
    const bool ok = n2 > 0.0 && n2 < INFINITY;
    if (mode == 0) {
        hdr->norm2 = n2;
        hdr->sig_cur = ok ? 1.0 / sqrt(n2) : 0.0;
        hdr->sig_prev = 0.0;
        hdr->cx = hdr->cp = 0.0;
        hdr->scale = 0.0;
        hdr->jdev = 0;
        hdr->status = ok ? 0 : kInitBad;
        b[0] = 0.0;
    } else {
        hdr->vinv = ok ? 1.0 / sqrt(n2) : 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_scaled(const T *__restrict__ in, T *__restrict__ out,
                                                     const Hdr *hdr, int64_t n, int use_vinv) {
    const double sc = use_vinv ? hdr->vinv : 1.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = use_vinv ? static_cast<T>((double)in[i] * sc) : in[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill0(T *__restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = T(0);
}

// ---------------------------------------------------------------------------
// launch configuration ("tile")
struct Tile {
    int up_wlog2;   // stripe width = 2^up_wlog2 columns (<= 64)
    int up_rc;      // rows per k_up workgroup
    int up_block;   // k_up threads per workgroup
    int dn_block;   // k_down threads per workgroup
    int dn_rpb;     // rows per k_down workgroup (0 = derive from LDS)
};

// Candidate tiles searched by ed_tune; id 0 means "heuristic default".
static const Tile kTiles[] = {
    {0, 0, 0, 0, 0},
    {6, 64, 256, 1024, 0}, {5, 64, 256, 1024, 0}, {4, 64, 256, 1024, 0},
    {6, 128, 256, 1024, 0}, {5, 128, 256, 1024, 0}, {4, 128, 256, 1024, 0},
    {6, 32, 256, 1024, 0}, {5, 32, 256, 1024, 0},
    {6, 64, 256, 512, 0}, {5, 64, 256, 512, 0}, {6, 64, 256, 256, 0}, {5, 64, 256, 256, 0},
    {6, 256, 256, 1024, 0}, {5, 256, 256, 1024, 0},
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kLdsBudget = 152 * 1024;

static int elem_size(const ed_ham *h) { return h->dtype == ED_F64 ? 8 : 4; }

static Tile resolve_tile(const ed_ham *h) {
    Tile t = (h->tile > 0 && h->tile < kNumTiles) ? kTiles[h->tile] : Tile{0, 0, 0, 0, 0};
    const int es = elem_size(h);
    if (t.up_block == 0) {
        t.up_wlog2 = es == 8 ? 5 : 6;
        t.up_rc = 64;
        t.up_block = 256;
        t.dn_block = h->dim_dn >= 1024 ? 1024 : 256;
    }
    // stripes narrower than the row are pointless
    while (t.up_wlog2 > 4 && (1 << (t.up_wlog2 - 1)) >= h->dim_dn) --t.up_wlog2;
    if (t.dn_rpb == 0) {
        const int64_t row_bytes = h->dim_dn * es;
        int64_t by_lds = std::max<int64_t>(1, kLdsBudget / row_bytes);
        int64_t by_fill = std::max<int64_t>(1, (2 * t.dn_block + h->dim_dn - 1) / h->dim_dn);
        t.dn_rpb = (int)std::min<int64_t>(std::min(by_lds, by_fill), h->dim_up);
    }
    return t;
}

static int check_ham(const ed_ham *h, const char *who) {
    if (!h) return set_error(ED_EINVAL, "%s: ham is NULL", who);
    if (h->dim_up < 1 || h->dim_dn < 1) return set_error(ED_EINVAL, "%s: bad dims", who);
    if (h->dim_up > 32767 || h->dim_dn > 32767)
        return set_error(ED_EOVERFLOW, "%s: per-spin dims must be <= 32767", who);
    if (h->w_up < 0 || h->w_dn < 0 || (h->w_up && !h->tab_up) || (h->w_dn && !h->tab_dn) || !h->st_up ||
        !h->st_dn)
        return set_error(ED_EINVAL, "%s: missing tables or states", who);
    if (h->dtype != ED_F64 && h->dtype != ED_F32) return set_error(ED_EINVAL, "%s: bad dtype %d", who, h->dtype);
    if (h->tile < 0 || h->tile >= kNumTiles) return set_error(ED_EINVAL, "%s: bad tile id %d", who, h->tile);
    if (!std::isfinite(h->t) || !std::isfinite(h->U)) return set_error(ED_EINVAL, "%s: non-finite t or U", who);
    return ED_OK;
}

static int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return ED_OK;
    return set_error(ED_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define ED_HIP(call)                                          \
    do {                                                      \
        int rc_ = hip_check((call), #call);                   \
        if (rc_) return rc_;                                  \
    } while (0)

#define ED_LAUNCHED(name)                                     \
    do {                                                      \
        int rc_ = hip_check(hipGetLastError(), name);         \
        if (rc_) return rc_;                                  \
    } while (0)

static int grid_for(int64_t n, int block, int cap = 4096) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

template <typename T>
static int launch_up(const ed_ham *h, const Tile &tl, const T *x, T *out, const Hdr *hdr, int gate, int max_steps,
                     hipStream_t s) {
    const int w = 1 << tl.up_wlog2;
    const int n_stripes = (int)((h->dim_dn + w - 1) / w);
    const int n_rc = (int)((h->dim_up + tl.up_rc - 1) / tl.up_rc);
    const int64_t grid = 8LL * n_rc * ((n_stripes + 7) / 8);
    if (grid > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "k_up grid too large");
    if (h->w_up == 0) {   // no up hopping: out = 0
        hipLaunchKernelGGL(k_fill0<T>, dim3(grid_for(h->dim_up * h->dim_dn, 256)), dim3(256), 0, s, out,
                           h->dim_up * h->dim_dn);
        ED_LAUNCHED("k_fill0");
        return ED_OK;
    }
    hipLaunchKernelGGL(k_up<T>, dim3((unsigned)grid), dim3(tl.up_block), 0, s, x, out, h->tab_up, (int)h->dim_up,
                       (int)h->dim_dn, h->w_up, tl.up_wlog2, tl.up_rc, n_stripes, n_rc, static_cast<T>(h->t), hdr,
                       gate, max_steps);
    ED_LAUNCHED("k_up");
    return ED_OK;
}

template <typename T, int MODE>
static int launch_down(const ed_ham *h, const Tile &tl, const T *x, T *io, const T *p, const double *bvec,
                       const Hdr *hdr, double *part, int max_steps, hipStream_t s) {
    const int64_t row_bytes = h->dim_dn * (int64_t)sizeof(T);
    const bool lds = row_bytes * tl.dn_rpb <= kLdsBudget;
    const int rpb = lds ? tl.dn_rpb : 1;
    const int grid = (int)((h->dim_up + rpb - 1) / rpb);
    const size_t shm = lds ? (size_t)(row_bytes * rpb) : 0;
    const T t = static_cast<T>(h->t), U = static_cast<T>(h->U);
    if (lds) {
        hipLaunchKernelGGL((k_down<T, MODE, true>), dim3(grid), dim3(tl.dn_block), shm, s, x, io, p, h->tab_dn,
                           h->st_up, h->st_dn, (int)h->dim_up, (int)h->dim_dn, h->w_dn, rpb, t, U, bvec, hdr, part,
                           max_steps);
    } else {
        hipLaunchKernelGGL((k_down<T, MODE, false>), dim3(grid), dim3(tl.dn_block), 0, s, x, io, p, h->tab_dn,
                           h->st_up, h->st_dn, (int)h->dim_up, (int)h->dim_dn, h->w_dn, 1, t, U, bvec, hdr, part,
                           max_steps);
    }
    ED_LAUNCHED("k_down");
    return ED_OK;
}

static int down_grid(const ed_ham *h, const Tile &tl) {
    const int es = elem_size(h);
    const bool lds = h->dim_dn * (int64_t)es * tl.dn_rpb <= kLdsBudget;
    const int rpb = lds ? tl.dn_rpb : 1;
    return (int)((h->dim_up + rpb - 1) / rpb);
}

// Kernels staging rows in LDS may use up to kLdsBudget bytes of it; set once,
// outside any stream capture.
static int ensure_attrs() {
    static int rc = -1000;
    if (rc != -1000) return rc;
    const void *fs[] = {
        reinterpret_cast<const void *>(k_down<double, 0, true>), reinterpret_cast<const void *>(k_down<double, 1, true>),
        reinterpret_cast<const void *>(k_down<double, 2, true>), reinterpret_cast<const void *>(k_down<float, 0, true>),
        reinterpret_cast<const void *>(k_down<float, 1, true>), reinterpret_cast<const void *>(k_down<float, 2, true>)};
    int r = ED_OK;
    for (const void *f : fs) {
        r = hip_check(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget),
                      "hipFuncSetAttribute(k_down)");
        if (r) break;
    }
    rc = r;
    return rc;
}

template <typename T>
static int hv_impl(const ed_ham *h, const T *x, T *y, hipStream_t s) {
    const Tile tl = resolve_tile(h);
    int rc = launch_up<T>(h, tl, x, y, nullptr, 0, 0, s);
    if (rc) return rc;
    return launch_down<T, 0>(h, tl, x, y, nullptr, nullptr, nullptr, nullptr, 0, s);
}

static int upd_grid(int64_t n) { return grid_for(n, 256 * 4, kUpdBlocks); }

// One Alg. 1 step on raw pointers (v != nullptr: also v += y_j f_j).  With
// ev != nullptr an event is recorded before each kernel and after the last.
template <typename T, int MODE>
static int step_impl(const ed_ham *h, const Tile &tl, const T *f_prev, const T *f_cur, T *f_next, double *a,
                     double *b, T *v, const WsLayout &w, int max_steps, hipStream_t s, hipEvent_t *ev = nullptr) {
    if (ev) ED_HIP(hipEventRecord(ev[0], s));
    int rc = launch_up<T>(h, tl, f_cur, f_next, w.hdr, 1, max_steps, s);
    if (rc) return rc;
    if (ev) ED_HIP(hipEventRecord(ev[1], s));
    rc = launch_down<T, MODE>(h, tl, f_cur, f_next, f_prev, b, w.hdr, w.part, max_steps, s);
    if (rc) return rc;
    if (ev) ED_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL(k_reduce<MODE>, dim3(1), dim3(1024), 0, s, w.part, down_grid(h, tl), w.hdr, a, max_steps);
    ED_LAUNCHED("k_reduce");
    if (ev) ED_HIP(hipEventRecord(ev[3], s));
    const int64_t n = h->dim_up * h->dim_dn;
    const int g = upd_grid(n);
    hipLaunchKernelGGL(k_update<T>, dim3(g), dim3(256), 0, s, f_next, f_cur, f_prev, v, w.y, w.hdr, w.part2, n,
                       max_steps);
    ED_LAUNCHED("k_update");
    if (ev) ED_HIP(hipEventRecord(ev[4], s));
    const double eps = MODE == 1 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -24);
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(1024), 0, s, w.part2, g, w.hdr, a, b, max_steps, eps);
    ED_LAUNCHED("k_norm");
    if (ev) ED_HIP(hipEventRecord(ev[5], s));
    return ED_OK;
}

static int step_dispatch(const ed_ham *h, const Tile &tl, void *f_prev, void *f_cur, void *f_next, double *a,
                         double *b, void *v, const WsLayout &w, int max_steps, hipStream_t s,
                         hipEvent_t *ev = nullptr) {
    if (h->dtype == ED_F64)
        return step_impl<double, 1>(h, tl, (const double *)f_prev, (const double *)f_cur, (double *)f_next, a, b,
                                    (double *)v, w, max_steps, s, ev);
    return step_impl<float, 2>(h, tl, (const float *)f_prev, (const float *)f_cur, (float *)f_next, a, b,
                               (float *)v, w, max_steps, s, ev);
}

// |in|^2 in float64 -> mode 0: start a run (sigma_1) / mode 1: vinv; then
// out = in (mode 0, the stored f_1 is the raw start vector) or in * vinv.
template <typename T>
static int norm_launch(const T *in, T *out, int64_t n, const WsLayout &w, double *b, int mode, hipStream_t s) {
    const int g = upd_grid(n);
    hipLaunchKernelGGL(k_sumsq<T>, dim3(g), dim3(256), 0, s, in, n, w.part2);
    ED_LAUNCHED("k_sumsq");
    hipLaunchKernelGGL(k_init_norm, dim3(1), dim3(1024), 0, s, w.part2, g, w.hdr, b, mode);
    ED_LAUNCHED("k_init_norm");
    hipLaunchKernelGGL(k_copy_scaled<T>, dim3(upd_grid(n)), dim3(256), 0, s, in, out, w.hdr, n, mode);
    ED_LAUNCHED("k_copy_scaled");
    return ED_OK;
}

static int check_lanczos(const ed_ham *h, const ed_lanczos *st, void *ws, const char *who) {
    int rc = check_ham(h, who);
    if (rc) return rc;
    if (!st || !st->f_prev || !st->f_cur || !st->f_next || !st->a || !st->b || !ws)
        return set_error(ED_EINVAL, "%s: missing Lanczos buffers or workspace", who);
    if (st->f_prev == st->f_cur || st->f_cur == st->f_next || st->f_prev == st->f_next)
        return set_error(ED_EINVAL, "%s: the three Lanczos vectors must be distinct", who);
    if (st->max_steps < 1) return set_error(ED_EINVAL, "%s: max_steps must be >= 1", who);
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return set_error(ED_EINVAL, "%s: ws not 256-byte aligned", who);
    return ED_OK;
}

static void rotate(ed_lanczos *st) {
    void *old_prev = st->f_prev;
    st->f_prev = st->f_cur;
    st->f_cur = st->f_next;
    st->f_next = old_prev;
    st->j += 1;
}

static int init_impl(const ed_ham *h, ed_lanczos *st, const void *f1, const WsLayout &w, hipStream_t s) {
    const int64_t n = h->dim_up * h->dim_dn;
    if (h->dtype == ED_F64)
        return norm_launch<double>((const double *)f1, (double *)st->f_cur, n, w, st->b, 0, s);
    return norm_launch<float>((const float *)f1, (float *)st->f_cur, n, w, st->b, 0, s);
}

static int read_hdr(const WsLayout &w, Hdr *out, hipStream_t s) {
    ED_HIP(hipMemcpyAsync(out, w.hdr, sizeof(Hdr), hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    return ED_OK;
}

// A private non-blocking stream ordered after the caller's stream (graph
// capture is not possible on the legacy default stream).
struct SideStream {
    hipStream_t user = nullptr, own = nullptr;
    hipEvent_t ev = nullptr;
    int open(hipStream_t u) {
        user = u;
        ED_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        ED_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ED_HIP(hipEventRecord(ev, user));
        ED_HIP(hipStreamWaitEvent(own, ev, 0));
        return ED_OK;
    }
    int close() {
        int rc = ED_OK;
        if (own && ev) {
            if (hipEventRecord(ev, own) != hipSuccess || hipStreamWaitEvent(user, ev, 0) != hipSuccess)
                rc = set_error(ED_EDEVICE, "stream join failed");
        }
        if (ev) (void)hipEventDestroy(ev);
        if (own) (void)hipStreamDestroy(own);
        ev = nullptr;
        own = nullptr;
        return rc;
    }
    ~SideStream() {
        if (ev) (void)hipEventDestroy(ev);
        if (own) (void)hipStreamDestroy(own);
    }
};

// Launch `nsteps` steps as a replayed graph of 3*k steps (three-buffer rotation).
struct StepGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    int steps = 0;
    ~StepGraph() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
    }
};

static int capture_steps(const ed_ham *h, const Tile &tl, ed_lanczos st_copy, const WsLayout &w, int nsteps,
                         hipStream_t s, StepGraph &sg) {
    ED_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = ED_OK;
    for (int k = 0; k < nsteps && rc == ED_OK; ++k) {
        rc = step_dispatch(h, tl, st_copy.f_prev, st_copy.f_cur, st_copy.f_next, st_copy.a, st_copy.b, nullptr, w,
                           st_copy.max_steps, s);
        rotate(&st_copy);
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    ED_HIP(e);
    sg.g = g;
    ED_HIP(hipGraphInstantiate(&sg.ge, g, nullptr, nullptr, 0));
    sg.steps = nsteps;
    return ED_OK;
}

}  // namespace ed

using namespace ed;

extern "C" {

int ed_workspace_size(const ed_ham *h, int32_t max_steps, int64_t *bytes) {
    clear_error();
    int rc = check_ham(h, "ed_workspace_size");
    if (rc) return rc;
    if (!bytes || max_steps < 0) return set_error(ED_EINVAL, "ed_workspace_size: bad arguments");
    *bytes = ws_bytes(h, max_steps);
    return ED_OK;
}

int ed_hv(const ed_ham *h, const void *x, void *y, void *ws, void *stream) {
    clear_error();
    int rc = check_ham(h, "ed_hv");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    if (!x || !y || x == y) return set_error(ED_EINVAL, "ed_hv: x and y must be distinct device buffers");
    (void)ws;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->dtype == ED_F64) return hv_impl<double>(h, (const double *)x, (double *)y, s);
    return hv_impl<float>(h, (const float *)x, (float *)y, s);
}

int ed_lanczos_init(const ed_ham *h, ed_lanczos *st, const void *f1, void *ws, void *stream) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_lanczos_init");
    if (rc) return rc;
    if (!f1 || f1 == st->f_cur) return set_error(ED_EINVAL, "ed_lanczos_init: f1 must be a buffer other than f_cur");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout w = ws_layout(h, ws, st->max_steps);
    rc = init_impl(h, st, f1, w, s);
    if (rc) return rc;
    Hdr hh;
    rc = read_hdr(w, &hh, s);
    if (rc) return rc;
    if (hh.status != 0) return set_error(ED_EINVAL, "ed_lanczos_init: start vector has zero or non-finite norm");
    st->j = 0;
    return ED_OK;
}

int ed_lanczos_step(const ed_ham *h, ed_lanczos *st, void *ws, void *stream) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_lanczos_step");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    const Tile tl = resolve_tile(h);
    const WsLayout w = ws_layout(h, ws, st->max_steps);
    rc = step_dispatch(h, tl, st->f_prev, st->f_cur, st->f_next, st->a, st->b, nullptr, w, st->max_steps,
                       static_cast<hipStream_t>(stream));
    if (rc) return rc;
    rotate(st);
    return ED_OK;
}

int ed_lanczos_step_timed(const ed_ham *h, ed_lanczos *st, void *ws, void *stream, double *ms) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_lanczos_step_timed");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    if (!ms) return set_error(ED_EINVAL, "ed_lanczos_step_timed: ms is NULL");
    const Tile tl = resolve_tile(h);
    const WsLayout w = ws_layout(h, ws, st->max_steps);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[6] = {};
    for (int k = 0; k < 6; ++k) ED_HIP(hipEventCreate(&ev[k]));
    rc = step_dispatch(h, tl, st->f_prev, st->f_cur, st->f_next, st->a, st->b, nullptr, w, st->max_steps, s, ev);
    if (rc == ED_OK) rc = hip_check(hipEventSynchronize(ev[5]), "hipEventSynchronize");
    for (int k = 0; k < 5 && rc == ED_OK; ++k) {
        float t = 0.f;
        rc = hip_check(hipEventElapsedTime(&t, ev[k], ev[k + 1]), "hipEventElapsedTime");
        ms[k] = t;
    }
    for (int k = 0; k < 6; ++k) (void)hipEventDestroy(ev[k]);
    if (rc) return rc;
    rotate(st);
    return ED_OK;
}

int ed_lanczos_read(const ed_ham *h, const ed_lanczos *st, void *ws, void *stream, int32_t *steps, int32_t *status,
                    double *a_host, double *b_host) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_lanczos_read");
    if (rc) return rc;
    if (!steps || !status) return set_error(ED_EINVAL, "ed_lanczos_read: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout w = ws_layout(h, ws, st->max_steps);
    Hdr hh;
    rc = read_hdr(w, &hh, s);
    if (rc) return rc;
    if (hh.status == kInitBad) return set_error(ED_EINVAL, "ed_lanczos_read: the run was not initialised");
    *steps = hh.jdev;
    *status = hh.status == ED_BREAKDOWN ? ED_BREAKDOWN : (hh.jdev >= st->max_steps ? ED_NOT_CONVERGED : ED_OK);
    if (a_host && hh.jdev > 0) ED_HIP(hipMemcpyAsync(a_host, st->a, 8 * (size_t)hh.jdev, hipMemcpyDeviceToHost, s));
    if (b_host) ED_HIP(hipMemcpyAsync(b_host, st->b, 8 * (size_t)(hh.jdev + 1), hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    return ED_OK;
}

int ed_ground_energy(const ed_ham *h, ed_lanczos *st, const void *f1, double tol, int32_t check_every, void *ws,
                     void *stream, double *e0, int32_t *steps, double *a_host, double *b_host) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_ground_energy");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    if (!e0 || !steps) return set_error(ED_EINVAL, "ed_ground_energy: e0/steps are NULL");
    if (!f1 || f1 == st->f_cur) return set_error(ED_EINVAL, "ed_ground_energy: f1 must be a buffer other than f_cur");
    const int max_steps = st->max_steps;
    int chunk = std::max(1, check_every);
    chunk = ((chunk + 2) / 3) * 3;
    const Tile tl = resolve_tile(h);
    const WsLayout w = ws_layout(h, ws, max_steps);

    SideStream ss;
    rc = ss.open(static_cast<hipStream_t>(stream));
    if (rc) return rc;
    rc = init_impl(h, st, f1, w, ss.own);
    if (rc) return rc;
    Hdr hh;
    rc = read_hdr(w, &hh, ss.own);
    if (rc) return rc;
    if (hh.status != 0) return set_error(ED_EINVAL, "ed_ground_energy: start vector has zero or non-finite norm");
    st->j = 0;

    StepGraph sg;
    rc = capture_steps(h, tl, *st, w, chunk, ss.own, sg);
    if (rc) return rc;

    std::vector<double> a(max_steps), b(max_steps + 1), e(max_steps + 1, 0.0);
    int have = 0;            // steps whose E0 is known
    int launched = 0;
    int result = ED_NOT_CONVERGED;
    int stop_at = -1;
    while (true) {
        ED_HIP(hipGraphLaunch(sg.ge, ss.own));
        launched += chunk;
        rc = read_hdr(w, &hh, ss.own);
        if (rc) return rc;
        const int jd = hh.jdev;
        if (jd > have) {
            ED_HIP(hipMemcpyAsync(a.data(), st->a, 8 * (size_t)jd, hipMemcpyDeviceToHost, ss.own));
            ED_HIP(hipMemcpyAsync(b.data(), st->b, 8 * (size_t)(jd + 1), hipMemcpyDeviceToHost, ss.own));
            ED_HIP(hipStreamSynchronize(ss.own));
            for (int j = have + 1; j <= jd; ++j) {
                e[j] = tridiag_lowest(a.data(), b.data() + 1, j);
                if (tol > 0 && j >= 3 && std::fabs(e[j] - e[j - 1]) < tol && std::fabs(e[j - 1] - e[j - 2]) < tol) {
                    stop_at = j;
                    break;
                }
            }
            have = jd;
        }
        if (stop_at > 0) { result = ED_OK; break; }
        if (hh.status == ED_BREAKDOWN) { result = ED_BREAKDOWN; stop_at = jd; break; }
        if (jd >= max_steps) { result = tol > 0 ? ED_NOT_CONVERGED : ED_OK; stop_at = jd; break; }
        if (launched > 4 * max_steps + 3 * chunk) return set_error(ED_EDEVICE, "ed_ground_energy: no progress");
    }
    for (int k = 0; k < launched; ++k) rotate(st);
    st->j = launched;
    *e0 = e[stop_at];
    *steps = stop_at;
    if (a_host) std::copy(a.begin(), a.begin() + stop_at, a_host);
    if (b_host) std::copy(b.begin(), b.begin() + stop_at + 1, b_host);
    rc = ss.close();
    if (rc) return rc;
    return result;
}

int ed_ground_state(const ed_ham *h, ed_lanczos *st, const void *f1, int32_t m, void *v, void *ws, void *stream,
                    double *e0, int32_t *steps) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_ground_state");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    if (!v || !e0 || !steps || m < 1 || m > st->max_steps)
        return set_error(ED_EINVAL, "ed_ground_state: bad arguments (need 1 <= m <= max_steps)");
    if (v == st->f_prev || v == st->f_cur || v == st->f_next || v == f1)
        return set_error(ED_EINVAL, "ed_ground_state: v must not alias f1 or the Lanczos vectors");
    // pass 1: m steps (fewer on breakdown)
    ed_lanczos s1 = *st;
    s1.max_steps = m;
    std::vector<double> a(m), b(m + 1);
    int32_t k = 0;
    double e;
    rc = ed_ground_energy(h, &s1, f1, 0.0, 30, ws, stream, &e, &k, a.data(), b.data());
    if (rc < 0) return rc;
    std::vector<double> y(k);
    rc = ed_tridiag_lowest_vector(a.data(), b.data() + 1, k, &e, y.data());
    if (rc) return rc;
    // pass 2: replay the identical steps, accumulating v = sum_j y_j f_j
    hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout w = ws_layout(h, ws, m);
    ED_HIP(hipMemcpyAsync(w.y, y.data(), 8 * (size_t)k, hipMemcpyHostToDevice, s));
    const int64_t n = h->dim_up * h->dim_dn;
    ed_lanczos s2 = *st;
    rc = init_impl(h, &s2, f1, w, s);
    if (rc) return rc;
    if (h->dtype == ED_F64)
        hipLaunchKernelGGL(k_fill0<double>, dim3(upd_grid(n)), dim3(256), 0, s, (double *)v, n);
    else
        hipLaunchKernelGGL(k_fill0<float>, dim3(upd_grid(n)), dim3(256), 0, s, (float *)v, n);
    ED_LAUNCHED("k_fill0");
    const Tile tl = resolve_tile(h);
    for (int j = 0; j < k; ++j) {
        rc = step_dispatch(h, tl, s2.f_prev, s2.f_cur, s2.f_next, s2.a, s2.b, v, w, k, s);
        if (rc) return rc;
        rotate(&s2);
    }
    if (h->dtype == ED_F64) rc = norm_launch<double>((const double *)v, (double *)v, n, w, s2.b, 1, s);
    else rc = norm_launch<float>((const float *)v, (float *)v, n, w, s2.b, 1, s);
    if (rc) return rc;
    ED_HIP(hipStreamSynchronize(s));
    *e0 = e;
    *steps = k;
    st->f_prev = s2.f_prev;
    st->f_cur = s2.f_cur;
    st->f_next = s2.f_next;
    st->j = k;
    return ED_OK;
}

}  // extern "C"
