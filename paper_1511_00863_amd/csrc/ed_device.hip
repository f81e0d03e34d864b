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
#include <atomic>
#include <type_traits>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/ed.h"
#include "ed_common.h"
#include "ed_internal.h"
#include "ed_launch.h"

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
// workspace layout: [Hdr: 256 B][queue counters: 256 B][y: max_steps doubles]
//                   [part: P x 8 doubles][part2: 8192 doubles]
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
constexpr int kPartStride = 8;    // doubles per partial-sum slot
constexpr int kUpdBlocks = 8192;  // k_update / k_sumsq grid cap = part2 slots

static inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

struct WsLayout {
    Hdr *hdr;
    int *ctr;
    double *y;
    double *part;
    double *part2;
};

// k_down partial-sum slots: one per workgroup.  Rows too long for LDS are split
// into column blocks until the launch has kDownBlocks workgroups, so the grid
// is at most dim_up + kDownBlocks.
// partial-sum slots of the down part: one per workgroup (rows, column blocks
// of long rows, or the windowed kernel's row-block pairs)
static int64_t n_partial_slots(const ed_ham *h) {
    const int64_t base = std::max<int64_t>(h->dim_up, 1) + kDownBlocks;
    const int64_t nb = h->win_dn && h->win_cols > 0 ? (h->dim_dn + h->win_cols - 1) / h->win_cols : 0;
    return std::max(base, h->dim_up * nb);
}

static int64_t ws_bytes(const ed_ham *h, int32_t max_steps) {
    return 512 + align256(8 * (int64_t)std::max(max_steps, 1)) + align256(8 * kPartStride * n_partial_slots(h)) +
           8 * kUpdBlocks;
}

static WsLayout ws_layout(const ed_ham *h, void *ws, int32_t max_steps) {
    char *p = static_cast<char *>(ws);
    WsLayout l;
    l.hdr = reinterpret_cast<Hdr *>(p);
    p += 256;
    l.ctr = reinterpret_cast<int *>(p);
    p += 256;
    l.y = reinterpret_cast<double *>(p);
    p += align256(8 * (int64_t)std::max(max_steps, 1));
    l.part = reinterpret_cast<double *>(p);
    p += align256(8 * kPartStride * n_partial_slots(h));
    l.part2 = reinterpret_cast<double *>(p);
    return l;
}

__device__ __forceinline__ bool frozen(const Hdr *hdr, int max_steps) {
    return hdr->status != 0 || hdr->jdev >= max_steps;
}

// Which up-part tile a (R, NCH, E) variant runs: one row per wave with all
// chunks in scalar registers, two rows per wave (16-bit tables of at most 4
// chunks), or the chunk-at-a-time tile otherwise (32-bit tables of 8 chunks
// would not fit the scalar registers of the one-row kernel).
template <typename T, int R, int NCH, typename E>
__device__ __forceinline__ void up_tile_any(const T *__restrict__ x, T *__restrict__ out, const E *__restrict__ tab,
                                            int Dup, int Ddn, int W8, int rc, int s, int rci, T t) {
    if constexpr (R == 1 && (sizeof(E) == 2 || NCH <= 4))
        up_tile_wide<T, NCH>(x, out, tab, Dup, Ddn, W8, rc, s, rci, t);
    else if constexpr (R == 2 && NCH <= 4 && sizeof(E) == 2)
        up_tile_pair<T, NCH>(x, out, tab, Dup, Ddn, W8, rc, s, rci, t);
    else
        up_tile<T, R>(x, out, tab, Dup, Ddn, W8, rc, s, rci, t);
}

template <typename T, int R, int NCH, typename E>
__global__ __launch_bounds__(512) void k_up(const T *__restrict__ x, T *__restrict__ out,
                                            const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc,
                                            int n_stripes, int n_rc, int map, T t, const Hdr *__restrict__ hdr,
                                            int gate, int max_steps) {
    if (gate && frozen(hdr, max_steps)) return;
    int s, rci;
    if (map == 0) {
        const int g = blockIdx.x, xcd = g & 7, local = g >> 3;
        const int sl = local / n_rc;
        rci = local - sl * n_rc;
        s = sl * 8 + xcd;
    } else {
        s = blockIdx.x / n_rc;
        rci = blockIdx.x - s * n_rc;
    }
    if (s >= n_stripes) return;
    up_tile_any<T, R, NCH>(x, out, tab, Dup, Ddn, W8, rc, s, rci, t);
}

// k_upv: k_up's tiling with 64*V-column stripes (V columns per lane).
template <typename T, int V, int NCH, typename E>
__global__ __launch_bounds__(512) void k_upv(const T *__restrict__ x, T *__restrict__ out,
                                             const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc,
                                             int n_stripes, int n_rc, int map, T t, const Hdr *__restrict__ hdr,
                                             int gate, int max_steps) {
    if (gate && frozen(hdr, max_steps)) return;
    int s, rci;
    if (map == 0) {
        const int g = blockIdx.x, xcd = g & 7, local = g >> 3;
        const int sl = local / n_rc;
        rci = local - sl * n_rc;
        s = sl * 8 + xcd;
    } else {
        s = blockIdx.x / n_rc;
        rci = blockIdx.x - s * n_rc;
    }
    if (s >= n_stripes) return;
    up_tile_vec<T, V, NCH>(x, out, tab, Dup, Ddn, W8, rc, s, rci, t);
}

// k_up_q, persistent mapping (map 2): one queue per XCD holding the tiles of
// the stripes s = q (mod 8).  A workgroup reads the XCD it runs on from the
// XCC_ID hardware register, drains that XCD's queue (integer atomics), then
// helps the other queues, so every tile is processed whatever the dispatch.
template <typename T, int R, int NCH, typename E>
__global__ __launch_bounds__(512) void k_up_q(const T *__restrict__ x, T *__restrict__ out,
                                              const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc,
                                              int n_stripes, int n_rc, T t, int *__restrict__ ctr,
                                              const Hdr *__restrict__ hdr, int gate, int max_steps) {
    if (gate && frozen(hdr, max_steps)) return;
    __shared__ int tile_sh;
    const int mine = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u);
    for (int qi = 0; qi < 8; ++qi) {
        const int q = (mine + qi) & 7;
        const int ntiles = (q < n_stripes ? (n_stripes - q + 7) / 8 : 0) * n_rc;
        while (true) {
            if (threadIdx.x == 0) tile_sh = atomicAdd(&ctr[q], 1);
            __syncthreads();
            const int tq = tile_sh;
            __syncthreads();
            if (tq >= ntiles) break;
            const int sl = tq / n_rc;
            up_tile_any<T, R, NCH>(x, out, tab, Dup, Ddn, W8, rc, q + 8 * sl, tq - sl * n_rc, t);
        }
    }
}

__global__ void k_ctr_reset(int *ctr, const Hdr *hdr, int gate, int max_steps) {
    if (gate && frozen(hdr, max_steps)) return;
    if (threadIdx.x < 8) ctr[threadIdx.x] = 0;
}

// float rows are half the size: three 512-thread workgroups fit a CU's LDS,
// which needs at most 80 VGPRs (6 waves per SIMD).  32-bit tables double the
// registers of the prefetched table chunks: workgroups of at most 512 threads
// (256 VGPRs) and no occupancy target.
template <typename T, int MODE, bool LDS, int NCH, bool MULTI, typename E, bool IO = true, bool WCH = false>
__global__ __launch_bounds__(sizeof(E) == 4 ? 512 : 1024)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NCH <= 4 && sizeof(E) == 2 ? 6 : 1)))
void k_down(const T *__restrict__ x, T *__restrict__ io, const T *__restrict__ p,
                                               const E *__restrict__ tab,
                                               const uint64_t *__restrict__ st_up,
                                               const uint64_t *__restrict__ st_dn, int Dup, int Ddn, int W8,
                                               int rpb, int csplit, T t, T U, const double *__restrict__ bvec,
                                               const Hdr *__restrict__ hdr, double *__restrict__ partials,
                                               int max_steps, const uint32_t *__restrict__ wch) {
    static_assert(!WCH || !MULTI, "per-wavefront chunk counts: one row per workgroup");
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
    // rows staged in LDS: rpb whole rows per workgroup; otherwise one row, or
    // one of its csplit column blocks (64-column aligned)
    int rblk = blockIdx.x, i0 = 0, iend = 0;
    if constexpr (!LDS) {
        rblk = blockIdx.x / csplit;
        const int cb = blockIdx.x - rblk * csplit;
        const int cw = ((Ddn + csplit - 1) / csplit + 63) & ~63;
        i0 = min(Ddn, cb * cw);
        iend = min(Ddn, i0 + cw);
    }
    const int r0 = rblk * rpb;
    const int nr = min(rpb, Dup - r0);
    if constexpr (LDS) iend = nr * Ddn;
    const int64_t base = (int64_t)r0 * Ddn;
    // one staged row is followed by a zero, the target of padding entries
    constexpr bool ZS = LDS && !MULTI;
    if (LDS) {
        stage_rows<T>(x + base, xs, nr * Ddn);
        if (ZS && threadIdx.x == 0) xs[Ddn] = T(0);
        __syncthreads();
    }
    constexpr int NV = MODE == 2 ? 5 : 1;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    down_rows<T, MODE, NCH, MULTI, IO, ZS, E, 0, WCH>(LDS ? xs : x + base, io, p, tab, st_up + r0, st_dn, Ddn, W8,
                                                      i0, iend, base, t, U, sig, cprev, MODE != 0 && has_prev, s,
                                                      0u, 0u, wch);
    if (MODE != 0) {
        double tot[NV];
        block_sum<NV>(s, tot);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NV; ++k) partials[(int64_t)blockIdx.x * kPartStride + k] = tot[k];
    }
}

// k_down with two rows per workgroup (down_rows2): rows 2b and 2b + 1 staged
// in LDS at 0 and S (S = the row length plus one, rounded up to 4 elements),
// each followed by a zero.  One table chunk load per column serves both rows.
// WCH: each wavefront reads only its own count of table chunks (wch).
template <typename T, int MODE, int NCH, typename E, bool WCH = false>
__global__ __launch_bounds__(sizeof(E) == 4 ? 512 : 1024)
void k_down2(const T *__restrict__ x, T *__restrict__ io, const T *__restrict__ p, const E *__restrict__ tab,
             const uint64_t *__restrict__ st_up, const uint64_t *__restrict__ st_dn, int Dup, int Ddn, int W8, int S,
             T t, T U, const double *__restrict__ bvec, const Hdr *__restrict__ hdr, double *__restrict__ partials,
             int max_steps, const uint32_t *__restrict__ wch) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *x0 = reinterpret_cast<T *>(smem);
    T *x1 = x0 + S;
    bool has_prev = false;
    T sig = T(1), cprev = T(0);
    if (MODE != 0) {
        if (frozen(hdr, max_steps)) return;
        const int j = hdr->jdev;
        has_prev = j > 0;
        sig = static_cast<T>(hdr->sig_cur);
        cprev = static_cast<T>(bvec[j] * hdr->sig_prev);
    }
    const int r0 = 2 * blockIdx.x;
    const bool two = r0 + 1 < Dup;
    const int64_t base = (int64_t)r0 * Ddn;
    stage_rows<T, true>(x + base, x0, Ddn);
    if (two) stage_rows<T, true>(x + base + Ddn, x1, Ddn);
    if (threadIdx.x == 0) {
        x0[Ddn] = T(0);
        x1[Ddn] = T(0);
    }
    __syncthreads();
    constexpr int NV = MODE == 2 ? 5 : 1;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    down_rows2<T, MODE, NCH, E, WCH>(x0, two ? x1 : x0, io, p, tab, st_up[r0], two ? st_up[r0 + 1] : 0ull, two, st_dn,
                                     Ddn, W8, base, t, U, sig, cprev, MODE != 0 && has_prev, s, wch);
    if (MODE != 0) {
        double tot[NV];
        block_sum<NV>(s, tot);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NV; ++k) partials[(int64_t)blockIdx.x * kPartStride + k] = tot[k];
    }
}

// k_down for rows too long for LDS, by column blocks (ed_row_windows): the
// workgroup of (row r, block b) stages x[r, lo_b..hi_b), the block's states
// and all their neighbours, in LDS with a zero after it, and runs the block's
// columns as the one-row kernel does (the same q bits).  win: the blocks'
// (lo, hi) pairs; wcols: states per block; nblk blocks per row; wmax: the
// LDS room (elements) before the zero.  A pair that does not fit that room or
// does not cover its block is not staged: that block gathers from global
// memory as the kernel for long rows does (the same bits again).  REL: a
// staged block reads rtab, the table with 16-bit window-relative columns
// (ed_pack_tables_windowed), instead of tab; with WCH each of its wavefronts
// reads only its own count of table chunks (wch, per 64 columns).
template <typename T, int MODE, int NCH, typename E, bool REL = false, bool WCH = false>
__global__ __launch_bounds__(sizeof(E) == 4 ? 512 : 1024)
void k_down_win(const T *__restrict__ x, T *__restrict__ io, const T *__restrict__ p, const E *__restrict__ tab,
                const uint64_t *__restrict__ st_up, const uint64_t *__restrict__ st_dn, int Dup, int Ddn, int W8,
                const int32_t *__restrict__ win, int wcols, int nblk, int wmax, T t, T U,
                const double *__restrict__ bvec, const Hdr *__restrict__ hdr, double *__restrict__ partials,
                int max_steps, const uint16_t *__restrict__ rtab, const uint32_t *__restrict__ wch) {
    static_assert(!WCH || REL, "per-wavefront chunk counts: the window-relative table only");
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
    const int r = blockIdx.x / nblk, b = blockIdx.x - r * nblk;
    const int lo = win[2 * b], hi = win[2 * b + 1];
    const int c0 = b * wcols, c1 = min(Ddn, c0 + wcols);
    const int64_t base = (int64_t)r * Ddn;
    const bool staged = lo >= 0 && lo <= c0 && hi >= c1 && hi <= Ddn && hi - lo <= wmax;
    if (staged) {
        stage_rows<T>(x + base + lo, xs, hi - lo);
        if (threadIdx.x == 0) xs[hi - lo] = T(0);
        __syncthreads();
    }
    constexpr int NV = MODE == 2 ? 5 : 1;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    if (REL && staged)
        down_rows<T, MODE, NCH, false, true, true, uint16_t, 2, WCH>(xs, io, p, rtab, st_up + r, st_dn, Ddn, W8, c0,
                                                                     c1, base, t, U, sig, cprev,
                                                                     MODE != 0 && has_prev, s, (unsigned)lo,
                                                                     (unsigned)(hi - lo), wch);
    else if (staged)
        down_rows<T, MODE, NCH, false, true, true, E, 1>(xs, io, p, tab, st_up + r, st_dn, Ddn, W8, c0, c1, base, t,
                                                         U, sig, cprev, MODE != 0 && has_prev, s, (unsigned)lo,
                                                         (unsigned)(hi - lo));
    else
        down_rows<T, MODE, NCH, false, true, false, E>(x + base, io, p, tab, st_up + r, st_dn, Ddn, W8, c0, c1, base, t,
                                                       U, sig, cprev, MODE != 0 && has_prev, s);
    if (MODE != 0) {
        double tot[NV];
        block_sum<NV>(s, tot);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < NV; ++k) partials[(int64_t)blockIdx.x * kPartStride + k] = tot[k];
    }
}

// ---------------------------------------------------------------------------
// Complex amplitudes.  Vectors are interleaved (re, im) pairs; every kernel of
// the step other than these two treats them as real arrays of 2D values, which
// is exact: a_j = Re(f_j^dagger q) is the real dot product of the pairs and the
// update coefficients are real.  A table entry is (col << 6) | index into the
// species' 64 complex amplitudes (sign included), padding 0xFFFFFFFF.
template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

// Up part, t * (H_up (x) I) x: one row per wave on 64-column stripes (XCD
// round-robin as in k_up); the row's entries are wave-uniform scalar loads,
// so its amplitudes are too; the 8 gathers of a chunk are issued together.
template <typename T>
__global__ __launch_bounds__(256) void k_upc(const typename Cplx<T>::type *__restrict__ x,
                                             typename Cplx<T>::type *__restrict__ out,
                                             const uint32_t *__restrict__ tab, const double *__restrict__ amp,
                                             int Dup, int Ddn, int W8, int rc, int n_stripes, int n_rc, T t,
                                             const Hdr *__restrict__ hdr, int gate, int max_steps) {
    using T2 = typename Cplx<T>::type;
    if (gate && frozen(hdr, max_steps)) return;
    const int g = blockIdx.x, xcd = g & 7, local = g >> 3;
    const int sl = local / n_rc;
    const int rci = local - sl * n_rc;
    const int s = sl * 8 + xcd;
    if (s >= n_stripes) return;
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = s * 64 + lane;
    const bool cok = c < Ddn;
    const T2 *xc = x + (cok ? c : 0);
    const int r1 = min(Dup, (rci + 1) * rc);
    const int nch = W8 >> 3;
    for (int r = rci * rc + wave; r < r1; r += nwave) {
        const uint32_t *row = tab + (int64_t)r * W8;
        T re = T(0), im = T(0);
        // two chunks (16 gathers) in flight per pass; a second chunk beyond the row's nch reads the next 8
        // entries of the table (still inside it: the interleaved half follows) and counts as padding
        for (int k8 = 0; k8 < nch; k8 += 2) {
            uint32_t e[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = row[8 * k8 + k];
                e[k] = (k < 8 || k8 + 1 < nch) ? v : 0xFFFFFFFFu;
            }
            if (e[0] == 0xFFFFFFFFu) break;   // ascending columns, padding at the end
            T2 v[16];
            T ar[16], ai[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const bool pk = e[k] != 0xFFFFFFFFu;
                const unsigned ia = pk ? (e[k] & 63u) : 0u;
                v[k] = xc[(int64_t)(pk ? (e[k] >> 6) : 0u) * Ddn];
                ar[k] = pk ? static_cast<T>(amp[2 * ia]) : T(0);
                ai[k] = pk ? static_cast<T>(amp[2 * ia + 1]) : T(0);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                re = fma_t(ar[k], v[k].x, re);
                re = fma_t(-ai[k], v[k].y, re);
                im = fma_t(ar[k], v[k].y, im);
                im = fma_t(ai[k], v[k].x, im);
            }
        }
        if (cok) {
            T2 o;
            o.x = t * re;
            o.y = t * im;
            out[(int64_t)r * Ddn + c] = o;
        }
    }
}

// Down part and the rest of the step row by row, as k_down: q = sig * (io +
// t * (I (x) H_dn) x + U Docc x) - cprev * p, in place on io, with partial
// dot products of the (re, im) pairs.  One row per workgroup, staged in LDS
// when it fits (after the amplitude table, whose slot kAmpSlots is zero and
// serves padding); longer rows are split into column blocks and gathered
// from global memory.
template <typename T, int MODE, bool LDS>
__global__ __launch_bounds__(1024) void k_downc(const typename Cplx<T>::type *__restrict__ x,
                                               typename Cplx<T>::type *__restrict__ io,
                                               const typename Cplx<T>::type *__restrict__ p,
                                               const uint32_t *__restrict__ tab, const double *__restrict__ amp,
                                               const uint64_t *__restrict__ st_up,
                                               const uint64_t *__restrict__ st_dn, int Ddn, int W8, int csplit,
                                               T t, T U, const double *__restrict__ bvec,
                                               const Hdr *__restrict__ hdr, double *__restrict__ partials,
                                               int max_steps) {
    using T2 = typename Cplx<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    T2 *amp_s = reinterpret_cast<T2 *>(smem);
    T2 *xs = amp_s + kAmpSlots + 2;   // kAmpSlots + 1 used; one more keeps 16-byte alignment for float2
    bool use_p = false;
    T sig = T(1), cprev = T(0);
    if (MODE != 0) {
        if (frozen(hdr, max_steps)) return;
        const int j = hdr->jdev;
        use_p = j > 0;
        sig = static_cast<T>(hdr->sig_cur);
        cprev = static_cast<T>(bvec[j] * hdr->sig_prev);
    }
    int r = blockIdx.x, i0 = 0, iend = Ddn;
    if constexpr (!LDS) {
        r = blockIdx.x / csplit;
        const int cb = blockIdx.x - r * csplit;
        const int cw = ((Ddn + csplit - 1) / csplit + 63) & ~63;
        i0 = min(Ddn, cb * cw);
        iend = min(Ddn, i0 + cw);
    }
    const int64_t base = (int64_t)r * Ddn;
    for (int k = threadIdx.x; k <= kAmpSlots; k += blockDim.x) {   // amp is NULL for a species without hopping
        T2 a;
        a.x = (amp && k < kAmpSlots) ? static_cast<T>(amp[2 * k]) : T(0);
        a.y = (amp && k < kAmpSlots) ? static_cast<T>(amp[2 * k + 1]) : T(0);
        amp_s[k] = a;
    }
    if constexpr (LDS)
        for (int k = threadIdx.x; k < Ddn; k += blockDim.x) xs[k] = x[base + k];
    __syncthreads();
    const T2 *row = LDS ? xs : x + base;
    const Chunk8<uint32_t> *til = reinterpret_cast<const Chunk8<uint32_t> *>(tab + (int64_t)Ddn * W8);
    const int nch = W8 >> 3;
    const uint64_t su = st_up[r];
    constexpr int NV = MODE == 2 ? 5 : 1;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int c = i0 + threadIdx.x; c < iend; c += blockDim.x) {
        // the epilogue's global operands first, so they are in flight during the gathers
        const T2 iov = io[base + c];
        const uint64_t sdv = st_dn[c];
        T2 pv;
        pv.x = T(0);
        pv.y = T(0);
        if (MODE != 0) {
            const T2 pl = p[base + c];   // always a valid element; zeroed when there is no f_{j-1}
            pv.x = keep_or_zero(pl.x, use_p);
            pv.y = keep_or_zero(pl.y, use_p);
        }
        T re = T(0), im = T(0);
        if (nch > 0) {   // a species without hopping may pass no table
            Chunk8<uint32_t> q = table_chunk<8, uint32_t>(til, 0, nch, Ddn, c);
            for (int k8 = 0; k8 < nch; ++k8) {
                const Chunk8<uint32_t> qn = table_chunk<8, uint32_t>(til, k8 + 1, nch, Ddn, c);   // next chunk
                if (!__any(!is_pad<uint32_t>(entry(q, 0)))) break;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const unsigned e = entry(q, k);
                    const bool pk = !is_pad<uint32_t>(e);
                    const T2 v = row[pk ? (int)(e >> 6) : 0];
                    const T2 a = amp_s[pk ? (int)(e & 63u) : kAmpSlots];
                    re = fma_t(a.x, v.x, re);
                    re = fma_t(-a.y, v.y, re);
                    im = fma_t(a.x, v.y, im);
                    im = fma_t(a.y, v.x, im);
                }
                q = qn;
            }
        }
        const T2 xv = row[c];
        const T nd = static_cast<T>(__popcll(su & sdv));
        T qr = iov.x + t * re + U * nd * xv.x;
        T qi = iov.y + t * im + U * nd * xv.y;
        if (MODE != 0) {
            qr *= sig;
            qi *= sig;
            qr -= cprev * pv.x;   // pv is zero without f_{j-1}
            qi -= cprev * pv.y;
        }
        T2 qv;
        qv.x = qr;
        qv.y = qi;
        io[base + c] = qv;
        if (MODE != 0) {
            s[0] += (double)qr * xv.x + (double)qi * xv.y;
            if constexpr (MODE == 2) {
                s[1] += (double)qr * pv.x + (double)qi * pv.y;
                s[2] += (double)xv.x * xv.x + (double)xv.y * xv.y;
                s[3] += (double)xv.x * pv.x + (double)xv.y * pv.y;
                s[4] += (double)pv.x * pv.x + (double)pv.y * pv.y;
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
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // four independent elements per trip keep more loads in flight
    for (; i + 3 * stride < n; i += 4 * stride) {
        double xv[4], qv[4], pv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xv[u] = x[i + u * stride];
            qv[u] = q[i + u * stride];
        }
        if (cp != 0.0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) pv[u] = p[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T st = static_cast<T>(qv[u] - cx * xv[u] - cp * pv[u]);
            q[i + u * stride] = st;
            const double sd = st;
            s[0] += sd * sd;
            if (v) v[i + u * stride] = static_cast<T>((double)v[i + u * stride] + yj * xv[u]);
        }
    }
    for (; i < n; i += stride) {
        const double xv = x[i];
        const double pv = cp != 0.0 ? (double)p[i] : 0.0;
        const T st = static_cast<T>((double)q[i] - cx * xv - cp * pv);
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
// mode 1: vinv = +-1/|v|, the sign making gauge_val * vinv >= 0 (gauge fix).
__global__ __launch_bounds__(1024) void k_init_norm(const double *__restrict__ part2, int n, Hdr *hdr, double *b,
                                                    int mode, double gauge_sign) {
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
        hdr->vinv = ok ? gauge_sign / sqrt(n2) : 0.0;
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
static int grid_for(int64_t n, int block, int cap = 4096) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Launch shape of k_down: rows per workgroup (LDS staging) or, for rows too
// long for LDS, one row per workgroup split into csplit column blocks.
struct DownShape { bool lds; int rpb, csplit, grid; bool pair, win; };

// LDS bytes of k_downc's amplitude table (kAmpSlots + 1 values, padded)
static int64_t complex_amp_lds(const ed_ham *h) { return (int64_t)(kAmpSlots + 2) * 2 * elem_size(h); }

// Row stride of the two-row down kernel in LDS: the row, its zero, rounded up
// to 4 elements (16 bytes of float, 32 of double).
static int64_t pair_stride(const ed_ham *h) { return (h->dim_dn + 1 + 3) & ~int64_t(3); }
// The two-row down kernel: asked for by the tile, real instances where both
// species hop, at least two rows, and both rows (with their zeros) in LDS.
static bool pair_rows(const ed_ham *h, const Tile &tl) {
    return tl.dn_pair && !h->cplx && h->w_up > 0 && h->w_dn > 0 && h->dim_up >= 2 &&
           (pair_stride(h) + h->dim_dn + 1) * elem_size(h) <= kLdsBudget;
}

// Column blocks of the down species' windows (0 without windows).
static int64_t win_blocks(const ed_ham *h) {
    return h->win_dn && h->win_cols > 0 ? (h->dim_dn + h->win_cols - 1) / h->win_cols : 0;
}

// The windowed down kernel: asked for by the tile, real instances where both
// species hop, down tables of at most 4 chunks, rows too long for LDS and
// every block's window (with its zero) in LDS.
static bool win_rows(const ed_ham *h, const Tile &tl) {
    return tl.dn_win && win_blocks(h) > 0 && !h->cplx && h->w_up > 0 && h->w_dn > 0 && (h->w_dn >> 3) <= 4 &&
           h->dim_dn * elem_size(h) > kLdsBudget && h->win_max > 0 && h->win_max <= h->dim_dn &&
           (h->win_max + 1) * elem_size(h) <= kLdsBudget;
}

static DownShape down_shape(const ed_ham *h, const Tile &tl) {
    DownShape d;
    d.pair = false;
    d.win = false;
    if (win_rows(h, tl)) {
        d.win = true;
        d.lds = false;
        d.rpb = 1;
        d.csplit = (int)win_blocks(h);
        d.grid = (int)(h->dim_up * d.csplit);
        return d;
    }
    if (pair_rows(h, tl)) {
        d.pair = true;
        d.lds = true;
        d.rpb = 2;
        d.csplit = 1;
        d.grid = (int)((h->dim_up + 1) / 2);
        return d;
    }
    const int64_t row_bytes = h->dim_dn * (int64_t)elem_size(h) * (h->cplx ? 2 : 1);
    if (h->cplx) {   // one row per workgroup
        d.lds = row_bytes + complex_amp_lds(h) <= kLdsBudget;
        d.rpb = 1;
    } else {
        d.lds = row_bytes * tl.dn_rpb <= kLdsBudget;
        d.rpb = d.lds ? tl.dn_rpb : 1;
    }
    d.csplit = 1;
    if (!d.lds) {
        const int64_t want = (kDownBlocks + h->dim_up - 1) / h->dim_up;
        const int64_t most = (h->dim_dn + tl.dn_block - 1) / tl.dn_block;
        d.csplit = (int)std::max<int64_t>(1, std::min(want, most));
    }
    d.grid = (int)((h->dim_up + d.rpb - 1) / d.rpb) * d.csplit;
    return d;
}

template <typename T, int R, int NCH, typename E>
static int up_queue_grid(int block) {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(k_up_q<T, R, NCH, E>), block,
                                                     0) != hipSuccess)
        return 0;
    cached = std::max(1, ncu * std::max(1, occ));
    return cached;
}

template <typename T, int R, int NCH, typename E>
static int launch_up_r(const ed_ham *h, const Tile &tl, const T *x, T *out, int *ctr, const Hdr *hdr, int gate,
                       int max_steps, hipStream_t s) {
    constexpr int w = 64 / R;
    const E *tab = static_cast<const E *>(h->tab_up);
    const int n_stripes = (int)((h->dim_dn + w - 1) / w);
    const int n_rc = (int)((h->dim_up + tl.up_rc - 1) / tl.up_rc);
    const T t = static_cast<T>(h->t);
    if (tl.up_map == 2) {
        if (!ctr) return set_error(ED_EINVAL, "k_up_q needs the workspace");
        const int total = n_stripes * n_rc;
        int grid = up_queue_grid<T, R, NCH, E>(tl.up_block);
        if (grid <= 0) return set_error(ED_EDEVICE, "occupancy query for k_up_q failed");
        grid = std::min(grid, total);
        hipLaunchKernelGGL(k_ctr_reset, dim3(1), dim3(64), 0, s, ctr, hdr, gate, max_steps);
        ED_LAUNCHED("k_ctr_reset");
        hipLaunchKernelGGL((k_up_q<T, R, NCH, E>), dim3(grid), dim3(tl.up_block), 0, s, x, out, tab, (int)h->dim_up,
                           (int)h->dim_dn, h->w_up, tl.up_rc, n_stripes, n_rc, t, ctr, hdr, gate, max_steps);
        ED_LAUNCHED("k_up_q");
        return ED_OK;
    }
    const int64_t grid = tl.up_map == 0 ? 8LL * n_rc * ((n_stripes + 7) / 8) : (int64_t)n_rc * n_stripes;
    if (grid > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "k_up grid too large");
    hipLaunchKernelGGL((k_up<T, R, NCH, E>), dim3((unsigned)grid), dim3(tl.up_block), 0, s, x, out, tab,
                       (int)h->dim_up, (int)h->dim_dn, h->w_up, tl.up_rc, n_stripes, n_rc, tl.up_map, t, hdr, gate,
                       max_steps);
    ED_LAUNCHED("k_up");
    return ED_OK;
}

template <typename T, typename E>
static int launch_up_e(const ed_ham *h, const Tile &tl, const T *x, T *out, int *ctr, const Hdr *hdr, int gate,
                       int max_steps, hipStream_t s) {
    if (h->w_up == 0) {   // no up hopping: out = 0, unless the down part does not read it
        if (!down_shape(h, tl).lds) return ED_OK;
        hipLaunchKernelGGL(k_fill0<T>, dim3(grid_for(h->dim_up * h->dim_dn, 256)), dim3(256), 0, s, out,
                           h->dim_up * h->dim_dn);
        ED_LAUNCHED("k_fill0");
        return ED_OK;
    }
    if (tl.up_wlog2 >= 7) {   // V columns per lane (resolve_tile_id guarantees W8 <= 32 and aligned rows)
        const int w = 1 << tl.up_wlog2;
        const int n_stripes = (int)((h->dim_dn + w - 1) / w);
        const int n_rc = (int)((h->dim_up + tl.up_rc - 1) / tl.up_rc);
        const int64_t grid = tl.up_map == 0 ? 8LL * n_rc * ((n_stripes + 7) / 8) : (int64_t)n_rc * n_stripes;
        if (grid > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "k_upv grid too large");
        const T t = static_cast<T>(h->t);
        const int map = tl.up_map == 0 ? 0 : 1;
        const int nc = nch_class(h->w_up >> 3);
#define ED_UPV(V, N)                                                                                          \
    hipLaunchKernelGGL((k_upv<T, V, N, E>), dim3((unsigned)grid), dim3(tl.up_block), 0, s, x, out,              \
                       static_cast<const E *>(h->tab_up),                                                      \
                       (int)h->dim_up, (int)h->dim_dn, h->w_up, tl.up_rc, n_stripes, n_rc, map, t, hdr, gate,  \
                       max_steps)
        if constexpr (sizeof(T) == 4 && sizeof(E) == 2) {
            if (tl.up_wlog2 == 8) {
                if (nc == 1) ED_UPV(4, 1); else if (nc == 2) ED_UPV(4, 2); else ED_UPV(4, 4);
                ED_LAUNCHED("k_upv");
                return ED_OK;
            }
        }
        if (nc == 1) ED_UPV(2, 1); else if (nc == 2) ED_UPV(2, 2); else ED_UPV(2, 4);
#undef ED_UPV
        ED_LAUNCHED("k_upv");
        return ED_OK;
    }
    switch (tl.up_wlog2) {
    case 6:
        switch (nch_class(h->w_up >> 3)) {
        case 1: return launch_up_r<T, 1, 1, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        case 2: return launch_up_r<T, 1, 2, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        case 4: return launch_up_r<T, 1, 4, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        default: return launch_up_r<T, 1, 8, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        }
    case 5:
        if constexpr (sizeof(E) == 4)   // chunk-at-a-time tile: one variant serves every width
            return launch_up_r<T, 2, 8, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        switch (nch_class(h->w_up >> 3)) {
        case 1: return launch_up_r<T, 2, 1, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        case 2: return launch_up_r<T, 2, 2, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        case 4: return launch_up_r<T, 2, 4, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        default: return launch_up_r<T, 2, 8, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
        }
    default: return launch_up_r<T, 4, 1, E>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
    }
}

template <typename T>
static int launch_up_c(const ed_ham *h, const Tile &tl, const T *x, T *out, const Hdr *hdr, int gate,
                       int max_steps, hipStream_t s) {
    using T2 = typename Cplx<T>::type;
    const int64_t n = 2 * h->dim_up * h->dim_dn;
    if (h->w_up == 0) {   // no up hopping: out = 0 (k_downc adds it)
        hipLaunchKernelGGL(k_fill0<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, out, n);
        ED_LAUNCHED("k_fill0");
        return ED_OK;
    }
    const int n_stripes = (int)((h->dim_dn + 63) / 64);
    const int n_rc = (int)((h->dim_up + tl.up_rc - 1) / tl.up_rc);
    const int64_t grid = 8LL * n_rc * ((n_stripes + 7) / 8);
    if (grid > 0x7fffffffLL) return set_error(ED_EOVERFLOW, "k_upc grid too large");
    hipLaunchKernelGGL((k_upc<T>), dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const T2 *>(x),
                       reinterpret_cast<T2 *>(out), static_cast<const uint32_t *>(h->tab_up), h->amp_up,
                       (int)h->dim_up, (int)h->dim_dn, h->w_up, tl.up_rc, n_stripes, n_rc, static_cast<T>(h->t), hdr,
                       gate, max_steps);
    ED_LAUNCHED("k_upc");
    return ED_OK;
}

template <typename T>
static int launch_up(const ed_ham *h, const Tile &tl, const T *x, T *out, int *ctr, const Hdr *hdr, int gate,
                     int max_steps, hipStream_t s) {
    if (h->cplx) return launch_up_c<T>(h, tl, x, out, hdr, gate, max_steps, s);
    if (wide_up(h)) return launch_up_e<T, uint32_t>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
    return launch_up_e<T, uint16_t>(h, tl, x, out, ctr, hdr, gate, max_steps, s);
}

template <typename T, int MODE, bool LDS, int NCH, typename E, bool IO = true, bool WCH = false>
static void launch_down_k(const ed_ham *h, const Tile &tl, int grid, int rpb, int csplit, size_t shm, const T *x,
                          T *io, const T *p, const double *bvec, const Hdr *hdr, double *part, int max_steps,
                          hipStream_t s) {
    const E *tab = static_cast<const E *>(h->tab_dn);
    if constexpr (WCH)
        hipLaunchKernelGGL((k_down<T, MODE, LDS, NCH, false, E, IO, true>), dim3(grid), dim3(tl.dn_block), shm, s,
                           x, io, p, tab, h->st_up, h->st_dn, (int)h->dim_up, (int)h->dim_dn, h->w_dn, rpb, csplit,
                           static_cast<T>(h->t), static_cast<T>(h->U), bvec, hdr, part, max_steps, h->wch_dn);
    else if (rpb > 1)
        hipLaunchKernelGGL((k_down<T, MODE, LDS, NCH, true, E, IO>), dim3(grid), dim3(tl.dn_block), shm, s, x, io, p,
                           tab, h->st_up, h->st_dn, (int)h->dim_up, (int)h->dim_dn, h->w_dn, rpb, csplit,
                           static_cast<T>(h->t), static_cast<T>(h->U), bvec, hdr, part, max_steps, nullptr);
    else
        hipLaunchKernelGGL((k_down<T, MODE, LDS, NCH, false, E, IO>), dim3(grid), dim3(tl.dn_block), shm, s, x, io, p,
                           tab, h->st_up, h->st_dn, (int)h->dim_up, (int)h->dim_dn, h->w_dn, rpb, csplit,
                           static_cast<T>(h->t), static_cast<T>(h->U), bvec, hdr, part, max_steps, nullptr);
}

template <typename T, int MODE, typename E>
static int launch_down_e(const ed_ham *h, const Tile &tl, const T *x, T *io, const T *p, const double *bvec,
                         const Hdr *hdr, double *part, int max_steps, hipStream_t s) {
    const DownShape d = down_shape(h, tl);
    const bool lds = d.lds;
    const int rpb = d.rpb, grid = d.grid, cs = d.csplit;
    // rows plus one slot (the zero after a single row), 16-byte granular
    const size_t shm = lds ? (size_t)(h->dim_dn * (int64_t)sizeof(T) * rpb) + 16 : 0;
    const int nch = h->w_dn >> 3;
    if (d.win) {
        const size_t shmw = (size_t)((h->win_max + 1) * (int64_t)sizeof(T) + 15) & ~size_t(15);
        const E *tab = static_cast<const E *>(h->tab_dn);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(tl.dn_block), shmw, s, x, io, p, tab, h->st_up, h->st_dn,
                               (int)h->dim_up, (int)h->dim_dn, h->w_dn, h->win_dn, h->win_cols, cs, h->win_max,
                               static_cast<T>(h->t), static_cast<T>(h->U), bvec, hdr, part, max_steps, h->win_tab,
                               h->wch_dn);
        };
        // a 32-bit table has a 16-bit window-relative copy when the windows allow it; on it a wavefront
        // reads only its own count of table chunks when the species carries them
        const bool rel = sizeof(E) == 4 && h->win_tab != nullptr;
        const bool wc = rel && h->wch_dn != nullptr;
        if (nch <= 2)
            wc ? go(k_down_win<T, MODE, 2, E, true, true>)
               : (rel ? go(k_down_win<T, MODE, 2, E, true>) : go(k_down_win<T, MODE, 2, E>));
        else
            wc ? go(k_down_win<T, MODE, 4, E, true, true>)
               : (rel ? go(k_down_win<T, MODE, 4, E, true>) : go(k_down_win<T, MODE, 4, E>));
        ED_LAUNCHED("k_down_win");
        return ED_OK;
    }
    if (d.pair) {
        const int S = (int)pair_stride(h);
        const size_t shm2 = (size_t)(S + h->dim_dn + 1) * sizeof(T);
        const E *tab = static_cast<const E *>(h->tab_dn);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(tl.dn_block), shm2, s, x, io, p, tab, h->st_up, h->st_dn,
                               (int)h->dim_up, (int)h->dim_dn, h->w_dn, S, static_cast<T>(h->t),
                               static_cast<T>(h->U), bvec, hdr, part, max_steps, h->wch_dn);
        };
        if (nch <= 2) go(k_down2<T, MODE, 2, E>);
        else if (nch <= 4) h->wch_dn && nch > 2 ? go(k_down2<T, MODE, 4, E, true>) : go(k_down2<T, MODE, 4, E>);
        else go(k_down2<T, MODE, 8, E>);
        ED_LAUNCHED("k_down2");
        return ED_OK;
    }
    if (!lds && h->w_up == 0) {   // one species: no up part to add (launch_up wrote nothing)
        // with per-wavefront chunk counts, each wavefront reads only the table chunks its columns need;
        // not for FP64 on 32-bit tables of more than 4 chunks, where that variant (two waves per SIMD) ran
        // slower although it read fewer bytes
        auto one = [&](auto nc, auto wc) {
            launch_down_k<T, MODE, false, decltype(nc)::value, E, false, decltype(wc)::value>(
                h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        };
        using W0 = std::false_type;
        using W1 = std::true_type;
        const bool wc = h->wch_dn != nullptr && !(sizeof(T) == 8 && sizeof(E) == 4 && nch > 4);
        if (nch == 0) {
            one(std::integral_constant<int, 0>(), W0());
        } else {
            if constexpr (sizeof(E) == 4) {
                if (nch <= 2) wc ? one(std::integral_constant<int, 2>(), W1()) : one(std::integral_constant<int, 2>(), W0());
                else if (nch <= 4) wc ? one(std::integral_constant<int, 4>(), W1()) : one(std::integral_constant<int, 4>(), W0());
                else wc ? one(std::integral_constant<int, 8>(), W1()) : one(std::integral_constant<int, 8>(), W0());
            } else {
                wc ? one(std::integral_constant<int, 8>(), W1()) : one(std::integral_constant<int, 8>(), W0());
            }
        }
        ED_LAUNCHED("k_down");
        return ED_OK;
    }
    if constexpr (sizeof(E) == 4) {   // no one-size variant without LDS: its chunk registers would spill
        if (!lds && nch == 0) launch_down_k<T, MODE, false, 0, E>(h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        else if (!lds && nch <= 2) launch_down_k<T, MODE, false, 2, E>(h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        else if (!lds && nch <= 4) launch_down_k<T, MODE, false, 4, E>(h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        else if (!lds) launch_down_k<T, MODE, false, 8, E>(h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        else if (nch == 0) launch_down_k<T, MODE, true, 0, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else if (nch <= 2) launch_down_k<T, MODE, true, 2, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else if (nch <= 4) launch_down_k<T, MODE, true, 4, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else launch_down_k<T, MODE, true, 8, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
    } else {
        if (lds && rpb == 1 && nch > 2 && nch <= 4 && h->wch_dn != nullptr)
            launch_down_k<T, MODE, true, 4, E, true, true>(h, tl, grid, 1, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else if (!lds && nch == 0) launch_down_k<T, MODE, false, 0, E>(h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        else if (!lds) launch_down_k<T, MODE, false, 8, E>(h, tl, grid, 1, cs, 0, x, io, p, bvec, hdr, part, max_steps, s);
        else if (nch == 0) launch_down_k<T, MODE, true, 0, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else if (nch <= 2) launch_down_k<T, MODE, true, 2, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else if (nch <= 4) launch_down_k<T, MODE, true, 4, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
        else launch_down_k<T, MODE, true, 8, E>(h, tl, grid, rpb, 1, shm, x, io, p, bvec, hdr, part, max_steps, s);
    }
    ED_LAUNCHED("k_down");
    return ED_OK;
}

template <typename T, int MODE>
static int launch_down_c(const ed_ham *h, const Tile &tl, const T *x, T *io, const T *p, const double *bvec,
                         const Hdr *hdr, double *part, int max_steps, hipStream_t s) {
    using T2 = typename Cplx<T>::type;
    const DownShape d = down_shape(h, tl);
    const int block = std::min(tl.dn_block, 1024);
    const size_t shm = (size_t)complex_amp_lds(h) + (d.lds ? (size_t)(h->dim_dn * 2 * sizeof(T)) : 0);
    const T2 *x2 = reinterpret_cast<const T2 *>(x), *p2 = reinterpret_cast<const T2 *>(p);
    T2 *io2 = reinterpret_cast<T2 *>(io);
    const uint32_t *tab = static_cast<const uint32_t *>(h->tab_dn);
    if (d.lds)
        hipLaunchKernelGGL((k_downc<T, MODE, true>), dim3(d.grid), dim3(block), shm, s, x2, io2, p2, tab, h->amp_dn,
                           h->st_up, h->st_dn, (int)h->dim_dn, h->w_dn, d.csplit, static_cast<T>(h->t),
                           static_cast<T>(h->U), bvec, hdr, part, max_steps);
    else
        hipLaunchKernelGGL((k_downc<T, MODE, false>), dim3(d.grid), dim3(block), shm, s, x2, io2, p2, tab,
                           h->amp_dn, h->st_up, h->st_dn, (int)h->dim_dn, h->w_dn, d.csplit, static_cast<T>(h->t),
                           static_cast<T>(h->U), bvec, hdr, part, max_steps);
    ED_LAUNCHED("k_downc");
    return ED_OK;
}

template <typename T, int MODE>
static int launch_down(const ed_ham *h, const Tile &tl, const T *x, T *io, const T *p, const double *bvec,
                       const Hdr *hdr, double *part, int max_steps, hipStream_t s) {
    if (h->cplx) return launch_down_c<T, MODE>(h, tl, x, io, p, bvec, hdr, part, max_steps, s);
    if (wide_dn(h)) return launch_down_e<T, MODE, uint32_t>(h, tl, x, io, p, bvec, hdr, part, max_steps, s);
    return launch_down_e<T, MODE, uint16_t>(h, tl, x, io, p, bvec, hdr, part, max_steps, s);
}

static int down_grid(const ed_ham *h, const Tile &tl) { return down_shape(h, tl).grid; }

// Kernels staging rows in LDS may use up to kLdsBudget bytes of rows plus the
// slot after them; set once, outside any stream capture.
template <typename T, int MODE, int NCH, typename E>
static hipError_t set_lds_attr_e() {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down<T, MODE, true, NCH, false, E>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
    if (e != hipSuccess) return e;
    if constexpr (NCH == 4 && sizeof(E) == 2) {
        const hipError_t e2 =
            hipFuncSetAttribute(reinterpret_cast<const void *>(k_down<T, MODE, true, NCH, false, E, true, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
        if (e2 != hipSuccess) return e2;
    }
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_down<T, MODE, true, NCH, true, E>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
}

template <typename T, int MODE, int NCH>
static hipError_t set_lds_attr() {
    hipError_t e = set_lds_attr_e<T, MODE, NCH, uint16_t>();
    if (e != hipSuccess) return e;
    e = set_lds_attr_e<T, MODE, NCH, uint32_t>();
    if (e != hipSuccess || NCH == 0) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down2<T, MODE, NCH == 0 ? 2 : NCH, uint16_t>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down2<T, MODE, NCH == 0 ? 2 : NCH, uint32_t>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
    if constexpr (NCH == 4) {
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down2<T, MODE, 4, uint16_t, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down2<T, MODE, 4, uint32_t, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
    }
    if constexpr (NCH == 2 || NCH == 4) {
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down_win<T, MODE, NCH, uint16_t>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down_win<T, MODE, NCH, uint32_t>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down_win<T, MODE, NCH, uint32_t, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_down_win<T, MODE, NCH, uint32_t, true, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
    }
    return e;
}

template <typename T>
static hipError_t set_lds_attrs_t() {
    const hipError_t es[] = {set_lds_attr<T, 0, 0>(), set_lds_attr<T, 0, 2>(), set_lds_attr<T, 0, 4>(),
                             set_lds_attr<T, 0, 8>(), set_lds_attr<T, 1, 0>(), set_lds_attr<T, 1, 2>(),
                             set_lds_attr<T, 1, 4>(), set_lds_attr<T, 1, 8>(), set_lds_attr<T, 2, 0>(),
                             set_lds_attr<T, 2, 2>(), set_lds_attr<T, 2, 4>(), set_lds_attr<T, 2, 8>()};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

template <typename T>
static hipError_t set_lds_attrs_c() {
    const void *ks[] = {reinterpret_cast<const void *>(k_downc<T, 0, true>),
                        reinterpret_cast<const void *>(k_downc<T, 1, true>),
                        reinterpret_cast<const void *>(k_downc<T, 2, true>)};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget + 256);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static int ensure_attrs() {
    static int rc = -1000;
    if (rc != -1000) return rc;
    hipError_t e = set_lds_attrs_t<double>();
    if (e == hipSuccess) e = set_lds_attrs_t<float>();
    if (e == hipSuccess) e = set_lds_attrs_c<double>();
    if (e == hipSuccess) e = set_lds_attrs_c<float>();
    rc = hip_check(e, "hipFuncSetAttribute(k_down)");
    return rc;
}

template <typename T>
static int hv_impl(const ed_ham *h, const Tile &tl, const T *x, T *y, int *ctr, hipStream_t s) {
    int rc = launch_up<T>(h, tl, x, y, ctr, nullptr, 0, 0, s);
    if (rc) return rc;
    return launch_down<T, 0>(h, tl, x, y, nullptr, nullptr, nullptr, nullptr, 0, s);
}

static int upd_grid(int64_t n) { return grid_for(n, 256 * 4, kUpdBlocks); }

// values of dtype per vector: D, or 2 D (re, im pairs) with complex amplitudes
static int64_t vec_len(const ed_ham *h) { return h->dim_up * h->dim_dn * (h->cplx ? 2 : 1); }

// One Alg. 1 step on raw pointers (v != nullptr: also v += y_j f_j).  With
// ev != nullptr an event is recorded before each kernel and after the last.
template <typename T, int MODE>
static int step_impl(const ed_ham *h, const Tile &tl, const T *f_prev, const T *f_cur, T *f_next, double *a,
                     double *b, T *v, const WsLayout &w, int max_steps, hipStream_t s, hipEvent_t *ev = nullptr) {
    if (ev) ED_HIP(hipEventRecord(ev[0], s));
    int rc = launch_up<T>(h, tl, f_cur, f_next, w.ctr, w.hdr, 1, max_steps, s);
    if (rc) return rc;
    if (ev) ED_HIP(hipEventRecord(ev[1], s));
    rc = launch_down<T, MODE>(h, tl, f_cur, f_next, f_prev, b, w.hdr, w.part, max_steps, s);
    if (rc) return rc;
    if (ev) ED_HIP(hipEventRecord(ev[2], s));
    hipLaunchKernelGGL(k_reduce<MODE>, dim3(1), dim3(1024), 0, s, w.part, down_grid(h, tl), w.hdr, a, max_steps);
    ED_LAUNCHED("k_reduce");
    if (ev) ED_HIP(hipEventRecord(ev[3], s));
    const int64_t n = vec_len(h);
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
static int norm_launch(const T *in, T *out, int64_t n, const WsLayout &w, double *b, int mode, hipStream_t s,
                       double gauge_sign = 1.0) {
    const int g = upd_grid(n);
    hipLaunchKernelGGL(k_sumsq<T>, dim3(g), dim3(256), 0, s, in, n, w.part2);
    ED_LAUNCHED("k_sumsq");
    hipLaunchKernelGGL(k_init_norm, dim3(1), dim3(1024), 0, s, w.part2, g, w.hdr, b, mode, gauge_sign);
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

// ---------------------------------------------------------------------------
// Host side of the runs: step orchestration, graphs, the autotuner, the entry
// points, and the kernels that only they launch.  Everything above this line
// (the step kernels and their launch shapes) is what the measured HBM traffic
// of the step kernels depends on.

// Largest |x_i| of a grid-stride share per workgroup, with its first index and
// its signed value: out[3 b .. 3 b + 2] = (|x_i|, i, x_i) for workgroup b.  A
// thread visits its elements in ascending order and keeps the first maximum;
// the workgroup takes the larger magnitude, the lower index among equals.
template <typename T>
__global__ __launch_bounds__(256) void k_absmax(const T *__restrict__ x, int64_t n, double *__restrict__ out) {
    double m = -1.0, val = 0.0;
    int64_t at = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = x[i], a = fabs(v);
        if (a > m) { m = a; at = i; val = v; }
    }
    __shared__ double sm[256], sv[256];
    __shared__ int64_t si[256];
    sm[threadIdx.x] = m;
    sv[threadIdx.x] = val;
    si[threadIdx.x] = at;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const int o = threadIdx.x + h;
            if (sm[o] > sm[threadIdx.x] || (sm[o] == sm[threadIdx.x] && si[o] < si[threadIdx.x])) {
                sm[threadIdx.x] = sm[o];
                sv[threadIdx.x] = sv[o];
                si[threadIdx.x] = si[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = sm[0];
        out[3 * blockIdx.x + 1] = (double)si[0];
        out[3 * blockIdx.x + 2] = sv[0];
    }
}

static void rotate(ed_lanczos *st) {
    void *old_prev = st->f_prev;
    st->f_prev = st->f_cur;
    st->f_cur = st->f_next;
    st->f_next = old_prev;
    st->j += 1;
}

static int init_impl(const ed_ham *h, ed_lanczos *st, const void *f1, const WsLayout &w, hipStream_t s) {
    const int64_t n = vec_len(h);
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
    ~SideStream() {   // an early return: drain what was queued before releasing the stream
        if (own) (void)hipStreamSynchronize(own);
        if (ev) (void)hipEventDestroy(ev);
        if (own) (void)hipStreamDestroy(own);
    }
};

// Launch `nsteps` steps as a replayed graph of 3*k steps (three-buffer rotation).  The stream the graph is
// launched on must outlive this object: on an early return a launch may still be in flight, so the stream is
// drained before the executable graph is released.
struct StepGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipStream_t s = nullptr;
    int steps = 0;
    ~StepGraph() {
        if (s) (void)hipStreamSynchronize(s);
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
    sg.s = s;
    sg.steps = nsteps;
    return ED_OK;
}

template <typename T>
static int tune_impl(const ed_ham *h, const T *x, T *y, const T *p, const WsLayout &w, int reps, hipStream_t s,
                     int32_t *tile, double *ms_up, double *ms_dn) {
    hipEvent_t e0, e1;
    ED_HIP(hipEventCreate(&e0));
    ED_HIP(hipEventCreate(&e1));
    int rc = ED_OK;
    double best_up = 1e300, best_dn = 1e300;
    int bu = 0, bd = 0;
    // complex instances: k_upc takes only the rows per tile from a tile and
    // k_downc only the workgroup size, so one candidate per distinct value
    std::vector<int> seen_rc, seen_block;
    auto first_of = [](std::vector<int> &seen, int v) {
        if (std::find(seen.begin(), seen.end(), v) != seen.end()) return false;
        seen.push_back(v);
        return true;
    };
    for (int ui = 1; ui < kNumUp && rc == ED_OK; ++ui) {
        const Tile tl = resolve_tile_id(h, ui);
        if (ms_up) ms_up[ui] = -1.0;
        if (h->cplx ? !first_of(seen_rc, tl.up_rc) : tl.up_wlog2 != kUpTiles[ui].wlog2)
            continue;   // the same launch as an earlier candidate (a clamped stripe, or complex)
        rc = launch_up<T>(h, tl, x, y, w.ctr, nullptr, 0, 0, s);
        if (rc) break;
        rc = hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < reps && rc == ED_OK; ++r) rc = launch_up<T>(h, tl, x, y, w.ctr, nullptr, 0, 0, s);
        if (rc == ED_OK) rc = hip_check(hipEventRecord(e1, s), "hipEventRecord");
        if (rc == ED_OK) rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float msf = 0.f;
        if (rc == ED_OK) rc = hip_check(hipEventElapsedTime(&msf, e0, e1), "hipEventElapsedTime");
        const double m = msf / reps;
        if (ms_up) ms_up[ui] = m;
        if (m < best_up) { best_up = m; bu = ui; }
    }
    // k_down is timed as in a Lanczos step (second step: f_{j-1} read, partial
    // sums written), from a synthetic header; p stands in for f_{j-1}.  Each
    // timed launch follows an untimed up part (the best tile's), as in a step,
    // so the caches hold what they hold there.
    Hdr fake{};
    fake.sig_cur = 1.0;
    fake.sig_prev = 1.0;
    fake.jdev = 1;
    fake.status = 0;
    const double bfake[2] = {0.0, 0.5};
    if (rc == ED_OK) rc = hip_check(hipMemcpyAsync(w.hdr, &fake, sizeof(Hdr), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (rc == ED_OK) rc = hip_check(hipMemcpyAsync(w.y, bfake, sizeof bfake, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (rc == ED_OK) rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    constexpr int SM = sizeof(T) == 8 ? 1 : 2;
    const Tile tl_up = resolve_tile_id(h, bu);
    for (int di = 1; di < kNumDn && rc == ED_OK; ++di) {
        const Tile tl = resolve_tile_id(h, di << 8);
        if (ms_dn) ms_dn[di] = -1.0;
        if (h->cplx) {
            if (!first_of(seen_block, std::min(tl.dn_block, 1024))) continue;   // one row per workgroup
        } else {
            if (kDnTiles[di].rpb > 0 && (int64_t)kDnTiles[di].rpb * h->dim_dn * (int64_t)sizeof(T) > kLdsBudget)
                continue;
            if (kDnTiles[di].rpb > h->dim_up) continue;
            if (kDnTiles[di].pair && !pair_rows(h, tl)) continue;   // would run as the one-row kernel
            if (kDnTiles[di].win && !win_rows(h, tl)) continue;
            if (tl.dn_block != kDnTiles[di].block) continue;   // clamped duplicate of a smaller workgroup
        }
        rc = launch_down<T, SM>(h, tl, x, y, p, w.y, w.hdr, w.part, 2, s);
        if (rc) break;
        double tot = 0.0;
        for (int r = 0; r < reps && rc == ED_OK; ++r) {
            rc = launch_up<T>(h, tl_up, x, y, w.ctr, nullptr, 0, 0, s);
            if (rc == ED_OK) rc = hip_check(hipEventRecord(e0, s), "hipEventRecord");
            if (rc == ED_OK) rc = launch_down<T, SM>(h, tl, x, y, p, w.y, w.hdr, w.part, 2, s);
            if (rc == ED_OK) rc = hip_check(hipEventRecord(e1, s), "hipEventRecord");
            if (rc == ED_OK) rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            float msf = 0.f;
            if (rc == ED_OK) rc = hip_check(hipEventElapsedTime(&msf, e0, e1), "hipEventElapsedTime");
            tot += msf;
        }
        const double m = tot / reps;
        if (ms_dn) ms_dn[di] = m;
        if (m < best_dn) { best_dn = m; bd = di; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *tile = bu | (bd << 8);
    return ED_OK;
}

// ---------------------------------------------------------------------------
// Device scratch of the run that allocates nothing (ed_ground_energy_noalloc):
// the workspace of a Lanczos run (header, partial sums, queue counters) in a
// file-scope array of every GPU the library runs on, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// only stands for the symbol): it takes the array's address on each device
// once, by hipGetSymbolAddress with that device current, and uses that.
constexpr int64_t kScratchBytes = 4 << 20;
constexpr int kScratchDevices = 64;
constexpr int kNoallocMaxSteps = 2048;   // coefficients held on the host stack
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::atomic<void *> scratch_addr[kScratchDevices];

static int scratch_on_current_device(void **out) {
    int dev = 0;
    ED_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices)
        return set_error(ED_EINVAL, "device scratch: device %d beyond the %d the library tracks", dev, kScratchDevices);
    void *p = scratch_addr[dev].load();
    if (!p) {
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        scratch_addr[dev].store(p);
    }
    *out = p;
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
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return set_error(ED_EINVAL, "ed_hv: ws must be a 256-byte aligned workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Tile tl = resolve_tile(h);
    const WsLayout w = ws_layout(h, ws, 0);
    if (h->dtype == ED_F64) return hv_impl<double>(h, tl, (const double *)x, (double *)y, w.ctr, s);
    return hv_impl<float>(h, tl, (const float *)x, (float *)y, w.ctr, s);
}

int ed_tile_params(int32_t tile, const ed_ham *h, int32_t *params) {
    clear_error();
    int rc = check_ham(h, "ed_tile_params");
    if (rc) return rc;
    if (!params || !valid_tile_id(tile)) return set_error(ED_EINVAL, "ed_tile_params: bad arguments");
    const Tile t = resolve_tile_id(h, tile);
    params[0] = 1 << t.up_wlog2;
    params[1] = t.up_rc;
    params[2] = t.up_block;
    params[3] = t.up_map;
    params[4] = t.dn_block;
    params[5] = t.dn_rpb;
    params[6] = pair_rows(h, t) ? 1 : (win_rows(h, t) ? 2 : 0);
    return ED_OK;
}

int ed_tune(const ed_ham *h, const void *x, void *y, const void *p, void *ws, void *stream, int32_t reps,
            int32_t *tile, double *ms_up, double *ms_dn) {
    clear_error();
    int rc = check_ham(h, "ed_tune");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    if (!x || !y || x == y || p == y || !ws || !tile || reps < 1) return set_error(ED_EINVAL, "ed_tune: bad arguments");
    if (!p) p = x;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout w = ws_layout(h, ws, 2);
    if (h->dtype == ED_F64)
        return tune_impl<double>(h, (const double *)x, (double *)y, (const double *)p, w, reps, s, tile, ms_up, ms_dn);
    return tune_impl<float>(h, (const float *)x, (float *)y, (const float *)p, w, reps, s, tile, ms_up, ms_dn);
}

int ed_tile_count(int32_t *n_up, int32_t *n_dn) {
    if (!n_up || !n_dn) return set_error(ED_EINVAL, "ed_tile_count: NULL");
    *n_up = kNumUp;
    *n_dn = kNumDn;
    return ED_OK;
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
    int launched = 0;

    std::vector<double> a(max_steps), b(max_steps + 1), e(max_steps + 1, 0.0);
    int have = 0;            // steps whose E0 is known
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
    // Launched steps beyond the device's step count were no-ops (the state
    // froze at a breakdown or at max_steps): the vectors rotated jd times.
    for (int k = 0; k < hh.jdev; ++k) rotate(st);
    st->j = hh.jdev;
    *e0 = e[stop_at];
    *steps = stop_at;
    if (a_host) std::copy(a.begin(), a.begin() + stop_at, a_host);
    if (b_host) std::copy(b.begin(), b.begin() + stop_at + 1, b_host);
    rc = ss.close();
    if (rc) return rc;
    return result;
}

int ed_ground_energy_noalloc(const ed_ham *h, ed_lanczos *st, const void *f1, double tol, int32_t check_every,
                             void *stream, double *e0, int32_t *steps, double *a_host, double *b_host) {
    clear_error();
    void *ws = nullptr;
    int rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    rc = check_lanczos(h, st, ws, "ed_ground_energy_noalloc");
    if (rc) return rc;
    if (!e0 || !steps) return set_error(ED_EINVAL, "ed_ground_energy_noalloc: e0/steps are NULL");
    if (!f1 || f1 == st->f_cur)
        return set_error(ED_EINVAL, "ed_ground_energy_noalloc: f1 must be a buffer other than f_cur");
    const int max_steps = st->max_steps;
    if (max_steps > kNoallocMaxSteps)
        return set_error(ED_ECAPACITY, "ed_ground_energy_noalloc: max_steps %d above %d", max_steps, kNoallocMaxSteps);
    if (ws_bytes(h, max_steps) > kScratchBytes)
        return set_error(ED_ECAPACITY, "ed_ground_energy_noalloc: the run needs %lld bytes of scratch, above %lld",
                         (long long)ws_bytes(h, max_steps), (long long)kScratchBytes);
    rc = ensure_attrs();
    if (rc) return rc;
    const int chunk = std::max(1, check_every);
    const Tile tl = resolve_tile(h);
    const WsLayout w = ws_layout(h, ws, max_steps);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = init_impl(h, st, f1, w, s);
    if (rc) return rc;
    Hdr hh;
    rc = read_hdr(w, &hh, s);
    if (rc) return rc;
    if (hh.status != 0) return set_error(ED_EINVAL, "ed_ground_energy_noalloc: start vector has zero or non-finite norm");
    st->j = 0;
    // the coefficients and Ritz values on the stack: no allocation on the host either
    double a[kNoallocMaxSteps], b[kNoallocMaxSteps + 1], e[kNoallocMaxSteps + 1];
    ed_lanczos cur = *st;
    int have = 0, launched = 0, stop_at = -1, result = ED_NOT_CONVERGED;
    while (true) {
        for (int k = 0; k < chunk; ++k) {
            rc = step_dispatch(h, tl, cur.f_prev, cur.f_cur, cur.f_next, cur.a, cur.b, nullptr, w, max_steps, s);
            if (rc) return rc;
            rotate(&cur);
        }
        launched += chunk;
        rc = read_hdr(w, &hh, s);
        if (rc) return rc;
        const int jd = hh.jdev;
        if (jd > have) {
            ED_HIP(hipMemcpyAsync(a, st->a, 8 * (size_t)jd, hipMemcpyDeviceToHost, s));
            ED_HIP(hipMemcpyAsync(b, st->b, 8 * (size_t)(jd + 1), hipMemcpyDeviceToHost, s));
            ED_HIP(hipStreamSynchronize(s));
            for (int j = have + 1; j <= jd; ++j) {
                e[j] = tridiag_lowest(a, b + 1, j);
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
        if (launched > 4 * max_steps + 3 * chunk) return set_error(ED_EDEVICE, "ed_ground_energy_noalloc: no progress");
    }
    // steps launched beyond the device's count were no-ops: the vectors rotated jd times
    for (int k = 0; k < hh.jdev; ++k) rotate(st);
    st->j = hh.jdev;
    *e0 = e[stop_at];
    *steps = stop_at;
    if (a_host) std::copy(a, a + stop_at, a_host);
    if (b_host) std::copy(b, b + stop_at + 1, b_host);
    return result;
}

int ed_ground_state(const ed_ham *h, ed_lanczos *st, const void *f1, int32_t m, double tol, int32_t extra,
                    int64_t gauge_index, void *v, void *ws, void *stream, double *e0, int32_t *steps) {
    clear_error();
    int rc = check_lanczos(h, st, ws, "ed_ground_state");
    if (rc) return rc;
    rc = ensure_attrs();
    if (rc) return rc;
    if (!v || !e0 || !steps || m < 1 || m > st->max_steps || extra < 0)
        return set_error(ED_EINVAL, "ed_ground_state: bad arguments (need 1 <= m <= max_steps, extra >= 0)");
    if (v == st->f_prev || v == st->f_cur || v == st->f_next || v == f1)
        return set_error(ED_EINVAL, "ed_ground_state: v must not alias f1 or the Lanczos vectors");
    if (h->cplx && gauge_index >= 0)
        return set_error(ED_EINVAL, "ed_ground_state: a complex state's phase is not fixed by an index (pass -1)");
    // pass 1: m steps (fewer on breakdown); with tol > 0, up to m: the steps until E0 settles (the rule of
    // ed_ground_energy), then `extra` more
    ed_lanczos s1 = *st;
    s1.max_steps = m;
    std::vector<double> a(m), b(m + 1);
    int32_t k = 0;
    double e;
    if (tol > 0.0) {
        rc = ed_ground_energy(h, &s1, f1, tol, 15, ws, stream, &e, &k, nullptr, nullptr);
        if (rc < 0) return rc;
        const int32_t want = (int32_t)std::min<int64_t>(m, (int64_t)k + extra);
        // the device may be past k (steps go in chunks); step on to `want` unless frozen
        int32_t done = 0, status = ED_OK;
        rc = ed_lanczos_read(h, &s1, ws, stream, &done, &status, nullptr, nullptr);
        if (rc) return rc;
        for (int32_t j = done; j < want && status == ED_OK; ++j) {
            rc = ed_lanczos_step(h, &s1, ws, stream);
            if (rc) return rc;
        }
        rc = ed_lanczos_read(h, &s1, ws, stream, &done, &status, a.data(), b.data());
        if (rc) return rc;
        k = std::min(done, want);
    } else {
        rc = ed_ground_energy(h, &s1, f1, 0.0, 30, ws, stream, &e, &k, a.data(), b.data());
        if (rc < 0) return rc;
    }
    std::vector<double> y(k);
    rc = ed_tridiag_lowest_vector(a.data(), b.data() + 1, k, &e, y.data());
    if (rc) return rc;
    // pass 2: replay the identical steps, accumulating v = sum_j y_j f_j
    hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout w = ws_layout(h, ws, m);
    ED_HIP(hipMemcpyAsync(w.y, y.data(), 8 * (size_t)k, hipMemcpyHostToDevice, s));
    const int64_t n = vec_len(h);
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
    double gsign = 1.0;
    if (gauge_index >= 0) {
        if (gauge_index >= n) return set_error(ED_EINVAL, "ed_ground_state: gauge index out of range");
        double gv = 0.0;
        if (h->dtype == ED_F64) {
            ED_HIP(hipMemcpyAsync(&gv, (const double *)v + gauge_index, 8, hipMemcpyDeviceToHost, s));
        } else {
            float gf = 0.f;
            ED_HIP(hipMemcpyAsync(&gf, (const float *)v + gauge_index, 4, hipMemcpyDeviceToHost, s));
            ED_HIP(hipStreamSynchronize(s));
            gv = gf;
        }
        // the largest |v_i| (first index among equals), per workgroup into the partial-norm slots, then on the host
        constexpr int kMaxBlocks = 1024;
        const int g = grid_for(n, 256, kMaxBlocks);
        if (h->dtype == ED_F64)
            hipLaunchKernelGGL(k_absmax<double>, dim3(g), dim3(256), 0, s, (const double *)v, n, w.part2);
        else
            hipLaunchKernelGGL(k_absmax<float>, dim3(g), dim3(256), 0, s, (const float *)v, n, w.part2);
        ED_LAUNCHED("k_absmax");
        std::vector<double> mx(3 * (size_t)g);
        ED_HIP(hipMemcpyAsync(mx.data(), w.part2, 8 * mx.size(), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        double best = -1.0, best_i = 0.0, best_v = 0.0;
        for (int b = 0; b < g; ++b)
            if (mx[3 * b] > best || (mx[3 * b] == best && mx[3 * b + 1] < best_i)) {
                best = mx[3 * b];
                best_i = mx[3 * b + 1];
                best_v = mx[3 * b + 2];
            }
        // the reference element decides unless it is below 1e-3 of the largest magnitude
        const double decide = std::fabs(gv) >= 1e-3 * best ? gv : best_v;
        gsign = decide < 0.0 ? -1.0 : 1.0;
    }
    if (h->dtype == ED_F64) rc = norm_launch<double>((const double *)v, (double *)v, n, w, s2.b, 1, s, gsign);
    else rc = norm_launch<float>((const float *)v, (float *)v, n, w, s2.b, 1, s, gsign);
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
