// The fused Lanczos step for gfx950: Alg. 1 with two passes over the vectors
// per step and no separate vector-update pass.
//
// H x = (H_up x I) x + (I x H_dn) x + U Docc o x (Eq. 3-5).  The down part
// wants whole rows X[r, :] (staged in LDS), the up part wants column stripes
// X[:, cs] (whole rows of the stripe are gathered).  A step of the reference
// kernels (ed_device.hip) is up pass, down pass, a_j, update pass: about 9pD
// bytes.  Here the update of Alg. 1 line 6 moves into the next step's down
// pass, which reads the rows of q_j and F_j anyway:
//
//   k_fdn   (rows)     F_{j+1} = q_j - cx F_j - cp F_{j-1}     (line 6, stored)
//                      Z = t down-part(F_{j+1}) + U Docc o F_{j+1}   (Eq. 5)
//                      partial sums of |F_{j+1}|^2
//   k_fnorm            b_{j+1} = |F_{j+1}|, breakdown test       (lines 7-8)
//   k_fup   (stripes)  q_{j+1} = sigma_{j+1} (Z + t up-part(F_{j+1}))
//                                - b_{j+1} sigma_j F_j            (Eq. 4, line 4)
//                      partial dots of q_{j+1} with F_{j+1} (and F_j)
//   k_freduce          a_{j+1} = q.f_{j+1} and the coefficients cx, cp (line 5)
//
// so a step reads q_j, F_j (and F_{j-1} in the mixed form) and writes F_{j+1}
// and Z in the down pass, then reads F_{j+1}, Z and F_j and writes q_{j+1}
// over Z in the up pass: 8pD in float64 against 9pD, in two kernels instead
// of three.  b_{j+1} is still the norm of the stored F_{j+1} and every scalar
// follows Alg. 1's order, so the coefficients are those of the reference step
// up to the order of additions inside H.v.
//
// The up pass gathers 128-byte row segments of a narrow column stripe; each
// XCD owns a contiguous band of stripes and its workgroups walk them stripe
// after stripe, so the stripe being gathered (1.65 MB at 4x4 8+8) stays in
// that XCD's L2 while ~17 output rows per input row re-read it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/ed.h"
#include "ed_common.h"
#include "ed_internal.h"
#include "ed_launch.h"
#include "ed_state.h"

namespace ed {

template <typename T, int V> struct VecOf;
template <> struct VecOf<double, 1> { using type = double; };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 1> { using type = float; };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <typename T, int V> using vec_t = typename VecOf<T, V>::type;

template <typename T, int V> __device__ __forceinline__ T vget(const vec_t<T, V> &a, int i) {
    if constexpr (V == 1) return a;
    else return a[i];
}
template <typename T, int V> __device__ __forceinline__ void vset(vec_t<T, V> &a, int i, T x) {
    if constexpr (V == 1) a = x;
    else a[i] = x;
}
template <typename T, int V> __device__ __forceinline__ vec_t<T, V> vzero() {
    vec_t<T, V> a;
#pragma unroll
    for (int i = 0; i < V; ++i) vset<T, V>(a, i, T(0));
    return a;
}
// the value if keep, else +0, without a branch
template <typename T, int V> __device__ __forceinline__ vec_t<T, V> vkeep(vec_t<T, V> a, bool keep) {
#pragma unroll
    for (int i = 0; i < V; ++i) vset<T, V>(a, i, keep_or_zero(vget<T, V>(a, i), keep));
    return a;
}

// ---------------------------------------------------------------------------
// Down pass.  One workgroup per block of rpb rows (the rows sit in LDS).
// PEND: the stored vector of the last step is q_j (xq); F_{j+1} = q_j - cx
// F_j - cp F_{j-1} is formed in float64, rounded once to T, written over q_j
// and staged; else F_{j+1} is read from xq as it stands.  Z goes to zdst,
// which in the pending mixed form is the buffer of F_{j-1}: its rows are read
// in the staging phase, before the barrier, and overwritten after it.
// ACCV (second pass of the two-pass ground state): v += w[j] F_{j+1}.
template <typename T, int MODE, bool PEND, bool ACCV, int NCH, bool MULTI>
__global__ __launch_bounds__(1024) void k_fdn(T *xq, const T *fj, const T *fjm, T *zdst, T *__restrict__ v,
                                              const double *__restrict__ wv, const uint16_t *__restrict__ tab,
                                              const uint64_t *__restrict__ st_up, const uint64_t *__restrict__ st_dn,
                                              int Dup, int Ddn, int W8, int rpb, T t, T U,
                                              const Hdr *__restrict__ hdr, int *__restrict__ ctr,
                                              double *__restrict__ partials, int max_steps) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *xs = reinterpret_cast<T *>(smem);
    if (frozen(hdr, max_steps)) return;
    if (blockIdx.x == 0 && threadIdx.x < 8) ctr[threadIdx.x] = 0;   // the up pass's tile queues
    const int r0 = blockIdx.x * rpb;
    const int nr = min(rpb, Dup - r0);
    const int n = nr * Ddn;
    const int64_t base = (int64_t)r0 * Ddn;
    double ss[1] = {0.0};
    // ---- staging: F_{j+1} rows into LDS (and back to HBM when formed here)
    {
        double cx = 0.0, cp = 0.0;
        if constexpr (PEND) {
            cx = hdr->cx;
            cp = MODE == 2 ? hdr->cp : 0.0;
        }
        double w = 0.0;
        if constexpr (ACCV) w = wv[hdr->jdev];
        constexpr int VS = 16 / sizeof(T);
        using VV = vec_t<T, VS>;
        const uintptr_t mis = (reinterpret_cast<uintptr_t>(xq + base) | reinterpret_cast<uintptr_t>(fj + base) |
                               reinterpret_cast<uintptr_t>(fjm + base) | (ACCV ? reinterpret_cast<uintptr_t>(v + base) : 0)) & 15;
        int done = 0;
        if (mis == 0) {
            const int nv = n / VS;
            const VV *q4 = reinterpret_cast<const VV *>(xq + base);
            const VV *f4 = reinterpret_cast<const VV *>(fj + base);
            const VV *p4 = reinterpret_cast<const VV *>(fjm + base);
            VV *d4 = reinterpret_cast<VV *>(xq + base);
            VV *v4 = reinterpret_cast<VV *>(v + base);
            VV *s4 = reinterpret_cast<VV *>(xs);
            int i = threadIdx.x;
            // two vectors per thread in flight per trip
            for (; i < nv; i += 2 * blockDim.x) {
                const int i2 = i + blockDim.x;
                const bool two = i2 < nv;
                VV qa = __builtin_nontemporal_load(q4 + i), qb = two ? __builtin_nontemporal_load(q4 + i2) : qa;
                VV fa, fb, pa, pb;
                if constexpr (PEND) {
                    fa = __builtin_nontemporal_load(f4 + i);
                    fb = two ? __builtin_nontemporal_load(f4 + i2) : fa;
                    if (MODE == 2 && cp != 0.0) {
                        pa = __builtin_nontemporal_load(p4 + i);
                        pb = two ? __builtin_nontemporal_load(p4 + i2) : pa;
                    } else {
                        pa = vzero<T, VS>();
                        pb = pa;
                    }
                }
                VV xa = qa, xb = qb;
                if constexpr (PEND) {
#pragma unroll
                    for (int k = 0; k < VS; ++k) {
                        const T a = static_cast<T>((double)vget<T, VS>(qa, k) - cx * (double)vget<T, VS>(fa, k) -
                                                   cp * (double)vget<T, VS>(pa, k));
                        const T b = static_cast<T>((double)vget<T, VS>(qb, k) - cx * (double)vget<T, VS>(fb, k) -
                                                   cp * (double)vget<T, VS>(pb, k));
                        vset<T, VS>(xa, k, a);
                        vset<T, VS>(xb, k, b);
                        ss[0] += (double)a * (double)a;
                        if (two) ss[0] += (double)b * (double)b;
                    }
                    d4[i] = xa;
                    if (two) d4[i2] = xb;
                }
                s4[i] = xa;
                if (two) s4[i2] = xb;
                if constexpr (ACCV) {
                    VV va = v4[i];
#pragma unroll
                    for (int k = 0; k < VS; ++k)
                        vset<T, VS>(va, k, static_cast<T>((double)vget<T, VS>(va, k) + w * (double)vget<T, VS>(xa, k)));
                    v4[i] = va;
                    if (two) {
                        VV vb = v4[i2];
#pragma unroll
                        for (int k = 0; k < VS; ++k)
                            vset<T, VS>(vb, k,
                                        static_cast<T>((double)vget<T, VS>(vb, k) + w * (double)vget<T, VS>(xb, k)));
                        v4[i2] = vb;
                    }
                }
            }
            done = nv * VS;
        }
        for (int k = done + threadIdx.x; k < n; k += blockDim.x) {
            T x = xq[base + k];
            if constexpr (PEND) {
                const double pv = (MODE == 2 && cp != 0.0) ? (double)fjm[base + k] : 0.0;
                x = static_cast<T>((double)x - cx * (double)fj[base + k] - cp * pv);
                xq[base + k] = x;
                ss[0] += (double)x * (double)x;
            }
            xs[k] = x;
            if constexpr (ACCV) v[base + k] = static_cast<T>((double)v[base + k] + w * (double)x);
        }
    }
    __syncthreads();
    // ---- down part and the on-site term from the staged rows
    const Chunk8<uint16_t> *til = reinterpret_cast<const Chunk8<uint16_t> *>(tab + (int64_t)Ddn * W8);
    const int nch = W8 >> 3;
    int i = threadIdx.x;
    if (i < n) {
        Chunk8<uint16_t> tq[NCH > 0 ? NCH : 1];
        int c, rr;
        if constexpr (MULTI) { rr = i / Ddn; c = i - rr * Ddn; } else { rr = 0; c = i; }
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = table_chunk<NCH, uint16_t>(til, k8, nch, Ddn, c);
        uint64_t sdv = st_dn[c], suv = st_up[r0 + rr];
        for (; i < n; i += blockDim.x) {
            const int in = min(i + (int)blockDim.x, n - 1);
            int cn, rrn;
            if constexpr (MULTI) { rrn = in / Ddn; cn = in - rrn * Ddn; } else { rrn = 0; cn = in; }
            Chunk8<uint16_t> tqn[NCH > 0 ? NCH : 1];
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) tqn[k8] = table_chunk<NCH, uint16_t>(til, k8, nch, Ddn, cn);
            const uint64_t sdn = st_dn[cn];
            uint64_t sun = suv;
            if constexpr (MULTI) sun = st_up[r0 + rrn];
            const T *xrow = xs + (int64_t)rr * Ddn;
            T acc0 = T(0), acc1 = T(0);
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) {
                if (k8 >= nch) break;
                if (!__any(!is_pad<uint16_t>(entry(tq[k8], 0)))) break;
                T vv[8], sg[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const unsigned e = entry(tq[k8], k);
                    const bool pk = !is_pad<uint16_t>(e);
                    sg[k] = pk ? ((e & 1u) ? T(-1) : T(1)) : T(0);
                    vv[k] = xrow[pk ? (int)(e >> 1) : 0];
                }
#pragma unroll
                for (int k = 0; k < 8; k += 2) {
                    acc0 += sg[k] * vv[k];
                    acc1 += sg[k + 1] * vv[k + 1];
                }
            }
            const T nd = static_cast<T>(__popcll(suv & sdv));
            const T z = t * (acc0 + acc1) + U * nd * xrow[c];
            __builtin_nontemporal_store(z, zdst + base + i);
            c = cn;
            rr = rrn;
            sdv = sdn;
            suv = sun;
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = tqn[k8];
        }
    }
    if constexpr (PEND) {
        double tot[1];
        block_sum<1>(ss, tot);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * kPartStride] = tot[0];
    }
}

// ---------------------------------------------------------------------------
// Up pass and the rest of Alg. 1 line 4, with the partial dot products.
// A tile is (stripe of SW = L*V columns, FUP_RC rows).  A workgroup is four
// compute wavefronts and one loader wavefront, working on two tiles at once
// through double-buffered LDS:
//  - the loader takes the next tile from its XCD's queue, streams that
//    tile's operands (the down-pass result Z, F_j for the recurrence term,
//    F_{j+1} for the dot products, and the up table's rows) into LDS, and
//    writes the q of the tile before last from LDS to HBM, so the stream to
//    and from HBM has a whole tile of latency behind it;
//  - the compute wavefronts gather the up part for the current tile from the
//    stripe X[:, stripe] (Eq. 4) and finish q = sigma (Z + t up) - cprev F_j
//    from LDS.  A wavefront covers G = 64/L rows at once: lanes L*g .. L*g+L-1
//    read V adjacent columns each of one row, so one gather instruction moves
//    G row segments of SW*sizeof(T) bytes, and the number of chunks live in
//    any row of the group selects straight-line code that issues every
//    gather before the first is consumed.
// Stripe s is served by XCD s mod 8; each XCD takes its stripes' tiles in
// order from its own queue (integer atomics; the loader finds its XCD in the
// XCC_ID hardware register, drains that queue, then helps the others), so the
// tiles in flight on an XCD cover part of one stripe, which that XCD's L2
// holds while ~17 output rows per input row gather from it.  The queues are
// reset by the down pass of the same step.
constexpr int FUP_RC = 64;

// Gathers of chunks k0 .. k0+NL-1 of a row group, all issued before any is used.
template <typename T, int V, int NL, int NCH>
__device__ __forceinline__ void fup_gather(const T *__restrict__ xs, int Ddn, const Chunk8<uint16_t> (&q)[NCH],
                                           int k0, T (&acc)[V]) {
    using VT = vec_t<T, V>;
    VT g[NL][8];
#pragma unroll
    for (int k8 = 0; k8 < NL; ++k8)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned e = entry(q[k0 + k8], k);
            g[k8][k] = *reinterpret_cast<const VT *>(xs + (int64_t)(!is_pad<uint16_t>(e) ? (e >> 1) : 0u) * Ddn);
        }
#pragma unroll
    for (int k8 = 0; k8 < NL; ++k8)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned e = entry(q[k0 + k8], k);
            const T sg = is_pad<uint16_t>(e) ? T(0) : ((e & 1u) ? T(-1) : T(1));
#pragma unroll
            for (int i = 0; i < V; ++i) acc[i] = fma_t(sg, vget<T, V>(g[k8][k], i), acc[i]);
        }
}

// LDS of one up-pass workgroup: two tiles' operands and results
template <typename T, int SW, int NCH> struct FupLds {
    T op[2][3][FUP_RC][SW];                                    // Z, F_j, F_{j+1} at the tile's elements
    T qo[2][FUP_RC][SW];                                       // q of the tile, for the loader to write
    Chunk8<uint16_t> tb[2][FUP_RC][NCH > 0 ? NCH : 1];         // table chunks of the tile's rows
    int tile[2][3];                                            // stripe, first row, valid
    int tile_id;
};

template <typename T, int MODE, int L, int V, int NCH>
__global__ __launch_bounds__(320) void k_fup(const T *__restrict__ x, T *__restrict__ zq, const T *__restrict__ p,
                                             const uint16_t *__restrict__ tab, int Dup, int Ddn, int W8, int n_rc,
                                             int n_stripes, T t, const double *__restrict__ bvec,
                                             const Hdr *__restrict__ hdr, int *__restrict__ ctr,
                                             double *__restrict__ partials, int max_steps) {
    constexpr int NV = MODE == 2 ? 5 : 1;
    constexpr int G = 64 / L;
    constexpr int SW = L * V;
    constexpr int SV = V;                    // the loader moves row segments in the compute lanes' pieces
    constexpr int PR = L;                    // pieces per row segment
    constexpr int RPI = G;                   // rows per loader instruction
    constexpr int NCW = 4;                   // compute wavefronts
    using VT = vec_t<T, V>;
    using PV = VT;
    static_assert(FUP_RC % RPI == 0 && FUP_RC % (NCW * G) == 0, "up-pass tile shape");
    extern __shared__ __align__(16) unsigned char fup_smem[];
    FupLds<T, SW, NCH> &sh = *reinterpret_cast<FupLds<T, SW, NCH> *>(fup_smem);
    if (frozen(hdr, max_steps)) return;
    const int j = hdr->jdev;
    const bool has_prev = j > 0;
    const T sig = static_cast<T>(hdr->sig_cur);
    const T cprev = has_prev ? static_cast<T>(bvec[j] * hdr->sig_prev) : T(0);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool loader = wave == NCW;
    const int nch = W8 >> 3;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;

    // ---- loader state: the queue it is draining
    int qi = 0, band = 0;
    const int mine = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u);   // XCC_ID
    auto next_tile = [&](int buf, int &r0) {
        // one lane takes a tile from the current band's queue; a drained band moves the loader to the next
        int st = -1;
        r0 = 0;
        while (qi < 8) {
            band = (mine + qi) & 7;
            const int ntile = (band < n_stripes ? (n_stripes - band + 7) / 8 : 0) * n_rc;
            int tl = 0;
            if (lane == 0) tl = atomicAdd(&ctr[band], 1);
            tl = __shfl(tl, 0, 64);
            if (tl < ntile) {
                const int sl = tl / n_rc;
                st = band + 8 * sl;
                r0 = (tl - sl * n_rc) * FUP_RC;
                break;
            }
            ++qi;
        }
        if (lane == 0) {
            sh.tile[buf][0] = st;
            sh.tile[buf][1] = r0;
            sh.tile[buf][2] = st >= 0;
        }
        return st;
    };
    // stream a tile's operands into LDS buffer buf (loads first, then one wait, then the LDS writes)
    auto load_tile = [&](int buf, int st, int r0) {
        if (st < 0) return;
        const int r1 = min(Dup, r0 + FUP_RC);
        const int c0 = st * SW;
        PV v[3][FUP_RC / RPI];
        Chunk8<uint16_t> tq[NCH > 0 ? (FUP_RC * NCH + 63) / 64 : 1];
#pragma unroll
        for (int u = 0; u < FUP_RC / RPI; ++u) {
            const int rr = min(r0 + u * RPI + lane / PR, r1 - 1);
            const int cc = min(c0 + (lane % PR) * SV, Ddn - SV);   // rows end on a whole piece (Ddn % V == 0)
            const int64_t off = (int64_t)rr * Ddn + cc;
            v[0][u] = __builtin_nontemporal_load(reinterpret_cast<const PV *>(zq + off));
            v[1][u] = __builtin_nontemporal_load(reinterpret_cast<const PV *>(p + off));
            v[2][u] = *reinterpret_cast<const PV *>(x + off);
        }
#pragma unroll
        for (int u = 0; u < (NCH > 0 ? (FUP_RC * NCH + 63) / 64 : 0); ++u) {
            constexpr int NC1 = NCH > 0 ? NCH : 1;
            const int idx = u * 64 + lane;          // (row, chunk) pairs of the tile
            const int rr = min(r0 + idx / NC1, r1 - 1);
            const int k8 = idx % NC1;
            tq[u] = *reinterpret_cast<const Chunk8<uint16_t> *>(tab + (int64_t)rr * W8 + 8 * (k8 < nch ? k8 : 0));
        }
#pragma unroll
        for (int u = 0; u < FUP_RC / RPI; ++u) {
            const int row = u * RPI + lane / PR, col = (lane % PR) * SV;
#pragma unroll
            for (int k = 0; k < 3; ++k) *reinterpret_cast<PV *>(&sh.op[buf][k][row][col]) = v[k][u];
        }
#pragma unroll
        for (int u = 0; u < (NCH > 0 ? (FUP_RC * NCH + 63) / 64 : 0); ++u) {
            constexpr int NC1 = NCH > 0 ? NCH : 1;
            const int idx = u * 64 + lane;
            if (idx < FUP_RC * NCH) {
                const int row = idx / NC1, k8 = idx % NC1;
                Chunk8<uint16_t> cv = tq[u];
                const unsigned m = (k8 < nch && r0 + row < r1) ? 0u : ~0u;   // rows past the tile read as padding
                cv.q[0] = make_uint4(cv.q[0].x | m, cv.q[0].y | m, cv.q[0].z | m, cv.q[0].w | m);
                sh.tb[buf][row][k8] = cv;
            }
        }
    };
    // write the q of the tile in buffer buf to HBM
    auto store_tile = [&](int buf) {
        const int st = sh.tile[buf][0], r0 = sh.tile[buf][1];
        if (!sh.tile[buf][2]) return;
        const int r1 = min(Dup, r0 + FUP_RC);
        const int c0 = st * SW;
#pragma unroll
        for (int u = 0; u < FUP_RC / RPI; ++u) {
            const int row = u * RPI + lane / PR, col = (lane % PR) * SV;
            const int r = r0 + row, c = c0 + col;
            const PV qv = *reinterpret_cast<const PV *>(&sh.qo[buf][row][col]);
            if (r < r1 && c < Ddn) __builtin_nontemporal_store(qv, reinterpret_cast<PV *>(zq + (int64_t)r * Ddn + c));
        }
    };
    // the compute wavefronts on the tile in buffer buf
    auto compute_tile = [&](int buf) {
        const int st = sh.tile[buf][0], r0 = sh.tile[buf][1];
        const int r1 = min(Dup, r0 + FUP_RC);
        const int sub = lane / L, cl = lane - sub * L;
        const int c = st * SW + cl * V;
        const bool cok = c < Ddn;
        const T *xs = x + (cok ? c : 0);
#pragma unroll
        for (int g0 = wave * G; g0 < FUP_RC; g0 += NCW * G) {
            const int row = g0 + sub;
            const bool rok = r0 + row < r1;
            Chunk8<uint16_t> q[NCH > 0 ? NCH : 1];
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) q[k8] = sh.tb[buf][row][k8];
            int nl = 0;
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) nl += __any(!is_pad<uint16_t>(entry(q[k8], 0))) ? 1 : 0;
            T acc[V];
#pragma unroll
            for (int i = 0; i < V; ++i) acc[i] = T(0);
            // every gather of the row group in one batch (four chunks at a time beyond four)
            if constexpr (NCH >= 1) {
#pragma unroll
                for (int k0 = 0; k0 < NCH; k0 += 4) {
                    const int m = min(4, nl - k0);
                    if (m <= 0) break;
                    switch (m) {
                    case 1: fup_gather<T, V, 1, NCH>(xs, Ddn, q, k0, acc); break;
                    case 2: if constexpr (NCH >= 2) fup_gather<T, V, 2, NCH>(xs, Ddn, q, k0, acc); break;
                    case 3: if constexpr (NCH >= 4) fup_gather<T, V, 3, NCH>(xs, Ddn, q, k0, acc); break;
                    default: if constexpr (NCH >= 4) fup_gather<T, V, 4, NCH>(xs, Ddn, q, k0, acc); break;
                    }
                }
            }
            const VT zv = *reinterpret_cast<const VT *>(&sh.op[buf][0][row][cl * V]);
            const VT pv = vkeep<T, V>(*reinterpret_cast<const VT *>(&sh.op[buf][1][row][cl * V]), has_prev);
            const VT xv = *reinterpret_cast<const VT *>(&sh.op[buf][2][row][cl * V]);
            VT qv;
#pragma unroll
            for (int i = 0; i < V; ++i)
                vset<T, V>(qv, i, sig * (vget<T, V>(zv, i) + t * acc[i]) - cprev * vget<T, V>(pv, i));
            *reinterpret_cast<VT *>(&sh.qo[buf][row][cl * V]) = qv;
            if (rok && cok) {
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    const double qd = vget<T, V>(qv, i), xd = vget<T, V>(xv, i);
                    s[0] += qd * xd;
                    if constexpr (MODE == 2) {
                        const double pd = vget<T, V>(pv, i);
                        s[1] += qd * pd;
                        s[2] += xd * xd;
                        s[3] += xd * pd;
                        s[4] += pd * pd;
                    }
                }
            }
        }
    };

    // prologue: the first tile
    if (loader) {
        int r0;
        const int st = next_tile(0, r0);
        load_tile(0, st, r0);
    }
    __syncthreads();
    int ph = 0;
    for (;; ++ph) {
        const int cur = ph & 1, nxt = cur ^ 1;
        if (!sh.tile[cur][2]) break;   // read after a barrier: uniform over the workgroup
        if (loader) {
            if (ph > 0) store_tile(nxt);   // the q of the tile before
            int r0;
            const int st = next_tile(nxt, r0);
            load_tile(nxt, st, r0);
        } else {
            compute_tile(cur);
        }
        __syncthreads();
    }
    // the last tile's q
    if (loader && ph > 0) store_tile((ph - 1) & 1);
    double tot[NV];
    block_sum<NV>(s, tot);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[(int64_t)blockIdx.x * kPartStride + k] = tot[k];
}

// ---------------------------------------------------------------------------
// a_j and the line-6 coefficients from the up pass's partial sums (the same
// arithmetic as the reference step's k_reduce), then the step is complete:
// jdev advances and q_j is pending.
template <int MODE>
__global__ __launch_bounds__(1024) void k_freduce(const double *__restrict__ partials, int n, Hdr *hdr, double *a,
                                                  int max_steps, int first) {
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
    if constexpr (MODE == 1) {
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
    if (first) hdr->jcall = j;
    hdr->jdev = j + 1;
    hdr->pending = 1;
}

// b_{j+1} = |F_{j+1}| from partial sums (slot stride `stride`), the
// breakdown test and the scales.  In a step (flush = 0) the step counter is
// not advanced: jdev already counts the step whose q produced F_{j+1}.  A flush
// runs only while a q is pending and the run has not broken down.
__global__ __launch_bounds__(1024) void k_fnorm(const double *__restrict__ partials, int stride, int n, Hdr *hdr,
                                                const double *a, double *b, int max_steps, double eps, int flush) {
    if (flush) {
        if (hdr->status != 0 || !hdr->pending) return;
    } else if (frozen(hdr, max_steps)) {
        return;
    }
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[0] += partials[(int64_t)i * stride];
    double tot[1];
    block_sum<1>(s, tot);
    if (threadIdx.x != 0) return;
    const int j = hdr->jdev;   // >= 1: a_j is known, F_{j+1} was just formed
    const double bn = sqrt(tot[0]);
    const double scale = fmax(hdr->scale, fmax(fabs(a[j - 1]), bn));
    b[j] = bn;
    hdr->scale = scale;
    const bool brk = !(bn > 64.0 * eps * scale);   // also true for NaN
    hdr->sig_prev = hdr->sig_cur;
    hdr->sig_cur = brk ? 0.0 : 1.0 / bn;
    hdr->pending = 0;
    if (brk) hdr->status = ED_BREAKDOWN;
}

// The line-6 update of the last step on its own (end of a run of fused
// steps): F_{j+1} = q_j - cx F_j - cp F_{j-1} over q_j, with partial sums of
// the stored squares.  b0, b1, b2 are the buffers (F_{j-1}, F_j, q_j) as they
// were when the run began; after r = jdev - jcall - 1 completed pending steps
// the roles have rotated r times.
template <typename T>
__global__ __launch_bounds__(256) void k_fflush(T *b0, T *b1, T *b2, const Hdr *__restrict__ hdr,
                                                double *__restrict__ part2, int64_t n) {
    if (hdr->status != 0 || !hdr->pending) return;
    const int r = (hdr->jdev - hdr->jcall - 1) % 3;
    const T *p = r == 0 ? b0 : (r == 1 ? b1 : b2);
    const T *x = r == 0 ? b1 : (r == 1 ? b2 : b0);
    T *q = r == 0 ? b2 : (r == 1 ? b0 : b1);
    const double cx = hdr->cx, cp = hdr->cp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double s[1] = {0.0};
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
        }
    }
    for (; i < n; i += stride) {
        const double pv = cp != 0.0 ? (double)p[i] : 0.0;
        const T st = static_cast<T>((double)q[i] - cx * (double)x[i] - cp * pv);
        q[i] = st;
        const double sd = st;
        s[0] += sd * sd;
    }
    double tot[1];
    block_sum<1>(s, tot);
    if (threadIdx.x == 0) part2[blockIdx.x] = tot[0];
}

// ---------------------------------------------------------------------------
// launch shapes
struct FupShape { int L, V; };

// Up-pass tile for an instance: 128-byte row segments (float64: 8 lanes of
// double2, float32: 16 lanes of float2); rows of odd length take one element
// per lane (float64: 16 lanes, float32: 32 lanes).
static FupShape fup_shape(const ed_ham *h) {
    FupShape f;
    const bool even = (h->dim_dn & 1) == 0;
    if (h->dtype == ED_F64) {
        f.L = even ? 8 : 16;
        f.V = even ? 2 : 1;
    } else {
        f.L = even ? 16 : 32;
        f.V = even ? 2 : 1;
    }
    return f;
}

struct FdnShape { int rpb, block, grid; size_t lds; };

static FdnShape fdn_shape(const ed_ham *h) {
    FdnShape d;
    const int es = elem_size(h);
    const int64_t row = h->dim_dn * (int64_t)es;
    d.block = 1024;
    const int64_t by_lds = std::max<int64_t>(1, kLdsBudget / row);
    const int64_t by_fill = std::max<int64_t>(1, (2 * d.block + h->dim_dn - 1) / h->dim_dn);
    d.rpb = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(by_lds, by_fill), h->dim_up));
    d.grid = (int)((h->dim_up + d.rpb - 1) / d.rpb);
    d.lds = (size_t)(d.rpb * row);
    return d;
}

// persistent grid of the up pass: what is resident at once (LDS-bound), at
// most one workgroup per tile and kFupSlots
template <typename T, int MODE, int L, int V, int NCH>
static int fup_grid(size_t lds, int n_tiles) {
    static int cap = 0;
    if (!cap) {
        const void *k = reinterpret_cast<const void *>(k_fup<T, MODE, L, V, NCH>);
        int dev = 0, ncu = 0, occ = 0;
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 320, lds) != hipSuccess)
            return 0;
        cap = std::max(1, ncu * std::max(1, occ));
    }
    return std::min(std::min(cap, std::max(1, n_tiles)), kFupSlots);
}

template <typename T, int MODE, int L, int V>
static int launch_fup_n(const ed_ham *h, const T *x, T *zq, const T *p, const double *b, const WsLayout &w,
                        int max_steps, hipStream_t s, int *grid_out) {
    const int nch = h->w_up >> 3;
    const int sw = L * V;
    const int n_stripes = (int)((h->dim_dn + sw - 1) / sw);
    const int n_rc = (int)((h->dim_up + FUP_RC - 1) / FUP_RC);
    const int n_tiles = n_stripes * n_rc;
    int g = 0;
    const uint16_t *tab = static_cast<const uint16_t *>(h->tab_up);
    const T tt = static_cast<T>(h->t);
#define ED_FUP(NCH)                                                                                                 \
    do {                                                                                                            \
        const size_t lds = sizeof(FupLds<T, L * V, NCH>);                                                           \
        g = fup_grid<T, MODE, L, V, NCH>(lds, n_tiles);                                                             \
        if (!g) return set_error(ED_EDEVICE, "k_fup: occupancy query failed");                                     \
        hipLaunchKernelGGL((k_fup<T, MODE, L, V, NCH>), dim3(g), dim3(320), lds, s, x, zq, p, tab, (int)h->dim_up,  \
                           (int)h->dim_dn, h->w_up, n_rc, n_stripes, tt, b, w.hdr, w.ctr, w.part3, max_steps);      \
    } while (0)
    switch (nch_class(nch) * (nch > 0 ? 1 : 0)) {
    case 0: ED_FUP(0); break;
    case 1: ED_FUP(1); break;
    case 2: ED_FUP(2); break;
    case 4: ED_FUP(4); break;
    default: ED_FUP(8); break;
    }
#undef ED_FUP
    ED_LAUNCHED("k_fup");
    *grid_out = g;
    return ED_OK;
}

template <typename T, int MODE>
static int launch_fup(const ed_ham *h, const T *x, T *zq, const T *p, const double *b, const WsLayout &w,
                      int max_steps, hipStream_t s, int *grid_out) {
    const FupShape f = fup_shape(h);
    if (f.L == 8 && f.V == 2) return launch_fup_n<T, MODE, 8, 2>(h, x, zq, p, b, w, max_steps, s, grid_out);
    if (f.L == 16 && f.V == 2) return launch_fup_n<T, MODE, 16, 2>(h, x, zq, p, b, w, max_steps, s, grid_out);
    if (f.L == 16 && f.V == 1) return launch_fup_n<T, MODE, 16, 1>(h, x, zq, p, b, w, max_steps, s, grid_out);
    return launch_fup_n<T, MODE, 32, 1>(h, x, zq, p, b, w, max_steps, s, grid_out);
}

template <typename T, int MODE, bool PEND, bool ACCV, bool MULTI>
static int launch_fdn_m(const ed_ham *h, const FdnShape &d, T *xq, const T *fj, const T *fjm, T *zdst, T *v,
                        const WsLayout &w, int max_steps, hipStream_t s) {
    const int nch = h->w_dn >> 3;
    const uint16_t *tab = static_cast<const uint16_t *>(h->tab_dn);
    const T tt = static_cast<T>(h->t), uu = static_cast<T>(h->U);
#define ED_FDN(NCH)                                                                                                \
    hipLaunchKernelGGL((k_fdn<T, MODE, PEND, ACCV, NCH, MULTI>), dim3(d.grid), dim3(d.block), d.lds, s, xq, fj, fjm, \
                       zdst, v, w.y, tab, h->st_up, h->st_dn, (int)h->dim_up, (int)h->dim_dn, h->w_dn, d.rpb, tt, uu,   \
                       w.hdr, w.ctr, w.part, max_steps)
    switch (nch_class(nch) * (nch > 0 ? 1 : 0)) {
    case 0: ED_FDN(0); break;
    case 1: ED_FDN(1); break;
    case 2: ED_FDN(2); break;
    case 4: ED_FDN(4); break;
    default: ED_FDN(8); break;
    }
#undef ED_FDN
    ED_LAUNCHED("k_fdn");
    return ED_OK;
}

template <typename T, int MODE, bool PEND, bool ACCV>
static int launch_fdn(const ed_ham *h, T *xq, const T *fj, const T *fjm, T *zdst, T *v, const WsLayout &w,
                      int max_steps, hipStream_t s, int *grid_out) {
    const FdnShape d = fdn_shape(h);
    *grid_out = d.grid;
    if (d.rpb > 1) return launch_fdn_m<T, MODE, PEND, ACCV, true>(h, d, xq, fj, fjm, zdst, v, w, max_steps, s);
    return launch_fdn_m<T, MODE, PEND, ACCV, false>(h, d, xq, fj, fjm, zdst, v, w, max_steps, s);
}

// every k_fdn variant may take up to kLdsBudget bytes of LDS; set once,
// outside any stream capture
template <typename T, int MODE, bool PEND, bool ACCV, bool MULTI>
static hipError_t fdn_attr_m() {
    const void *ks[] = {reinterpret_cast<const void *>(k_fdn<T, MODE, PEND, ACCV, 0, MULTI>),
                        reinterpret_cast<const void *>(k_fdn<T, MODE, PEND, ACCV, 1, MULTI>),
                        reinterpret_cast<const void *>(k_fdn<T, MODE, PEND, ACCV, 2, MULTI>),
                        reinterpret_cast<const void *>(k_fdn<T, MODE, PEND, ACCV, 4, MULTI>),
                        reinterpret_cast<const void *>(k_fdn<T, MODE, PEND, ACCV, 8, MULTI>)};
    for (const void *k : ks) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int MODE>
static hipError_t fdn_attrs() {
    const hipError_t es[] = {fdn_attr_m<T, MODE, false, false, false>(), fdn_attr_m<T, MODE, false, false, true>(),
                             fdn_attr_m<T, MODE, false, true, false>(),  fdn_attr_m<T, MODE, false, true, true>(),
                             fdn_attr_m<T, MODE, true, false, false>(),  fdn_attr_m<T, MODE, true, false, true>(),
                             fdn_attr_m<T, MODE, true, true, false>(),   fdn_attr_m<T, MODE, true, true, true>()};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

int fused_prepare() {
    static int rc = -1000;
    if (rc != -1000) return rc;
    hipError_t e = fdn_attrs<double, 1>();
    if (e == hipSuccess) e = fdn_attrs<float, 2>();
    rc = hip_check(e, "hipFuncSetAttribute(k_fdn)");
    return rc;
}

bool fused_eligible(const ed_ham *h) {
    if (h->cplx || h->eb_up == 4 || h->eb_dn == 4) return false;
    if (h->dim_dn * (int64_t)elem_size(h) > kLdsBudget) return false;   // whole rows in LDS
    return true;
}

template <typename T, int MODE>
static int step_t(const ed_ham *h, T *fp, T *f, T *q, bool pending, double *a, double *b, T *v, const WsLayout &w,
                  int max_steps, hipStream_t s, hipEvent_t *ev) {
    const double eps = MODE == 1 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -24);
    int gd = 0, gu = 0, rc;
    if (ev) ED_HIP(hipEventRecord(ev[0], s));
    // F_{j+1}: formed over q (pending) or read from f; Z over fp (pending) or into q
    T *xbuf = pending ? q : f;
    T *zbuf = pending ? fp : q;
    T *prev = pending ? f : fp;   // F_j of the recurrence term
    if (pending) {
        rc = v ? launch_fdn<T, MODE, true, true>(h, q, f, fp, fp, v, w, max_steps, s, &gd)
               : launch_fdn<T, MODE, true, false>(h, q, f, fp, fp, v, w, max_steps, s, &gd);
    } else {
        rc = v ? launch_fdn<T, MODE, false, true>(h, f, f, f, q, v, w, max_steps, s, &gd)
               : launch_fdn<T, MODE, false, false>(h, f, f, f, q, v, w, max_steps, s, &gd);
    }
    if (rc) return rc;
    if (ev) ED_HIP(hipEventRecord(ev[1], s));
    if (pending) {
        hipLaunchKernelGGL(k_fnorm, dim3(1), dim3(1024), 0, s, w.part, kPartStride, gd, w.hdr, a, b, max_steps, eps, 0);
        ED_LAUNCHED("k_fnorm");
    }
    if (ev) ED_HIP(hipEventRecord(ev[2], s));
    rc = launch_fup<T, MODE>(h, xbuf, zbuf, prev, b, w, max_steps, s, &gu);
    if (rc) return rc;
    if (ev) ED_HIP(hipEventRecord(ev[3], s));
    hipLaunchKernelGGL(k_freduce<MODE>, dim3(1), dim3(1024), 0, s, w.part3, gu, w.hdr, a, max_steps, pending ? 0 : 1);
    ED_LAUNCHED("k_freduce");
    if (ev) ED_HIP(hipEventRecord(ev[4], s));
    return ED_OK;
}

int fused_step(const ed_ham *h, void *fp, void *f, void *q, bool pending, double *a, double *b, void *v,
               const WsLayout &w, int max_steps, hipStream_t s, hipEvent_t *ev) {
    if (h->dtype == ED_F64)
        return step_t<double, 1>(h, (double *)fp, (double *)f, (double *)q, pending, a, b, (double *)v, w, max_steps,
                                 s, ev);
    return step_t<float, 2>(h, (float *)fp, (float *)f, (float *)q, pending, a, b, (float *)v, w, max_steps, s, ev);
}

int fused_flush(const ed_ham *h, void *fp, void *f, void *q, const double *a, double *b, const WsLayout &w,
                int max_steps, hipStream_t s, hipEvent_t *ev) {
    const int64_t n = h->dim_up * h->dim_dn;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, kUpdBlocks));
    const double eps = h->dtype == ED_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -24);
    if (ev) ED_HIP(hipEventRecord(ev[0], s));
    if (h->dtype == ED_F64)
        hipLaunchKernelGGL(k_fflush<double>, dim3(g), dim3(256), 0, s, (double *)fp, (double *)f, (double *)q, w.hdr,
                           w.part2, n);
    else
        hipLaunchKernelGGL(k_fflush<float>, dim3(g), dim3(256), 0, s, (float *)fp, (float *)f, (float *)q, w.hdr,
                           w.part2, n);
    ED_LAUNCHED("k_fflush");
    if (ev) ED_HIP(hipEventRecord(ev[1], s));
    hipLaunchKernelGGL(k_fnorm, dim3(1), dim3(1024), 0, s, w.part2, 1, g, w.hdr, a, b, max_steps, eps, 1);
    ED_LAUNCHED("k_fnorm");
    if (ev) ED_HIP(hipEventRecord(ev[2], s));
    return ED_OK;
}

}  // namespace ed

namespace ed {
namespace {

int check_run(const ed_ham *h, const ed_lanczos *st, void *ws, int32_t n, const char *who) {
    int rc = check_ham(h, who);
    if (rc) return rc;
    if (!st || !st->f_prev || !st->f_cur || !st->f_next || !st->a || !st->b || !ws)
        return set_error(ED_EINVAL, "%s: missing Lanczos buffers or workspace", who);
    if (st->f_prev == st->f_cur || st->f_cur == st->f_next || st->f_prev == st->f_next)
        return set_error(ED_EINVAL, "%s: the three Lanczos vectors must be distinct", who);
    if (st->max_steps < 1) return set_error(ED_EINVAL, "%s: max_steps must be >= 1", who);
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return set_error(ED_EINVAL, "%s: ws not 256-byte aligned", who);
    if (n < 1) return set_error(ED_EINVAL, "%s: n must be >= 1", who);
    return ED_OK;
}

void rotate_roles(void *&fp, void *&f, void *&q) {
    void *old = fp;
    fp = f;
    f = q;
    q = old;
}

// n fused steps and the closing update, asynchronous on s; ev (5n + 3 events)
// brackets every kernel when given.
int run_fused(const ed_ham *h, ed_lanczos *st, int32_t n, void *ws, hipStream_t s, hipEvent_t *ev) {
    const WsLayout w = ws_layout(h, ws, st->max_steps);
    void *b0 = st->f_prev, *b1 = st->f_cur, *b2 = st->f_next;
    void *fp = b0, *f = b1, *q = b2;
    for (int k = 0; k < n; ++k) {
        int rc = fused_step(h, fp, f, q, k > 0, st->a, st->b, nullptr, w, st->max_steps, s, ev ? ev + 5 * k : nullptr);
        if (rc) return rc;
        if (k > 0) rotate_roles(fp, f, q);
    }
    return fused_flush(h, b0, b1, b2, st->a, st->b, w, st->max_steps, s, ev ? ev + 5 * n : nullptr);
}

}  // namespace
}  // namespace ed

using namespace ed;

extern "C" {

int ed_lanczos_steps(const ed_ham *h, ed_lanczos *st, int32_t n, void *ws, void *stream) {
    clear_error();
    int rc = check_run(h, st, ws, n, "ed_lanczos_steps");
    if (rc) return rc;
    if (!fused_eligible(h)) {
        for (int k = 0; k < n; ++k) {
            rc = ed_lanczos_step(h, st, ws, stream);
            if (rc) return rc;
        }
        return ED_OK;
    }
    rc = fused_prepare();
    if (rc) return rc;
    rc = run_fused(h, st, n, ws, static_cast<hipStream_t>(stream), nullptr);
    if (rc) return rc;
    for (int k = 0; k < n; ++k) {
        void *old = st->f_prev;
        st->f_prev = st->f_cur;
        st->f_cur = st->f_next;
        st->f_next = old;
    }
    st->j += n;
    return ED_OK;
}

int ed_lanczos_steps_timed(const ed_ham *h, ed_lanczos *st, int32_t n, void *ws, void *stream, double *ms) {
    clear_error();
    int rc = check_run(h, st, ws, n, "ed_lanczos_steps_timed");
    if (rc) return rc;
    if (!ms) return set_error(ED_EINVAL, "ed_lanczos_steps_timed: ms is NULL");
    if (!fused_eligible(h)) return set_error(ED_EINVAL, "ed_lanczos_steps_timed: the instance takes the reference step");
    rc = fused_prepare();
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nev = 5 * n + 3;
    std::vector<hipEvent_t> ev(nev, nullptr);
    for (int k = 0; k < nev && rc == ED_OK; ++k) rc = hip_check(hipEventCreate(&ev[k]), "hipEventCreate");
    if (rc == ED_OK) rc = run_fused(h, st, n, ws, s, ev.data());
    if (rc == ED_OK) rc = hip_check(hipEventSynchronize(ev[5 * n + 2]), "hipEventSynchronize");
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < n && rc == ED_OK; ++k)
        for (int i = 0; i < 4 && rc == ED_OK; ++i) {
            float t = 0.f;
            rc = hip_check(hipEventElapsedTime(&t, ev[5 * k + i], ev[5 * k + i + 1]), "hipEventElapsedTime");
            acc[i] += t;
        }
    for (int i = 0; i < 2 && rc == ED_OK; ++i) {
        float t = 0.f;
        rc = hip_check(hipEventElapsedTime(&t, ev[5 * n + i], ev[5 * n + i + 1]), "hipEventElapsedTime");
        acc[4 + i] = t;
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    for (int i = 0; i < 4; ++i) ms[i] = acc[i] / n;
    ms[4] = acc[4];
    ms[5] = acc[5];
    for (int k = 0; k < n; ++k) {
        void *old = st->f_prev;
        st->f_prev = st->f_cur;
        st->f_cur = st->f_next;
        st->f_next = old;
    }
    st->j += n;
    return ED_OK;
}

}  // extern "C"
