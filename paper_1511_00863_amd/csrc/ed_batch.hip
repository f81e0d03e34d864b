// Batched ground-state runs: many independent instances (different U, t and
// fillings, hence uneven dimensions) taken through the Lanczos iteration
// (Alg. 1, mixed form: float32 vectors, float64 scalars) by ONE persistent
// cooperative kernel.  Every step of every live instance is the same five
// phases as the single-instance path (up part, down part with partial dots,
// a_j, update with partial norms, b_{j+1}); in each phase the workgroups
// share out the union of the live instances' tiles, and a grid barrier
// separates the phases.  Each instance tests its own convergence on the
// device: E0(j), the lowest eigenvalue of T_j (Sec. 2.2), comes from a
// 64-way Sturm-count multisection run by one wavefront, and the instance
// stops when |E0(j) - E0(j-1)| < tol at two consecutive steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ed.h"
#include "ed_common.h"
#include "ed_internal.h"
#include "ed_launch.h"

namespace ed {

#define ED_GLOBAL __attribute__((address_space(1)))

constexpr int kBatchBlock = 256;
constexpr int kBatchUpRows = 64;            // rows per up tile at least: amortises the queue's atomic and barriers
constexpr int kBatchLds = 32 * 1024;        // rows of up to 8192 floats; four workgroups per CU
constexpr int kBatchShm = kBatchLds + 16;   // the rows and the zero after a single row
constexpr int64_t kUpdChunk = 65536;         // elements per update tile
constexpr int kConverged = 10;
constexpr int kBadStart = 100;
constexpr unsigned long long kSpinLimit = 1ull << 24;   // about a second of s_sleep(2)

struct BInst {
    // set by the host
    int Dup, Ddn, W8u, W8d;
    int R, V, rc, n_stripes, n_rc;   // rows and columns per lane of the up-part tile
    int up_tiles, rpb, dn_tiles, upd_tiles;
    int64_t n, part_off, part2_off;
    // global-memory pointers: typed so, the kernel's loads through pointers
    // read from this descriptor are global (not flat) instructions
    const ED_GLOBAL uint16_t *tab_up, *tab_dn;
    const ED_GLOBAL uint64_t *st_up, *st_dn;
    const ED_GLOBAL float *f1;
    ED_GLOBAL float *vec[3];
    ED_GLOBAL double *a, *b, *e;
    double t, U;
    // device state
    int j, status, rot, conv;
    double sig_cur, sig_prev, cx, cp, scale, pad;
};

// The arrival counter and the generation word sit on cache lines of their
// own, so waiters polling the generation do not contend with arrivals.
struct GridBar {
    unsigned count;
    unsigned pad0[31];
    unsigned gen;
    unsigned pad1[31];
    int err;
    int pad2;
    unsigned long long phase[6];   // wall-clock ticks per phase (init, up, down, a_j, update, b_j) seen by WG 0
    unsigned pad3[16];
    // up-phase tile counters: [step parity][queue][own 128-byte line]
    unsigned upq[2][8][32];
};

// phase bookkeeping of workgroup 0 (the other workgroups do not record)
struct PhaseClock {
    unsigned long long last;
    __device__ void start() { last = wall_clock64(); }
    __device__ void lap(GridBar *gb, int k) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const unsigned long long now = wall_clock64();
            gb->phase[k] += now - last;
            last = now;
        }
    }
};

__device__ __forceinline__ bool b_live(const BInst &I, int max_steps) { return I.status == 0 && I.j < max_steps; }

// All workgroups wait until all have arrived.  Each arrival publishes this
// workgroup's writes once (release: L2 write-back) and each departure makes
// the others' writes visible once (acquire: L2 invalidate).  Waiters poll
// with relaxed loads: an acquire load in the loop would invalidate the XCD's
// L2 on every poll and evict the lines that workgroups still working in the
// phase depend on.  Spins are bounded: a timeout sets gb->err and releases
// the waiter, so the kernel always ends.
__device__ void grid_sync(GridBar *gb) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned g = __hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (arrived == gridDim.x) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&gb->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while (__hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit) {
                    atomicExch(&gb->err, 1);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
}

// Walks the instances in order; (ci, cbase) is a cursor that only moves
// forward because a workgroup visits its tiles in increasing order.
enum TileKind { kUpT, kDnT, kUpdT, kInitT };

__device__ __forceinline__ int tiles_of(const BInst &I, TileKind k) {
    return k == kUpT ? I.up_tiles : (k == kDnT ? I.dn_tiles : I.upd_tiles);
}

__device__ __forceinline__ bool next_tile(const BInst *inst, int ni, int max_steps, TileKind kind, int64_t tg,
                                          int &ci, int64_t &cbase) {
    while (ci < ni) {
        const BInst &I = inst[ci];
        const bool use = kind == kInitT ? true : b_live(I, max_steps);
        const int cnt = use ? tiles_of(I, kind) : 0;
        if (tg < cbase + cnt) return true;
        cbase += cnt;
        ++ci;
    }
    return false;
}

__device__ int sturm_count(const double *a, const double *boff, int m, double x, double pivmin) {
    int cnt = 0;
    double d = a[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
    for (int k = 1; k < m; ++k) {
        d = (a[k] - x) - boff[k - 1] * boff[k - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// Lowest eigenvalue of T_m (diag a[0..m-1], off-diagonal boff[0..m-2]) by one
// wavefront: each round 64 lanes test 64 interior points of the bracket.
__device__ double ritz_lowest_wave(const double *a, const double *boff, int m) {
    const int lane = threadIdx.x & 63;
    double lo = INFINITY, hi = -INFINITY, bmax = 0.0;
    for (int k = lane; k < m; k += 64) {
        const double r = (k > 0 ? fabs(boff[k - 1]) : 0.0) + (k < m - 1 ? fabs(boff[k]) : 0.0);
        lo = fmin(lo, a[k] - r);
        hi = fmax(hi, a[k] + r);
        if (k < m - 1) bmax = fmax(bmax, fabs(boff[k]));
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
        bmax = fmax(bmax, __shfl_xor(bmax, o, 64));
    }
    const double pivmin = fmax(2.2250738585072014e-308 * fmax(1.0, bmax * bmax), 1e-300);
    const double pad = 4e-16 * fmax(fabs(lo), fabs(hi)) + pivmin;
    lo -= pad;
    hi += pad;
    for (int round = 0; round < 9; ++round) {
        const double w = (hi - lo) / 65.0;
        const double x = lo + w * (lane + 1);
        const int cnt = sturm_count(a, boff, m, x, pivmin);
        const unsigned long long mask = __ballot(cnt >= 1);
        if (mask == 0ull) {
            lo = lo + 64.0 * w;
        } else {
            const int f = __ffsll((long long)mask) - 1;
            const double nhi = lo + w * (f + 1), nlo = lo + w * f;
            lo = nlo;
            hi = nhi;
        }
    }
    return 0.5 * (lo + hi);
}

__global__ __launch_bounds__(kBatchBlock, 4) void k_batch(BInst *__restrict__ inst, int ni, double *__restrict__ part,
                                                       double *__restrict__ part2, GridBar *gb, int max_steps,
                                                       double tol) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);
    __shared__ int s_any;
    const int64_t G = gridDim.x;
    PhaseClock clk;
    clk.start();

    // ---- start: F_1 = copy of f1, |f1|^2 partials
    {
        int ci = 0;
        int64_t cb = 0;
        for (int64_t tg = blockIdx.x; next_tile(inst, ni, max_steps, kInitT, tg, ci, cb); tg += G) {
            const BInst &I = inst[ci];
            const int local = (int)(tg - cb);
            const int64_t lo = (int64_t)local * kUpdChunk, hi = min(I.n, lo + kUpdChunk);
            double s[1] = {0.0};
            const int64_t B = blockDim.x;
            int64_t k = lo + threadIdx.x;
            for (; k + 3 * B < hi; k += 4 * B) {
                float v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = I.f1[k + u * B];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    I.vec[0][k + u * B] = v[u];
                    s[0] += (double)v[u] * (double)v[u];
                }
            }
            for (; k < hi; k += B) {
                const float v = I.f1[k];
                I.vec[0][k] = v;
                s[0] += (double)v * (double)v;
            }
            double tot[1];
            block_sum<1>(s, tot);
            if (threadIdx.x == 0) part2[I.part2_off + local] = tot[0];
            __syncthreads();
        }
    }
    grid_sync(gb);
    clk.lap(gb, 0);
    for (int i = blockIdx.x; i < ni; i += G) {
        BInst &I = inst[i];
        double s[1] = {0.0};
        for (int k = threadIdx.x; k < I.upd_tiles; k += blockDim.x) s[0] += part2[I.part2_off + k];
        double tot[1];
        block_sum<1>(s, tot);
        if (threadIdx.x == 0) {
            const bool ok = tot[0] > 0.0 && tot[0] < INFINITY;
            I.sig_cur = ok ? 1.0 / sqrt(tot[0]) : 0.0;
            I.sig_prev = 0.0;
            I.cx = I.cp = 0.0;
            I.scale = 0.0;
            I.j = 0;
            I.rot = 0;
            I.conv = 0;
            I.status = ok ? 0 : kBadStart;
            I.b[0] = 0.0;
        }
        __syncthreads();
    }
    grid_sync(gb);
    clk.lap(gb, 0);

    for (int step = 0; step < max_steps; ++step) {
        if (threadIdx.x == 0) {
            int any = 0;
            for (int i = 0; i < ni; ++i) any |= b_live(inst[i], max_steps) ? 1 : 0;
            s_any = any && !__hip_atomic_load(&gb->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (!s_any) break;

        // ---- up part (Eq. 4): T = t * up(F_j) into the next buffer.  The
        // stripes of the live instances are numbered on from one instance to
        // the next, and queue q = blockIdx % 8 holds the tiles of the stripes
        // numbered q (mod 8) (so a stripe's tiles share one XCD's L2 when
        // workgroups are placed round-robin over the XCDs); its workgroups
        // take tiles in order from an atomic counter, which keeps the tiles
        // in flight within a narrow window of stripes, as in-order hardware
        // dispatch would.  Every queue has workgroups (gridDim.x >= 8), so
        // all tiles are processed whatever the placement.
        {
            const int xq = blockIdx.x & 7;
            unsigned *ctr = &gb->upq[step & 1][xq][0];
            __shared__ unsigned s_tile;
            if (threadIdx.x == 0) s_tile = atomicAdd(ctr, 1u);
            __syncthreads();
            int64_t qi = s_tile;
            __syncthreads();
            // stripes are numbered on across the live instances, and stripe
            // number g goes to queue g mod 8: every queue gets the same share
            // (to one stripe) and the queues move through the instances together
            int ci = 0;
            int64_t cb = 0;
            int gcum = 0;      // stripes of the live instances before inst[ci]
            int off = xq;      // first stripe of inst[ci] that falls to this queue
            while (true) {
                bool found = false;
                while (ci < ni) {
                    const BInst &I = inst[ci];
                    const bool live = b_live(I, max_steps);
                    off = (xq - (gcum & 7) + 8) & 7;
                    const int cnt = live && off < I.n_stripes ? I.n_rc * ((I.n_stripes - off + 7) >> 3) : 0;
                    if (qi < cb + cnt) {
                        found = true;
                        break;
                    }
                    cb += cnt;
                    if (live) gcum += I.n_stripes;
                    ++ci;
                }
                if (!found) break;
                unsigned pre = 0;
                if (threadIdx.x == 0) pre = atomicAdd(ctr, 1u);   // next tile, in flight during this one
                const BInst &I = inst[ci];
                const int local = (int)(qi - cb);
                const int sl = local / I.n_rc, rci = local - sl * I.n_rc;
                const int s = sl * 8 + off;
                const float *x = (const float *)I.vec[I.rot];
                float *out = (float *)I.vec[(I.rot + 1) % 3];
                const uint16_t *tab = (const uint16_t *)I.tab_up;
                const float t = (float)I.t;
                if (I.V == 2) {   // the plan guarantees W8 <= 32 and an even row length
                    switch (nch_class(I.W8u >> 3)) {
                    case 1: up_tile_vec<float, 2, 1>(x, out, tab, I.Dup, I.Ddn, I.W8u, I.rc, s, rci, t); break;
                    case 2: up_tile_vec<float, 2, 2>(x, out, tab, I.Dup, I.Ddn, I.W8u, I.rc, s, rci, t); break;
                    default: up_tile_vec<float, 2, 4>(x, out, tab, I.Dup, I.Ddn, I.W8u, I.rc, s, rci, t); break;
                    }
                } else {
                    switch (nch_class(I.W8u >> 3)) {
                    case 1: up_tile_wide<float, 1>(x, out, tab, I.Dup, I.Ddn, I.W8u, I.rc, s, rci, t); break;
                    case 2: up_tile_wide<float, 2>(x, out, tab, I.Dup, I.Ddn, I.W8u, I.rc, s, rci, t); break;
                    default: up_tile_wide<float, 4>(x, out, tab, I.Dup, I.Ddn, I.W8u, I.rc, s, rci, t); break;
                    }
                }
                if (threadIdx.x == 0) s_tile = pre;
                __syncthreads();
                qi = s_tile;
                __syncthreads();
            }
            // the other parity's counters were last used a step ago: clear them
            // for the next step (the barriers in between order this)
            if (blockIdx.x == 0 && threadIdx.x < 8)
                __hip_atomic_store(&gb->upq[(step + 1) & 1][threadIdx.x][0], 0u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        grid_sync(gb);
        clk.lap(gb, 1);

        // ---- down part (Eq. 5) + U term + recurrence, partial dots
        {
            int ci = 0;
            int64_t cb = 0;
            for (int64_t tg = blockIdx.x; next_tile(inst, ni, max_steps, kDnT, tg, ci, cb); tg += G) {
                const BInst &I = inst[ci];
                const int local = (int)(tg - cb);
                const int r0 = local * I.rpb, nr = min(I.rpb, I.Dup - r0);
                const int64_t base = (int64_t)r0 * I.Ddn;
                const float *x = (const float *)I.vec[I.rot];
                float *io = (float *)I.vec[(I.rot + 1) % 3];
                const float *p = (const float *)I.vec[(I.rot + 2) % 3];
                __syncthreads();
                stage_rows<float>(x + base, xs, nr * I.Ddn);
                if (I.rpb == 1 && threadIdx.x == 0) xs[I.Ddn] = 0.f;   // the target of padding entries
                __syncthreads();
                double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                const bool has_prev = I.j > 0;
                const float sig = (float)I.sig_cur;
                const float cprev = (float)(I.b[I.j] * I.sig_prev);
                const uint16_t *tdn = (const uint16_t *)I.tab_dn;
                const uint64_t *su = (const uint64_t *)I.st_up + r0, *sd = (const uint64_t *)I.st_dn;
                const float tt = (float)I.t, uu = (float)I.U;
                if (I.W8d == 0)   // the down species cannot hop: no table to read
                    down_rows<float, 2, 0, true>(xs, io, p, tdn, su, sd, I.Ddn, I.W8d, 0, nr * I.Ddn, base, tt, uu, sig, cprev,
                                                 has_prev, s);
                else if (I.rpb > 1)
                    down_rows<float, 2, 4, true>(xs, io, p, tdn, su, sd, I.Ddn, I.W8d, 0, nr * I.Ddn, base, tt, uu, sig, cprev,
                                                 has_prev, s);
                else
                    down_rows<float, 2, 4, false, true, true>(xs, io, p, tdn, su, sd, I.Ddn, I.W8d, 0, nr * I.Ddn, base, tt,
                                                              uu, sig, cprev, has_prev, s);
                double tot[5];
                block_sum<5>(s, tot);
                if (threadIdx.x == 0)
                    for (int k = 0; k < 5; ++k) part[I.part_off + (int64_t)local * 5 + k] = tot[k];
            }
        }
        grid_sync(gb);
        clk.lap(gb, 2);

        // ---- a_j and the update coefficients (Gram projection, float64)
        for (int i = blockIdx.x; i < ni; i += G) {
            BInst &I = inst[i];
            if (!b_live(I, max_steps)) continue;
            double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int k = threadIdx.x; k < I.dn_tiles; k += blockDim.x)
                for (int u = 0; u < 5; ++u) s[u] += part[I.part_off + (int64_t)k * 5 + u];
            double tot[5];
            block_sum<5>(s, tot);
            if (threadIdx.x == 0) {
                const double sx = I.sig_cur, sp = I.sig_prev;
                const double qx = sx * tot[0], qp = sp * tot[1];
                const double xx = sx * sx * tot[2], xp = sx * sp * tot[3], pp = sp * sp * tot[4];
                double alpha, beta = 0.0;
                if (I.j > 0) {
                    const double det = xx * pp - xp * xp;
                    alpha = (pp * qx - xp * qp) / det;
                    beta = (xx * qp - xp * qx) / det;
                } else {
                    alpha = qx / xx;
                }
                I.a[I.j] = alpha;
                I.cx = alpha * sx;
                I.cp = I.j > 0 ? beta * sp : 0.0;
            }
            __syncthreads();
        }
        grid_sync(gb);
        clk.lap(gb, 3);

        // ---- F_{j+1} = q - cx F_j - cp F_{j-1}, partial norms
        {
            int ci = 0;
            int64_t cb = 0;
            for (int64_t tg = blockIdx.x; next_tile(inst, ni, max_steps, kUpdT, tg, ci, cb); tg += G) {
                const BInst &I = inst[ci];
                const int local = (int)(tg - cb);
                const int64_t lo = (int64_t)local * kUpdChunk, hi = min(I.n, lo + kUpdChunk);
                const float *x = (const float *)I.vec[I.rot];
                float *q = (float *)I.vec[(I.rot + 1) % 3];
                const float *p = (const float *)I.vec[(I.rot + 2) % 3];
                const double cx = I.cx, cp = I.cp;
                double s[1] = {0.0};
                const int64_t B = blockDim.x;
                int64_t k = lo + threadIdx.x;
                // 16-byte loads (four elements per lane, two in flight) when the
                // vectors are 16-byte aligned; chunk starts are multiples of 4
                const bool al = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(q) |
                                  reinterpret_cast<uintptr_t>(p)) & 15) == 0;
                if (al) {
                    const int64_t nv = (hi - lo) >> 2;
                    const float4 *x4 = reinterpret_cast<const float4 *>(x + lo);
                    const float4 *p4 = reinterpret_cast<const float4 *>(p + lo);
                    float4 *q4 = reinterpret_cast<float4 *>(q + lo);
                    const bool use_p = cp != 0.0;
                    auto upd4 = [&](const float4 &xv, const float4 &qv, const float4 &pv) {
                        float4 st;
                        st.x = (float)((double)qv.x - cx * (double)xv.x - cp * (double)pv.x);
                        st.y = (float)((double)qv.y - cx * (double)xv.y - cp * (double)pv.y);
                        st.z = (float)((double)qv.z - cx * (double)xv.z - cp * (double)pv.z);
                        st.w = (float)((double)qv.w - cx * (double)xv.w - cp * (double)pv.w);
                        s[0] += (double)st.x * (double)st.x + (double)st.y * (double)st.y +
                                (double)st.z * (double)st.z + (double)st.w * (double)st.w;
                        return st;
                    };
                    int64_t v = threadIdx.x;
                    for (; v + B < nv; v += 2 * B) {
                        const float4 xa = x4[v], qa = q4[v], xb = x4[v + B], qb = q4[v + B];
                        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                        const float4 pa = use_p ? p4[v] : z, pb = use_p ? p4[v + B] : z;
                        q4[v] = upd4(xa, qa, pa);
                        q4[v + B] = upd4(xb, qb, pb);
                    }
                    for (; v < nv; v += B) {
                        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                        q4[v] = upd4(x4[v], q4[v], use_p ? p4[v] : z);
                    }
                    k = lo + 4 * nv + threadIdx.x;   // the tail (n not a multiple of 4)
                } else {
                    for (; k + 3 * B < hi; k += 4 * B) {   // four independent elements in flight
                        float xv[4], qv[4], pv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            xv[u] = x[k + u * B];
                            qv[u] = q[k + u * B];
                            pv[u] = cp != 0.0 ? p[k + u * B] : 0.f;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float st = (float)((double)qv[u] - cx * (double)xv[u] - cp * (double)pv[u]);
                            q[k + u * B] = st;
                            s[0] += (double)st * (double)st;
                        }
                    }
                }
                for (; k < hi; k += B) {
                    double qv = (double)q[k] - cx * (double)x[k];
                    if (cp != 0.0) qv -= cp * (double)p[k];
                    const float st = (float)qv;
                    q[k] = st;
                    s[0] += (double)st * (double)st;
                }
                double tot[1];
                block_sum<1>(s, tot);
                if (threadIdx.x == 0) part2[I.part2_off + local] = tot[0];
                __syncthreads();
            }
        }
        grid_sync(gb);
        clk.lap(gb, 4);

        // ---- b_{j+1}, breakdown, E0(j+1) and the convergence test
        for (int i = blockIdx.x; i < ni; i += G) {
            BInst &I = inst[i];
            if (!b_live(I, max_steps)) continue;
            double s[1] = {0.0};
            for (int k = threadIdx.x; k < I.upd_tiles; k += blockDim.x) s[0] += part2[I.part2_off + k];
            double tot[1];
            block_sum<1>(s, tot);
            __shared__ int s_brk;
            __shared__ int s_m;
            if (threadIdx.x == 0) {
                const int j = I.j;
                const double bn = sqrt(tot[0]);
                const double scale = fmax(I.scale, fmax(fabs(I.a[j]), bn));
                I.b[j + 1] = bn;
                I.scale = scale;
                const bool brk = !(bn > 64.0 * 5.960464477539063e-08 * scale);
                I.sig_prev = I.sig_cur;
                I.sig_cur = brk ? 0.0 : 1.0 / bn;
                I.j = j + 1;
                I.rot = (I.rot + 1) % 3;
                s_brk = brk ? 1 : 0;
                s_m = j + 1;
            }
            __syncthreads();
            if (threadIdx.x < 64) {
                const int m = s_m;
                const double e = ritz_lowest_wave((const double *)I.a, (const double *)I.b + 1, m);
                if (threadIdx.x == 0) {
                    I.e[m] = e;
                    if (m >= 2 && fabs(e - I.e[m - 1]) < tol) I.conv += 1; else I.conv = 0;
                    if (s_brk) I.status = ED_BREAKDOWN;
                    else if (I.conv >= 2) I.status = kConverged;
                }
            }
            __syncthreads();
        }
        grid_sync(gb);
        clk.lap(gb, 5);
    }
}

static int batch_grid(int *grid) {
    static int cached = 0;
    if (!cached) {
        int dev = 0, ncu = 0, occ = 0;
        ED_HIP(hipGetDevice(&dev));
        ED_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        ED_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, kBatchShm));
        ED_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(k_batch),
                                                            kBatchBlock, kBatchShm));
        if (occ < 1) return set_error(ED_EDEVICE, "k_batch cannot be resident on a CU");
        cached = ncu * occ;
        if (cached < 8) return set_error(ED_EDEVICE, "k_batch needs at least 8 resident workgroups");
    }
    *grid = cached;
    return ED_OK;
}

struct BatchPlan {
    std::vector<BInst> inst;
    int64_t part_doubles = 0, part2_doubles = 0;
};

static int plan_batch(const ed_batch_item *items, int n, int32_t max_steps, BatchPlan &plan, bool fill_ptrs) {
    plan.inst.assign(n, BInst{});
    plan.part_doubles = plan.part2_doubles = 0;
    for (int i = 0; i < n; ++i) {
        const ed_ham &h = items[i].h;
        int rc = check_real(&h, "ed_ground_energy_batch");
        if (rc) return rc;
        if (h.dtype != ED_F32) return set_error(ED_EINVAL, "ed_ground_energy_batch: item %d is not ED_F32", i);
        if (wide_up(&h) || wide_dn(&h))
            return set_error(ED_EINVAL, "ed_ground_energy_batch: item %d has 32-bit tables", i);
        // the persistent kernel's registers serve every phase: its tiles hold at most 4 table chunks
        if (h.w_dn > 32 || h.w_up > 32) return set_error(ED_EOVERFLOW, "ed_ground_energy_batch: table stride above 32");
        if (h.w_up == 0) return set_error(ED_EINVAL, "ed_ground_energy_batch: item %d has no up-spin hopping", i);
        if (h.dim_dn * 4 > kBatchLds) return set_error(ED_EOVERFLOW, "ed_ground_energy_batch: rows above 32 KB");
        if (fill_ptrs) {
            const ed_batch_item &it = items[i];
            if (!it.f1 || !it.vec[0] || !it.vec[1] || !it.vec[2] || !it.a || !it.b)
                return set_error(ED_EINVAL, "ed_ground_energy_batch: item %d has a NULL buffer", i);
        }
        const Tile tl = resolve_tile_id(&h, h.tile);
        BInst &I = plan.inst[i];
        I.Dup = (int)h.dim_up;
        I.Ddn = (int)h.dim_dn;
        I.W8u = h.w_up;
        I.W8d = h.w_dn;
        // one row per wave on 64- or 128-column stripes (two columns per lane
        // where the tile asks for wider stripes and the rows allow it)
        I.R = 1;
        I.V = (tl.up_wlog2 >= 7 && !(I.Ddn & 1) && I.W8u <= 32) ? 2 : 1;
        const int w = 64 * I.V;
        I.rc = std::max(tl.up_rc, kBatchUpRows);
        I.n_stripes = (I.Ddn + w - 1) / w;
        I.n_rc = (I.Dup + I.rc - 1) / I.rc;
        I.up_tiles = h.w_up ? 8 * I.n_rc * ((I.n_stripes + 7) / 8) : 0;
        const int by_lds = std::max(1, (int)(kBatchLds / (I.Ddn * 4)));
        const int by_fill = std::max(1, (2 * kBatchBlock + I.Ddn - 1) / I.Ddn);
        I.rpb = std::max(1, std::min(std::min(by_lds, by_fill), I.Dup));
        I.dn_tiles = (I.Dup + I.rpb - 1) / I.rpb;
        I.n = (int64_t)I.Dup * I.Ddn;
        I.upd_tiles = (int)((I.n + kUpdChunk - 1) / kUpdChunk);
        I.part_off = plan.part_doubles;
        I.part2_off = plan.part2_doubles;
        plan.part_doubles += (int64_t)I.dn_tiles * 5;
        plan.part2_doubles += I.upd_tiles;
        I.tab_up = (const ED_GLOBAL uint16_t *)h.tab_up;
        I.tab_dn = (const ED_GLOBAL uint16_t *)h.tab_dn;
        I.st_up = (const ED_GLOBAL uint64_t *)h.st_up;
        I.st_dn = (const ED_GLOBAL uint64_t *)h.st_dn;
        I.t = h.t;
        I.U = h.U;
        if (fill_ptrs) {
            const ed_batch_item &it = items[i];
            I.f1 = (const ED_GLOBAL float *)it.f1;
            for (int k = 0; k < 3; ++k) I.vec[k] = (ED_GLOBAL float *)it.vec[k];
            I.a = (ED_GLOBAL double *)it.a;
            I.b = (ED_GLOBAL double *)it.b;
        }
    }
    return ED_OK;
}

// per instance in the result staging area: a[0..max_steps), b[0..max_steps], E0 of the last step
__host__ __device__ inline int64_t stage_stride(int32_t max_steps) { return 2 * (int64_t)max_steps + 2; }

static int64_t batch_ws_bytes(const BatchPlan &plan, int n, int32_t max_steps) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    return al(sizeof(GridBar)) + al((int64_t)n * sizeof(BInst)) + al(8 * plan.part_doubles) +
           al(8 * plan.part2_doubles) + al(8 * (int64_t)n * (max_steps + 1)) +
           al(8 * (int64_t)n * stage_stride(max_steps));
}

// Gathers every instance's a_j, b_j and last E0 into one array, so that the
// host fetches them with one copy.  One workgroup per instance; j <= max_steps.
__global__ __launch_bounds__(256) void k_batch_collect(const BInst *__restrict__ inst, int max_steps,
                                                       double *__restrict__ stage) {
    const BInst &I = inst[blockIdx.x];
    const int k = I.j;
    double *o = stage + (int64_t)blockIdx.x * stage_stride(max_steps);
    for (int t = threadIdx.x; t < k; t += blockDim.x) o[t] = I.a[t];
    for (int t = threadIdx.x; t <= k; t += blockDim.x) o[max_steps + t] = I.b[t];
    if (threadIdx.x == 0) o[2 * max_steps + 1] = k > 0 ? I.e[k] : 0.0;
}

// Steps between the host's convergence checks when a batch runs one of its
// large instances on its own (ed_ground_energy).
constexpr int kSoloCheck = 9;

}  // namespace ed

namespace {

using namespace ed;

// Instances of at least solo_dim states (solo_dim > 0) run one by one.
bool solo_item(const ed_batch_item &it, int64_t solo_dim) {
    return solo_dim > 0 && it.h.dim_up * it.h.dim_dn >= solo_dim;
}

int64_t al256(int64_t b) { return (b + 255) & ~int64_t(255); }

// Workspace of the persistent launch over `items` (0 for none) and of the
// largest one-by-one run among `solo`.
int batch_parts_bytes(const std::vector<ed_batch_item> &items, const std::vector<ed_batch_item> &solo,
                      int32_t max_steps, int64_t *persist, int64_t *single) {
    *persist = 0;
    *single = 0;
    if (!items.empty()) {
        BatchPlan plan;
        const int rc = plan_batch(items.data(), (int)items.size(), max_steps, plan, false);
        if (rc) return rc;
        *persist = batch_ws_bytes(plan, (int)items.size(), max_steps);
    }
    for (const ed_batch_item &it : solo) {
        int64_t b = 0;
        const int rc = ed_workspace_size(&it.h, max_steps, &b);
        if (rc) return rc;
        *single = std::max(*single, b);
    }
    return ED_OK;
}

void split_items(const ed_batch_item *items, int32_t n, int64_t solo_dim, std::vector<ed_batch_item> &group,
                 std::vector<int> &gidx, std::vector<ed_batch_item> &solo, std::vector<int> &sidx) {
    for (int i = 0; i < n; ++i) {
        if (solo_item(items[i], solo_dim)) {
            solo.push_back(items[i]);
            sidx.push_back(i);
        } else {
            group.push_back(items[i]);
            gidx.push_back(i);
        }
    }
}

}  // namespace

namespace ed {

// The persistent cooperative launch over n items (the whole of a batch, or
// the part of it below solo_dim).
static int persistent_run(const ed_batch_item *items, int32_t n, int32_t max_steps, double tol, void *ws,
                          int64_t ws_bytes, void *stream, int32_t use_graph, double *e0, int32_t *steps,
                          int32_t *status, double *e0_device, int32_t *graph_used, double *phase_ms) {
    BatchPlan plan;
    int rc = plan_batch(items, n, max_steps, plan, true);
    if (rc) return rc;
    if (ws_bytes < batch_ws_bytes(plan, n, max_steps))
        return set_error(ED_ECAPACITY, "ed_ground_energy_batch: workspace too small");
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    char *p = static_cast<char *>(ws);
    GridBar *gb = reinterpret_cast<GridBar *>(p);
    p += al(sizeof(GridBar));
    BInst *dinst = reinterpret_cast<BInst *>(p);
    p += al((int64_t)n * sizeof(BInst));
    double *part = reinterpret_cast<double *>(p);
    p += al(8 * plan.part_doubles);
    double *part2 = reinterpret_cast<double *>(p);
    p += al(8 * plan.part2_doubles);
    double *ev = reinterpret_cast<double *>(p);
    for (int i = 0; i < n; ++i) plan.inst[i].e = (ED_GLOBAL double *)(ev + (int64_t)i * (max_steps + 1));
    p += al(8 * (int64_t)n * (max_steps + 1));
    double *stage = reinterpret_cast<double *>(p);

    // The kernel takes the instances largest first: every phase then ends on
    // the small instances' tiles.  order[k] is the item at position k.
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return plan.inst[x].n > plan.inst[y].n; });
    {
        std::vector<BInst> sorted(n);
        for (int k = 0; k < n; ++k) sorted[k] = plan.inst[order[k]];
        plan.inst.swap(sorted);
    }

    int grid = 0;
    rc = batch_grid(&grid);
    if (rc) return rc;

    hipStream_t user = static_cast<hipStream_t>(stream);
    GridBar gb0{};
    ED_HIP(hipMemcpyAsync(gb, &gb0, sizeof gb0, hipMemcpyHostToDevice, user));
    ED_HIP(hipMemcpyAsync(dinst, plan.inst.data(), n * sizeof(BInst), hipMemcpyHostToDevice, user));

    int ni = n, ms = max_steps;
    double tl = tol;
    void *args[] = {&dinst, &ni, &part, &part2, &gb, &ms, &tl};
    bool graphed = false;
    if (use_graph) {
        // one graph holding the single persistent cooperative launch
        hipStream_t cs = nullptr;
        hipEvent_t ev = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
                  hipEventRecord(ev, user) == hipSuccess && hipStreamWaitEvent(cs, ev, 0) == hipSuccess;
        if (ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const hipError_t le = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_batch), dim3(grid),
                                                             dim3(kBatchBlock), args, kBatchShm, cs);
            const hipError_t ee = hipStreamEndCapture(cs, &g);
            ok = le == hipSuccess && ee == hipSuccess && g != nullptr &&
                 hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
            if (ok) ok = hipGraphLaunch(ge, cs) == hipSuccess && hipEventRecord(ev, cs) == hipSuccess &&
                         hipStreamWaitEvent(user, ev, 0) == hipSuccess;
            graphed = ok;
        } else {
            ok = false;
        }
        (void)hipGetLastError();   // a refused capture leaves no sticky error
        // The graph's cooperative kernel may still be running: the executable
        // graph, the graph, the event and the capture stream are released only
        // after the capture stream (where the graph was launched) has drained.
        const hipError_t se = cs ? hipStreamSynchronize(cs) : hipSuccess;
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (ev) (void)hipEventDestroy(ev);
        if (cs) (void)hipStreamDestroy(cs);
        if (graphed) ED_HIP(se);
    }
    if (!graphed) {
        ED_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_batch), dim3(grid), dim3(kBatchBlock),
                                          args, kBatchShm, user));
    }
    if (graph_used) *graph_used = graphed ? 1 : 0;
    std::vector<BInst> out(n);
    GridBar gbh{};
    const int64_t sst = stage_stride(max_steps);
    std::vector<double> staged((size_t)n * sst);
    hipLaunchKernelGGL(k_batch_collect, dim3(n), dim3(256), 0, user, dinst, (int)max_steps, stage);
    ED_HIP(hipGetLastError());
    ED_HIP(hipMemcpyAsync(out.data(), dinst, n * sizeof(BInst), hipMemcpyDeviceToHost, user));
    ED_HIP(hipMemcpyAsync(&gbh, gb, sizeof gbh, hipMemcpyDeviceToHost, user));
    ED_HIP(hipMemcpyAsync(staged.data(), stage, 8 * staged.size(), hipMemcpyDeviceToHost, user));
    ED_HIP(hipStreamSynchronize(user));
    if (gbh.err) return set_error(ED_EDEVICE, "ed_ground_energy_batch: grid barrier timed out");
    if (phase_ms) {
        int dev = 0, khz = 0;
        ED_HIP(hipGetDevice(&dev));
        ED_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        for (int k = 0; k < 6; ++k) phase_ms[k] = khz > 0 ? (double)gbh.phase[k] / (double)khz : -1.0;
    }
    int result = ED_OK;
    for (int pos = 0; pos < n; ++pos) {
        const int i = order[pos];
        const BInst &I = out[pos];
        if (I.status == kBadStart) return set_error(ED_EINVAL, "ed_ground_energy_batch: item %d has a zero start", i);
        const int k = I.j;
        steps[i] = k;
        status[i] = I.status == kConverged ? ED_OK : (I.status == ED_BREAKDOWN ? ED_BREAKDOWN : ED_NOT_CONVERGED);
        if (status[i] == ED_NOT_CONVERGED) result = ED_NOT_CONVERGED;
        const double *a = staged.data() + (size_t)pos * sst, *b = a + max_steps;
        e0[i] = k > 0 ? tridiag_lowest(a, b + 1, k) : NAN;
        if (e0_device) e0_device[i] = k > 0 ? a[2 * max_steps + 1] : NAN;
    }
    return result;
}

}  // namespace ed

extern "C" {

int ed_batch_workspace_size(const ed_batch_item *items, int32_t n, int32_t max_steps, int64_t solo_dim,
                            int64_t *bytes) {
    using namespace ed;
    clear_error();
    if (!items || n < 1 || max_steps < 1 || !bytes) return set_error(ED_EINVAL, "ed_batch_workspace_size: bad arguments");
    BatchPlan all;
    int rc = plan_batch(items, n, max_steps, all, false);   // every item meets the batch's limits
    if (rc) return rc;
    std::vector<ed_batch_item> group, solo;
    std::vector<int> gidx, sidx;
    split_items(items, n, solo_dim, group, gidx, solo, sidx);
    int64_t persist = 0, single = 0;
    rc = batch_parts_bytes(group, solo, max_steps, &persist, &single);
    if (rc) return rc;
    *bytes = al256(persist) + single;
    return ED_OK;
}

int ed_ground_energy_batch(const ed_batch_item *items, int32_t n, int32_t max_steps, double tol, int64_t solo_dim,
                           void *ws, int64_t ws_bytes, void *stream, int32_t use_graph, double *e0, int32_t *steps,
                           int32_t *status, double *e0_device, int32_t *graph_used, double *phase_ms) {
    using namespace ed;
    clear_error();
    if (!items || n < 1 || max_steps < 1 || !ws || !e0 || !steps || !status || !(tol > 0))
        return set_error(ED_EINVAL, "ed_ground_energy_batch: bad arguments");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return set_error(ED_EINVAL, "ed_ground_energy_batch: ws not aligned");
    BatchPlan all;
    int rc = plan_batch(items, n, max_steps, all, true);   // limits and buffers of every item
    if (rc) return rc;
    std::vector<ed_batch_item> group, solo;
    std::vector<int> gidx, sidx;
    split_items(items, n, solo_dim, group, gidx, solo, sidx);
    int64_t persist = 0, single = 0;
    rc = batch_parts_bytes(group, solo, max_steps, &persist, &single);
    if (rc) return rc;
    if (ws_bytes < al256(persist) + single) return set_error(ED_ECAPACITY, "ed_ground_energy_batch: workspace too small");
    if (graph_used) *graph_used = 0;
    if (phase_ms)
        for (int k = 0; k < 6; ++k) phase_ms[k] = 0.0;
    int result = ED_OK;
    if (!group.empty()) {
        const int ng = (int)group.size();
        std::vector<double> ge0(ng), ged(ng);
        std::vector<int32_t> gst(ng), gss(ng);
        rc = persistent_run(group.data(), ng, max_steps, tol, ws, al256(persist), stream, use_graph, ge0.data(),
                            gst.data(), gss.data(), ged.data(), graph_used, phase_ms);
        if (rc != ED_OK && rc != ED_NOT_CONVERGED) return rc;
        result = rc;
        for (int k = 0; k < ng; ++k) {
            const int i = gidx[k];
            e0[i] = ge0[k];
            steps[i] = gst[k];
            status[i] = gss[k];
            if (e0_device) e0_device[i] = ged[k];
        }
    }
    // the large instances, one after another on the same stream, through the
    // one-instance run (the same stopping rule, checked every kSoloCheck steps)
    void *ws_single = static_cast<char *>(ws) + al256(persist);
    for (size_t k = 0; k < solo.size(); ++k) {
        const ed_batch_item &it = solo[k];
        const int i = sidx[k];
        ed_lanczos st{};
        st.f_prev = it.vec[0];
        st.f_cur = it.vec[1];
        st.f_next = it.vec[2];
        st.a = it.a;
        st.b = it.b;
        st.j = 0;
        st.max_steps = max_steps;
        double e = NAN;
        int32_t j = 0;
        rc = ed_ground_energy(&it.h, &st, it.f1, tol, kSoloCheck, ws_single, stream, &e, &j, nullptr, nullptr);
        if (rc != ED_OK && rc != ED_BREAKDOWN && rc != ED_NOT_CONVERGED) return rc;
        e0[i] = e;
        steps[i] = j;
        status[i] = rc;
        if (e0_device) e0_device[i] = e;
        if (rc == ED_NOT_CONVERGED) result = ED_NOT_CONVERGED;
    }
    return result;
}

}  // extern "C"
