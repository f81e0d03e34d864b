// Diagonal observables of a state vector in the occupation basis (Sec. 2.1: a
// basis state fixes every occupation number n_i,sigma).  Everything follows
// from the occupation moments
//     G[a][b] = sum_x |psi_x|^2 n_a(x) n_b(x) / sum_x |psi_x|^2
// over the 2*N_s occupation numbers a = i (up) and a = N_s + i (down).  With
// x = (r, c), r the up state and c the down state, the three blocks need only
//     up-up:     rowsum[r]  = sum_c |psi[r,c]|^2
//     up-down:   T[r][j]    = sum_c |psi[r,c]|^2 n_j,dn(c)
//     down-down: colsum[c]  = sum_r |psi[r,c]|^2
// which two passes over psi produce (k_obs_rows, k_obs_cols with k_obs_colsum);
// k_obs_final contracts them with the per-spin occupation bits.  All sums are float64 in
// a fixed order: the result does not depend on the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/ed.h"
#include "ed_common.h"
#include "ed_internal.h"
#include "ed_launch.h"

namespace ed {

constexpr int kObsMaxSites = 32;   // G is at most 64 x 64
constexpr int kObsRowChunk = 256;  // rows per column-sum partial

// one workgroup per up state r: rowsum[r] and T[r][0..ns)
template <typename T>
__global__ __launch_bounds__(256) void k_obs_rows(const T *__restrict__ psi, const uint64_t *__restrict__ st_dn,
                                                  int Ddn, int ns, double *__restrict__ rowsum,
                                                  double *__restrict__ trow) {
    const int r = blockIdx.x;
    const T *row = psi + (int64_t)r * Ddn;
    double v[kObsMaxSites + 1];
#pragma unroll
    for (int j = 0; j <= kObsMaxSites; ++j) v[j] = 0.0;
    for (int c = threadIdx.x; c < Ddn; c += blockDim.x) {
        const double a = (double)row[c];
        const double w = a * a;
        const uint64_t bits = st_dn[c];
        v[kObsMaxSites] += w;
#pragma unroll
        for (int j = 0; j < kObsMaxSites; ++j) v[j] += ((bits >> j) & 1ull) ? w : 0.0;
    }
    double tot[kObsMaxSites + 1];
    block_sum<kObsMaxSites + 1>(v, tot);
    if (threadIdx.x == 0) {
        rowsum[r] = tot[kObsMaxSites];
        for (int j = 0; j < ns; ++j) trow[(int64_t)r * ns + j] = tot[j];
    }
}

// column sums over chunks of kObsRowChunk rows: colpart[chunk][c]
template <typename T>
__global__ __launch_bounds__(256) void k_obs_cols(const T *__restrict__ psi, int Dup, int Ddn,
                                                  double *__restrict__ colpart) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (c >= Ddn) return;
    const int r0 = chunk * kObsRowChunk, r1 = min(Dup, r0 + kObsRowChunk);
    double s0 = 0.0, s1 = 0.0;
    int r = r0;
    for (; r + 1 < r1; r += 2) {   // two independent loads in flight
        const double a = (double)psi[(int64_t)r * Ddn + c], b = (double)psi[(int64_t)(r + 1) * Ddn + c];
        s0 += a * a;
        s1 += b * b;
    }
    if (r < r1) {
        const double a = (double)psi[(int64_t)r * Ddn + c];
        s0 += a * a;
    }
    colpart[(int64_t)chunk * Ddn + c] = s0 + s1;
}

// colsum[c] = sum over chunks of colpart[chunk][c], in chunk order, into colpart[0][c]
__global__ __launch_bounds__(256) void k_obs_colsum(double *__restrict__ colpart, int nchunk, int Ddn) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Ddn) return;
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += colpart[(int64_t)k * Ddn + c];
    colpart[c] = s;
}

// one workgroup per entry e = (a, b) of G: its sum and the norm sum_x |psi_x|^2,
// each over the rows (or columns) strided by thread and then in the fixed
// order of block_sum
__global__ __launch_bounds__(256) void k_obs_final(const double *__restrict__ rowsum,
                                                   const double *__restrict__ trow,
                                                   const double *__restrict__ colsum,
                                                   const uint64_t *__restrict__ st_up,
                                                   const uint64_t *__restrict__ st_dn, int Dup, int Ddn, int ns,
                                                   double *__restrict__ g) {
    const int n2 = 2 * ns;
    const int e = blockIdx.x, a = e / n2, b = e - a * n2;
    double p[2] = {0.0, 0.0};   // norm, entry
    for (int r = threadIdx.x; r < Dup; r += blockDim.x) p[0] += rowsum[r];
    if (a < ns && b < ns) {          // up-up: sum_r rowsum[r] n_a n_b
        const uint64_t m = (1ull << a) | (1ull << b);
        for (int r = threadIdx.x; r < Dup; r += blockDim.x)
            if ((st_up[r] & m) == m) p[1] += rowsum[r];
    } else if (a < ns) {             // up-down
        const int j = b - ns;
        for (int r = threadIdx.x; r < Dup; r += blockDim.x)
            if ((st_up[r] >> a) & 1ull) p[1] += trow[(int64_t)r * ns + j];
    } else if (b < ns) {             // down-up: the transpose
        const int j = a - ns;
        for (int r = threadIdx.x; r < Dup; r += blockDim.x)
            if ((st_up[r] >> b) & 1ull) p[1] += trow[(int64_t)r * ns + j];
    } else {                         // down-down: sum_c colsum[c] n_a n_b
        const uint64_t m = (1ull << (a - ns)) | (1ull << (b - ns));
        for (int c = threadIdx.x; c < Ddn; c += blockDim.x)
            if ((st_dn[c] & m) == m) p[1] += colsum[c];
    }
    double tot[2];
    block_sum<2>(p, tot);
    if (threadIdx.x == 0) g[e] = tot[0] > 0.0 ? tot[1] / tot[0] : 0.0;
}

// ---------------------------------------------------------------------------
// Spin-flip moments C[i][j] = <S+_i S-_j> / <psi|psi> with S+_i = c+_i,up c_i,dn
// and S-_j = c+_j,dn c_j,up.  For i != j the operator moves an up particle
// j -> i and a down particle i -> j: reordered, it is -(c+_i,up c_j,up)
// (c+_j,dn c_i,dn), each factor a same-species hop with the sign of the
// occupied sites strictly between i and j (the rule of the hopping tables).
// On the diagonal it is n_i,up (1 - n_i,dn).  One launch per i; a workgroup
// takes one up state r, whose up hop is uniform (its target row and sign are
// computed once into LDS); each lane takes down states and applies the down
// hop, finding the target's rank from a binomial table.  Sums are fixed-order
// block reductions: the result does not depend on the launch.
constexpr int kFlipSlots = kObsMaxSites + 1;   // the ns values of row i of C, then |psi|^2

__device__ __forceinline__ int64_t colex_rank_lds(uint64_t s, const int64_t (*binom)[kObsMaxSites + 1]) {
    int64_t r = 0;
    int k = 0;
    while (s) {
        const int p = __ffsll((unsigned long long)s) - 1;
        r += binom[p][k + 1];
        ++k;
        s &= s - 1;
    }
    return r;
}

__device__ __forceinline__ uint64_t between_mask(int i, int j) {
    const int lo = min(i, j), hi = max(i, j);
    return ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
}

// The down half of the flip for site i: tgt[j * Ddn + c] = (rank << 1) | sign
// of the state c with the down particle moved i -> j (the sign of the occupied
// sites strictly between), or all ones where column c has no particle at i or
// one at j.  It depends on (c, j) only, so every row of psi shares it.
constexpr uint32_t kNoFlip = 0xFFFFFFFFu;

__global__ __launch_bounds__(256) void k_sflip_targets(const uint64_t *__restrict__ st_dn, int Ddn, int ns, int i,
                                                       uint32_t *__restrict__ tgt) {
    __shared__ int64_t binom[kObsMaxSites][kObsMaxSites + 1];   // C(n, k), n < 32
    for (int e = threadIdx.x; e < kObsMaxSites * (kObsMaxSites + 1); e += blockDim.x) {
        const int n = e / (kObsMaxSites + 1), k = e - n * (kObsMaxSites + 1);
        int64_t c = k > n ? 0 : 1;
        for (int m = 1; m <= k && k <= n; ++m) c = c * (n - k + m) / m;   // exact at every step
        binom[n][k] = c;
    }
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Ddn) return;
    const uint64_t sd = st_dn[c], bi = 1ull << i;
    for (int j = 0; j < ns; ++j) {
        uint32_t e = kNoFlip;
        if ((sd & bi) && !((sd >> j) & 1ull)) {
            const int64_t c2 = colex_rank_lds(sd ^ bi ^ (1ull << j), binom);
            e = ((uint32_t)c2 << 1) | (uint32_t)(__popcll(sd & between_mask(i, j)) & 1);
        }
        tgt[(int64_t)j * Ddn + c] = e;
    }
}

// NSM: a compile-time bound on the sites (16 or 32), so a 16-site lattice
// keeps half the accumulators and loop trips
template <typename T, int NSM>
__global__ __launch_bounds__(256) void k_sflip(const T *__restrict__ psi, const uint64_t *__restrict__ st_up,
                                               const uint64_t *__restrict__ st_dn, int Ddn, int ns, int i,
                                               const uint32_t *__restrict__ tgt, double *__restrict__ part) {
    __shared__ int64_t binom[kObsMaxSites][kObsMaxSites + 1];   // C(n, k), n < 32
    __shared__ int64_t row2[kObsMaxSites];                      // target up row of the hop j -> i, or -1
    __shared__ double sgn_up[kObsMaxSites];
    for (int e = threadIdx.x; e < kObsMaxSites * (kObsMaxSites + 1); e += blockDim.x) {
        const int n = e / (kObsMaxSites + 1), k = e - n * (kObsMaxSites + 1);
        int64_t c = k > n ? 0 : 1;
        for (int m = 1; m <= k && k <= n; ++m) c = c * (n - k + m) / m;   // exact at every step
        binom[n][k] = c;
    }
    __syncthreads();
    const int r = blockIdx.x;
    const uint64_t su = st_up[r];
    const uint64_t bi = 1ull << i;
    if (threadIdx.x < kObsMaxSites) {
        const int j = threadIdx.x;
        const bool ok = j < ns && !(su & bi) && ((su >> j) & 1ull);
        row2[j] = ok ? colex_rank_lds(su ^ bi ^ (1ull << j), binom) : -1;
        sgn_up[j] = (__popcll(su & between_mask(i, j)) & 1) ? -1.0 : 1.0;
    }
    __syncthreads();
    double acc[NSM + 1];   // row i of C for j < NSM, then |psi|^2
#pragma unroll
    for (int j = 0; j <= NSM; ++j) acc[j] = 0.0;
    const T *row = psi + (int64_t)r * Ddn;
    const bool up_hole = !(su & bi);
    for (int c = threadIdx.x; c < Ddn; c += blockDim.x) {
        const double x = (double)row[c];
        const uint64_t sd = st_dn[c];
        acc[NSM] += x * x;
        if (up_hole) {
            if (sd & bi) {
#pragma unroll
                for (int j = 0; j < NSM; ++j) {
                    if (row2[j] >= 0) {
                        const uint32_t e = tgt[(int64_t)j * Ddn + c];
                        if (e != kNoFlip) {
                            const int64_t c2 = (int64_t)(e >> 1);
                            const double sd_sign = (e & 1u) ? -1.0 : 1.0;
                            acc[j] -= sgn_up[j] * sd_sign * x * (double)psi[row2[j] * Ddn + c2];
                        }
                    }
                }
            }
        } else if (!(sd & bi)) {   // diagonal: n_i,up (1 - n_i,dn)
#pragma unroll
            for (int j = 0; j < NSM; ++j)
                if (j == i) acc[j] += x * x;
        }
    }
    double tot[NSM + 1];
    block_sum<NSM + 1>(acc, tot);
    if (threadIdx.x == 0) {
        for (int j = 0; j < NSM; ++j) part[(int64_t)r * kFlipSlots + j] = tot[j];
        part[(int64_t)r * kFlipSlots + kObsMaxSites] = tot[NSM];
    }
}

// row i of C: sums over the up rows in a fixed order (thread t adds the rows
// of its contiguous chunk, then the threads' sums are added in thread order),
// normalised by the same sum of |psi|^2
constexpr int kFinalThreads = 512;

__global__ __launch_bounds__(kFinalThreads) void k_sflip_final(const double *__restrict__ part, int Dup, int ns,
                                                               int i, double *__restrict__ c) {
    __shared__ double red[kFinalThreads];
    __shared__ double s_tot[kObsMaxSites + 1];
    const int t = threadIdx.x;
    const int chunk = (Dup + kFinalThreads - 1) / kFinalThreads;
    const int lo = min(Dup, t * chunk), hi = min(Dup, lo + chunk);
    for (int j = 0; j <= ns; ++j) {
        const int slot = j < ns ? j : kObsMaxSites;   // the last pass: |psi|^2
        double s = 0.0;
        for (int r = lo; r < hi; ++r) s += part[(int64_t)r * kFlipSlots + slot];
        red[t] = s;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int k = 0; k < kFinalThreads; ++k) tot += red[k];
            s_tot[j] = tot;
        }
        __syncthreads();
    }
    if (t < ns) c[i * ns + t] = s_tot[ns] > 0.0 ? s_tot[t] / s_tot[ns] : 0.0;
}

static int64_t flip_ws_bytes(const ed_ham *h) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    return al(8 * kFlipSlots * h->dim_up) + al(8 * kObsMaxSites * kObsMaxSites) + al(4 * kObsMaxSites * h->dim_dn);
}

template <typename T>
static int flip_impl(const ed_ham *h, int ns, const T *psi, char *ws, hipStream_t s, double *c_host) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    double *part = reinterpret_cast<double *>(ws);
    double *c = reinterpret_cast<double *>(ws + al(8 * kFlipSlots * h->dim_up));
    uint32_t *tgt = reinterpret_cast<uint32_t *>(ws + al(8 * kFlipSlots * h->dim_up) + al(8 * kObsMaxSites * kObsMaxSites));
    const int Ddn = (int)h->dim_dn;
    for (int i = 0; i < ns; ++i) {
        hipLaunchKernelGGL(k_sflip_targets, dim3((unsigned)((Ddn + 255) / 256)), dim3(256), 0, s, h->st_dn, Ddn, ns, i,
                           tgt);
        ED_LAUNCHED("k_sflip_targets");
        if (ns <= 16)
            hipLaunchKernelGGL((k_sflip<T, 16>), dim3((unsigned)h->dim_up), dim3(256), 0, s, psi, h->st_up, h->st_dn,
                               Ddn, ns, i, (const uint32_t *)tgt, part);
        else
            hipLaunchKernelGGL((k_sflip<T, kObsMaxSites>), dim3((unsigned)h->dim_up), dim3(256), 0, s, psi, h->st_up,
                               h->st_dn, Ddn, ns, i, (const uint32_t *)tgt, part);
        ED_LAUNCHED("k_sflip");
        hipLaunchKernelGGL(k_sflip_final, dim3(1), dim3(kFinalThreads), 0, s, part, (int)h->dim_up, ns, i, c);
        ED_LAUNCHED("k_sflip_final");
    }
    ED_HIP(hipMemcpyAsync(c_host, c, sizeof(double) * ns * ns, hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    return ED_OK;
}

// ---------------------------------------------------------------------------
// Bond moments K[b][sigma] = <c+_i c_j + c+_j c_i>_sigma / <psi|psi> for bonds
// b = (i, j).  An up hop over b is uniform along a row (target row and sign
// computed once into LDS), so its part is a dot product of two rows; a down
// hop is per lane, the target found by its colex rank.  kBondGroup bonds per
// launch; sums in a fixed order.
constexpr int kBondGroup = 16;
constexpr int kBondSlots = 2 * kBondGroup + 1;   // up and down per bond, then |psi|^2

template <typename T>
__global__ __launch_bounds__(256) void k_bond(const T *__restrict__ psi, const uint64_t *__restrict__ st_up,
                                              const uint64_t *__restrict__ st_dn, int Ddn,
                                              const int32_t *__restrict__ bonds, int nb,
                                              double *__restrict__ part) {
    __shared__ int64_t binom[kObsMaxSites][kObsMaxSites + 1];
    __shared__ int64_t row2[kBondGroup];
    __shared__ double sgn_up[kBondGroup];
    __shared__ uint64_t bmask[kBondGroup], bbetween[kBondGroup];
    for (int e = threadIdx.x; e < kObsMaxSites * (kObsMaxSites + 1); e += blockDim.x) {
        const int n = e / (kObsMaxSites + 1), k = e - n * (kObsMaxSites + 1);
        int64_t c = k > n ? 0 : 1;
        for (int m = 1; m <= k && k <= n; ++m) c = c * (n - k + m) / m;
        binom[n][k] = c;
    }
    const int r = blockIdx.x;
    const uint64_t su = st_up[r];
    if (threadIdx.x < kBondGroup) {
        const int b = threadIdx.x;
        uint64_t m = 0, btw = 0;
        if (b < nb) {
            const int i = bonds[2 * b], j = bonds[2 * b + 1];
            m = (1ull << i) | (1ull << j);
            btw = between_mask(i, j);
        }
        bmask[b] = m;
        bbetween[b] = btw;
    }
    __syncthreads();
    if (threadIdx.x < kBondGroup) {
        const int b = threadIdx.x;
        const uint64_t m = bmask[b], o = su & m;
        const bool hop = m && o && o != m;
        row2[b] = hop ? colex_rank_lds(su ^ m, binom) : -1;
        sgn_up[b] = (__popcll(su & bbetween[b]) & 1) ? -1.0 : 1.0;
    }
    __syncthreads();
    double acc[kBondSlots];
#pragma unroll
    for (int k = 0; k < kBondSlots; ++k) acc[k] = 0.0;
    const T *row = psi + (int64_t)r * Ddn;
    for (int c = threadIdx.x; c < Ddn; c += blockDim.x) {
        const double x = (double)row[c];
        const uint64_t sd = st_dn[c];
        acc[2 * kBondGroup] += x * x;
#pragma unroll
        for (int b = 0; b < kBondGroup; ++b) {
            if (row2[b] >= 0) acc[2 * b] += sgn_up[b] * x * (double)psi[row2[b] * Ddn + c];
            const uint64_t m = bmask[b], o = sd & m;
            if (m && o && o != m) {
                const int64_t c2 = colex_rank_lds(sd ^ m, binom);
                const double sg = (__popcll(sd & bbetween[b]) & 1) ? -1.0 : 1.0;
                acc[2 * b + 1] += sg * x * (double)row[c2];
            }
        }
    }
    double tot[kBondSlots];
    block_sum<kBondSlots>(acc, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < kBondSlots; ++k) part[(int64_t)r * kBondSlots + k] = tot[k];
}

// the group's 2 nb values, summed over the up rows in the fixed order of
// k_sflip_final and normalised by |psi|^2
__global__ __launch_bounds__(kFinalThreads) void k_bond_final(const double *__restrict__ part, int Dup, int nb,
                                                              int b0, double *__restrict__ kout) {
    __shared__ double red[kFinalThreads];
    __shared__ double s_tot[kBondSlots];
    const int t = threadIdx.x;
    const int chunk = (Dup + kFinalThreads - 1) / kFinalThreads;
    const int lo = min(Dup, t * chunk), hi = min(Dup, lo + chunk);
    for (int k = 0; k <= 2 * nb; ++k) {
        const int slot = k < 2 * nb ? k : 2 * kBondGroup;   // the last pass: |psi|^2
        double s = 0.0;
        for (int r = lo; r < hi; ++r) s += part[(int64_t)r * kBondSlots + slot];
        red[t] = s;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int q = 0; q < kFinalThreads; ++q) tot += red[q];
            s_tot[k] = tot;
        }
        __syncthreads();
    }
    if (t < 2 * nb) kout[2 * b0 + t] = s_tot[2 * nb] > 0.0 ? s_tot[t] / s_tot[2 * nb] : 0.0;
}

static int64_t bond_ws_bytes(const ed_ham *h, int n_bonds) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    return al(8 * kBondSlots * h->dim_up) + al(8 * 2 * (int64_t)n_bonds) + al(8 * (int64_t)n_bonds);
}

template <typename T>
static int bond_impl(const ed_ham *h, const int32_t *bonds_host, int n_bonds, const T *psi, char *ws, hipStream_t s,
                     double *k_host) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    double *part = reinterpret_cast<double *>(ws);
    double *kout = reinterpret_cast<double *>(ws + al(8 * kBondSlots * h->dim_up));
    int32_t *bonds = reinterpret_cast<int32_t *>(ws + al(8 * kBondSlots * h->dim_up) + al(8 * 2 * (int64_t)n_bonds));
    ED_HIP(hipMemcpyAsync(bonds, bonds_host, sizeof(int32_t) * 2 * n_bonds, hipMemcpyHostToDevice, s));
    for (int b0 = 0; b0 < n_bonds; b0 += kBondGroup) {
        const int nb = std::min(kBondGroup, n_bonds - b0);
        hipLaunchKernelGGL(k_bond<T>, dim3((unsigned)h->dim_up), dim3(256), 0, s, psi, h->st_up, h->st_dn,
                           (int)h->dim_dn, bonds + 2 * b0, nb, part);
        ED_LAUNCHED("k_bond");
        hipLaunchKernelGGL(k_bond_final, dim3(1), dim3(kFinalThreads), 0, s, part, (int)h->dim_up, nb, b0, kout);
        ED_LAUNCHED("k_bond_final");
    }
    ED_HIP(hipMemcpyAsync(k_host, kout, sizeof(double) * 2 * n_bonds, hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    return ED_OK;
}

static int64_t obs_ws_bytes(const ed_ham *h, int ns) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t nchunk = (h->dim_up + kObsRowChunk - 1) / kObsRowChunk;
    return al(8 * h->dim_up) + al(8 * h->dim_up * ns) + al(8 * nchunk * h->dim_dn) + al(8 * 4 * ns * ns);
}

static int obs_check(const ed_ham *h, int ns, const char *who) {
    int rc = check_real(h, who);
    if (rc) return rc;
    if (ns < 1 || ns > kObsMaxSites) return set_error(ED_EINVAL, "%s: n_sites %d outside 1..%d", who, ns, kObsMaxSites);
    return ED_OK;
}

// the calls that find a target state by its colex rank: both bases ascending
static int ranked_check(const ed_ham *h, int ns, const char *who) {
    int rc = obs_check(h, ns, who);
    if (rc) return rc;
    if (h->order) return set_error(ED_EINVAL, "%s: needs both species in ascending basis order (order = 0)", who);
    return ED_OK;
}

template <typename T>
static int obs_impl(const ed_ham *h, int ns, const T *psi, char *ws, hipStream_t s, double *g_host) {
    auto al = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int Dup = (int)h->dim_up, Ddn = (int)h->dim_dn;
    const int nchunk = (Dup + kObsRowChunk - 1) / kObsRowChunk;
    double *rowsum = reinterpret_cast<double *>(ws);
    double *trow = reinterpret_cast<double *>(ws + al(8LL * Dup));
    double *colpart = reinterpret_cast<double *>(ws + al(8LL * Dup) + al(8LL * Dup * ns));
    double *g = reinterpret_cast<double *>(ws + al(8LL * Dup) + al(8LL * Dup * ns) + al(8LL * nchunk * Ddn));
    hipLaunchKernelGGL(k_obs_rows<T>, dim3(Dup), dim3(256), 0, s, psi, h->st_dn, Ddn, ns, rowsum, trow);
    ED_LAUNCHED("k_obs_rows");
    hipLaunchKernelGGL(k_obs_cols<T>, dim3((Ddn + 255) / 256, nchunk), dim3(256), 0, s, psi, Dup, Ddn, colpart);
    ED_LAUNCHED("k_obs_cols");
    hipLaunchKernelGGL(k_obs_colsum, dim3((Ddn + 255) / 256), dim3(256), 0, s, colpart, nchunk, Ddn);
    ED_LAUNCHED("k_obs_colsum");
    hipLaunchKernelGGL(k_obs_final, dim3(4 * ns * ns), dim3(256), 0, s, rowsum, trow, colpart, h->st_up, h->st_dn, Dup, Ddn,
                       ns, g);
    ED_LAUNCHED("k_obs_final");
    ED_HIP(hipMemcpyAsync(g_host, g, sizeof(double) * 4 * ns * ns, hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    return ED_OK;
}

}  // namespace ed

using namespace ed;

extern "C" {

int ed_occupation_moments_ws(const ed_ham *h, int32_t n_sites, int64_t *bytes) {
    clear_error();
    int rc = obs_check(h, n_sites, "ed_occupation_moments_ws");
    if (rc) return rc;
    if (!bytes) return set_error(ED_EINVAL, "ed_occupation_moments_ws: bytes is NULL");
    *bytes = obs_ws_bytes(h, n_sites);
    return ED_OK;
}

int ed_occupation_moments(const ed_ham *h, int32_t n_sites, const void *psi, void *ws, int64_t ws_bytes,
                          void *stream, double *g) {
    clear_error();
    int rc = obs_check(h, n_sites, "ed_occupation_moments");
    if (rc) return rc;
    if (!psi || !ws || !g) return set_error(ED_EINVAL, "ed_occupation_moments: NULL buffer");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return set_error(ED_EINVAL, "ed_occupation_moments: ws not aligned");
    if (ws_bytes < obs_ws_bytes(h, n_sites))
        return set_error(ED_ECAPACITY, "ed_occupation_moments: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->dtype == ED_F64)
        return obs_impl<double>(h, n_sites, static_cast<const double *>(psi), static_cast<char *>(ws), s, g);
    return obs_impl<float>(h, n_sites, static_cast<const float *>(psi), static_cast<char *>(ws), s, g);
}

int ed_spin_flip_moments_ws(const ed_ham *h, int32_t n_sites, int64_t *bytes) {
    clear_error();
    int rc = ranked_check(h, n_sites, "ed_spin_flip_moments_ws");
    if (rc) return rc;
    if (!bytes) return set_error(ED_EINVAL, "ed_spin_flip_moments_ws: bytes is NULL");
    *bytes = flip_ws_bytes(h);
    return ED_OK;
}

int ed_spin_flip_moments(const ed_ham *h, int32_t n_sites, const void *psi, void *ws, int64_t ws_bytes,
                         void *stream, double *c) {
    clear_error();
    int rc = ranked_check(h, n_sites, "ed_spin_flip_moments");
    if (rc) return rc;
    if (!psi || !ws || !c) return set_error(ED_EINVAL, "ed_spin_flip_moments: NULL buffer");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return set_error(ED_EINVAL, "ed_spin_flip_moments: ws not aligned");
    if (ws_bytes < flip_ws_bytes(h)) return set_error(ED_ECAPACITY, "ed_spin_flip_moments: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->dtype == ED_F64)
        return flip_impl<double>(h, n_sites, static_cast<const double *>(psi), static_cast<char *>(ws), s, c);
    return flip_impl<float>(h, n_sites, static_cast<const float *>(psi), static_cast<char *>(ws), s, c);
}

int ed_bond_moments_ws(const ed_ham *h, int32_t n_sites, int32_t n_bonds, int64_t *bytes) {
    clear_error();
    int rc = ranked_check(h, n_sites, "ed_bond_moments_ws");
    if (rc) return rc;
    if (!bytes || n_bonds < 1) return set_error(ED_EINVAL, "ed_bond_moments_ws: bad arguments");
    *bytes = bond_ws_bytes(h, n_bonds);
    return ED_OK;
}

int ed_bond_moments(const ed_ham *h, int32_t n_sites, const int32_t *bonds, int32_t n_bonds, const void *psi,
                    void *ws, int64_t ws_bytes, void *stream, double *k) {
    clear_error();
    int rc = ranked_check(h, n_sites, "ed_bond_moments");
    if (rc) return rc;
    if (!bonds || n_bonds < 1 || !psi || !ws || !k) return set_error(ED_EINVAL, "ed_bond_moments: bad arguments");
    for (int b = 0; b < n_bonds; ++b) {
        const int i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || j < 0 || i >= n_sites || j >= n_sites || i == j)
            return set_error(ED_EINVAL, "ed_bond_moments: bond %d = (%d, %d) invalid", b, i, j);
    }
    if (reinterpret_cast<uintptr_t>(ws) & 255) return set_error(ED_EINVAL, "ed_bond_moments: ws not aligned");
    if (ws_bytes < bond_ws_bytes(h, n_bonds)) return set_error(ED_ECAPACITY, "ed_bond_moments: workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->dtype == ED_F64)
        return bond_impl<double>(h, bonds, n_bonds, static_cast<const double *>(psi), static_cast<char *>(ws), s, k);
    return bond_impl<float>(h, bonds, n_bonds, static_cast<const float *>(psi), static_cast<char *>(ws), s, k);
}

}  // extern "C"
