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
#include "ed_common.cuh"
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

// one workgroup: the (2 ns)^2 entries of G, normalised by sum_x |psi_x|^2
__global__ __launch_bounds__(1024) void k_obs_final(const double *__restrict__ rowsum,
                                                    const double *__restrict__ trow,
                                                    const double *__restrict__ colsum,
                                                    const uint64_t *__restrict__ st_up,
                                                    const uint64_t *__restrict__ st_dn, int Dup, int Ddn, int ns,
                                                    double *__restrict__ g) {
    __shared__ double s_norm;
    double p[1] = {0.0};
    for (int r = threadIdx.x; r < Dup; r += blockDim.x) p[0] += rowsum[r];
    double tot[1];
    block_sum<1>(p, tot);
    if (threadIdx.x == 0) s_norm = tot[0];
    __syncthreads();
    const double inv = s_norm > 0.0 ? 1.0 / s_norm : 0.0;
    const int n2 = 2 * ns;
    for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) {
        const int a = e / n2, b = e - a * n2;
        double s = 0.0;
        if (a < ns && b < ns) {          // up-up: sum_r rowsum[r] n_a n_b
            const uint64_t m = (1ull << a) | (1ull << b);
            for (int r = 0; r < Dup; ++r)
                if ((st_up[r] & m) == m) s += rowsum[r];
        } else if (a < ns) {             // up-down
            const int j = b - ns;
            for (int r = 0; r < Dup; ++r)
                if ((st_up[r] >> a) & 1ull) s += trow[(int64_t)r * ns + j];
        } else if (b < ns) {             // down-up: the transpose
            const int j = a - ns;
            for (int r = 0; r < Dup; ++r)
                if ((st_up[r] >> b) & 1ull) s += trow[(int64_t)r * ns + j];
        } else {                         // down-down: sum_c colsum[c] n_a n_b
            const uint64_t m = (1ull << (a - ns)) | (1ull << (b - ns));
            for (int c = 0; c < Ddn; ++c)
                if ((st_dn[c] & m) == m) s += colsum[c];
        }
        g[e] = s * inv;
    }
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
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(1024), 0, s, rowsum, trow, colpart, h->st_up, h->st_dn, Dup, Ddn,
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

}  // extern "C"
