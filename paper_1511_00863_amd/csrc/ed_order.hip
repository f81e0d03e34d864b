// Vectors between basis orders.  A species' basis may be reordered
// (ed_permute_basis); H then acts on the correspondingly permuted vector
// elements, and this gather moves a vector from one order to another:
// y[p, q] = x[perm_up[p], perm_dn[q]] over the (up, down) element grid of
// Eq. 3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/ed.h"
#include "ed_internal.h"
#include "ed_launch.h"

namespace ed {

constexpr int kPermBlock = 256;
constexpr int64_t kPermMaxGrid = 16384;

// one tile = 256 consecutive columns of one output row; NC reals per element
// (2 for complex pairs).  A permutation entry outside its range gives NaN
// (the load then reads element 0, which always exists).
template <typename T, int NC>
__global__ __launch_bounds__(kPermBlock) void k_permute(const T *__restrict__ x, T *__restrict__ y,
                                                        const int64_t *__restrict__ pu, const int64_t *__restrict__ pd,
                                                        int64_t Dup, int64_t Ddn, int64_t nblk, int64_t ntiles) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t p = t / nblk;
        const int64_t q = (t - p * nblk) * kPermBlock + threadIdx.x;
        if (q >= Ddn) continue;
        const int64_t sr = pu ? pu[p] : p;
        const int64_t sc = pd ? pd[q] : q;
        const bool ok = sr >= 0 && sr < Dup && sc >= 0 && sc < Ddn;
        const int64_t src = ok ? (sr * Ddn + sc) * NC : 0;
        const int64_t dst = (p * Ddn + q) * NC;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const T v = x[src + k];
            y[dst + k] = ok ? v : T(NAN);
        }
    }
}

template <typename T, int NC>
static int permute_launch(const ed_ham *h, const int64_t *pu, const int64_t *pd, const void *x, void *y,
                          hipStream_t s) {
    const int64_t nblk = (h->dim_dn + kPermBlock - 1) / kPermBlock;
    const int64_t ntiles = h->dim_up * nblk;
    const int grid = (int)std::min<int64_t>(ntiles, kPermMaxGrid);
    hipLaunchKernelGGL((k_permute<T, NC>), dim3(grid), dim3(kPermBlock), 0, s, static_cast<const T *>(x),
                       static_cast<T *>(y), pu, pd, h->dim_up, h->dim_dn, nblk, ntiles);
    return hip_check(hipGetLastError(), "ed_permute_vector");
}

}  // namespace ed

using namespace ed;

extern "C" {

int ed_permute_vector(const ed_ham *h, const int64_t *perm_up, const int64_t *perm_dn, const void *x, void *y,
                      void *stream) {
    clear_error();
    int rc = check_ham(h, "ed_permute_vector");
    if (rc) return rc;
    if (!x || !y) return set_error(ED_EINVAL, "ed_permute_vector: NULL vector");
    const int64_t bytes = h->dim_up * h->dim_dn * (h->dtype == ED_F64 ? 8 : 4) * (h->cplx ? 2 : 1);
    const char *xb = static_cast<const char *>(x), *yb = static_cast<const char *>(y);
    if (xb < yb + bytes && yb < xb + bytes) return set_error(ED_EINVAL, "ed_permute_vector: x and y overlap");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->dtype == ED_F64)
        return h->cplx ? permute_launch<double, 2>(h, perm_up, perm_dn, x, y, s)
                       : permute_launch<double, 1>(h, perm_up, perm_dn, x, y, s);
    return h->cplx ? permute_launch<float, 2>(h, perm_up, perm_dn, x, y, s)
                   : permute_launch<float, 1>(h, perm_up, perm_dn, x, y, s);
}

}  // extern "C"
