// Device-side state of a Lanczos run (the workspace header and partial-sum
// slots) shared by the step kernels of ed_device.hip and the fused step of
// ed_fused.hip, and the internal entry points of the fused step.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/ed.h"
#include "ed_launch.h"

namespace ed {

// ---------------------------------------------------------------------------
// Vectors are stored unnormalised ("deferred normalisation"): the buffer of
// Lanczos vector f_j holds s_j f_j with s_1 = |f1| and s_j = b_j, and the
// kernels apply sigma_j = 1/s_j on the fly.  The reference step is
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
// The fused step (ed_fused.hip) computes the same quantities in the same
// order with two passes over the vectors; between its steps q is kept and the
// update of line 6 is applied by the next step's first pass ("pending").
//
// workspace layout: [Hdr: 256 B][queue counters: 256 B][y: max_steps doubles]
//                   [part: P x 8 doubles][part2: 8192 doubles][part3: 8192 x 8 doubles]
struct Hdr {
    double sig_cur;    // 1 / s_j of the current vector
    double sig_prev;   // 1 / s_{j-1}
    double cx, cp;     // update coefficients on the stored F_j and F_{j-1}
    double scale;      // max_k(|a_k|, b_k) so far (breakdown threshold)
    double vinv;       // 1 / |v| for the two-pass ground state
    double norm2;      // |f1|^2 of the last init
    int32_t jdev;      // completed steps
    int32_t status;    // 0 running, ED_BREAKDOWN, or kInitBad
    int32_t pending;   // fused step: q of the last step is stored, its line-6 update not yet applied
    int32_t jcall;     // fused step: jdev when the current run of fused steps began
};
static_assert(sizeof(Hdr) <= 256, "header too large");
constexpr int32_t kInitBad = 100;
constexpr int kPartStride = 8;    // doubles per partial-sum slot
constexpr int kUpdBlocks = 8192;  // k_update / k_sumsq grid cap = part2 slots
constexpr int kFupSlots = 8192;   // fused up pass: grid cap = part3 slots

static inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

struct WsLayout {
    Hdr *hdr;
    int *ctr;
    double *y;
    double *part;
    double *part2;
    double *part3;
};

// k_down partial-sum slots: one per workgroup.  Rows too long for LDS are split
// into column blocks until the launch has kDownBlocks workgroups, so the grid
// is at most dim_up + kDownBlocks.
static inline int64_t n_partial_slots(const ed_ham *h) { return std::max<int64_t>(h->dim_up, 1) + kDownBlocks; }

static inline int64_t ws_bytes(const ed_ham *h, int32_t max_steps) {
    return 512 + align256(8 * (int64_t)std::max(max_steps, 1)) + align256(8 * kPartStride * n_partial_slots(h)) +
           8 * kUpdBlocks + 8 * kPartStride * kFupSlots;
}

static inline WsLayout ws_layout(const ed_ham *h, void *ws, int32_t max_steps) {
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
    p += 8 * kUpdBlocks;
    l.part3 = reinterpret_cast<double *>(p);
    return l;
}

__device__ __forceinline__ bool frozen(const Hdr *hdr, int max_steps) {
    return hdr->status != 0 || hdr->jdev >= max_steps;
}

// ---------------------------------------------------------------------------
// The fused step (ed_fused.hip).  Buffer roles (fp, f, q):
//   first step of a run (pending = false): fp = F_{j-1} (or unused at j = 1),
//     f = F_j, q = free; q receives q_j.  No rotation afterwards.
//   later steps (pending = true): fp = F_{j-2}, f = F_{j-1}, q = q_{j-1};
//     F_j = q_{j-1} - cx F_{j-1} - cp F_{j-2} is written over q, then q_j over
//     fp; afterwards the roles rotate (fp, f, q) <- (f, q, fp).
//   flush: F_{j+1} = q_j - cx F_j - cp F_{j-1} over q, b_{j+1}; then rotate.
// v != nullptr (two-pass ground state): v += w[j] F_j with w = y_j / s_j
// taken from the workspace's y array.
bool fused_eligible(const ed_ham *h);
// whether ed_ground_energy / ed_ground_state run on the fused step (no
// instance at present: the reference step is faster wherever measured)
inline bool fused_for_runs(const ed_ham *) { return false; }
int fused_step(const ed_ham *h, void *fp, void *f, void *q, bool pending, double *a, double *b, void *v,
               const WsLayout &w, int max_steps, hipStream_t s, hipEvent_t *ev = nullptr);
int fused_flush(const ed_ham *h, void *fp, void *f, void *q, const double *a, double *b, const WsLayout &w,
                int max_steps, hipStream_t s, hipEvent_t *ev = nullptr);
int fused_prepare();   // one-time function attributes (outside any capture)

}  // namespace ed
