// Device building blocks shared by the single-instance kernels and the
// batched persistent kernel: reductions, table decoding, the up-part tile
// (Eq. 4) and the down-part row block (Eq. 5).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ed {

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


// ---------------------------------------------------------------------------
// table entries e = (col << 1) | negative in an unsigned type E: uint16_t for a
// per-spin dimension up to 32767 (padding 0xFFFF), uint32_t beyond it (padding
// 0xFFFFFFFF).  Kernels read them in chunks of 8 (16 or 32 bytes); every
// kernel is generic over E, which the table pointer's type selects.
template <typename E> struct Chunk8 { uint4 q[sizeof(E) / 2]; };

template <typename E> __device__ __forceinline__ constexpr unsigned pad_entry() {
    return sizeof(E) == 2 ? 0xFFFFu : 0xFFFFFFFFu;
}
template <typename E> __device__ __forceinline__ bool is_pad(unsigned e) { return e == pad_entry<E>(); }

template <typename E> __device__ __forceinline__ Chunk8<E> pad_chunk() {
    Chunk8<E> c;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(E) / 2); ++i) c.q[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    return c;
}

template <typename E> __device__ __forceinline__ unsigned entry(const Chunk8<E> &c, int k) {
    if constexpr (sizeof(E) == 2) {
        const uint4 &q = c.q[0];
        const unsigned w = k < 2 ? q.x : (k < 4 ? q.y : (k < 6 ? q.z : q.w));
        return (k & 1) ? (w >> 16) : (w & 0xFFFFu);
    } else {
        const uint4 &q = c.q[k >> 2];
        const int j = k & 3;
        return j == 0 ? q.x : (j == 1 ? q.y : (j == 2 ? q.z : q.w));
    }
}

// One rounding per term: every up-part kernel adds a row's terms as
// acc = fma(sign, x, acc) in ascending column order, so all of them (every
// tile, the batched launch) produce the same bits.
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Up part (Eq. 4) on one tile = (column stripe s of width w = 64/R, row chunk rci):
// out[r, c] = t * sum_k sgn_k * x[J_up[r,k], c].  A wave serves R consecutive
// rows x w columns; the row index is wave-uniform, so each row's table chunks
// are scalar loads, chunks that are padding for every row of the wave are
// skipped, and the 8 gathers of a chunk per row are issued back to back
// (padding inside a chunk re-reads x[0, c] and is multiplied by zero).
template <typename T, int R, typename E>
__device__ __forceinline__ void up_tile(const T *__restrict__ x, T *__restrict__ out,
                                        const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc, int s,
                                        int rci, T t) {
    constexpr int w = 64 / R;
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = R == 1 ? 0 : lane / w;
    const int c = s * w + (lane & (w - 1));
    const bool cok = c < Ddn;
    const int cc = cok ? c : 0;
    const T *xc = x + cc;
    const int r1 = min(Dup, (rci + 1) * rc);
    const int nch = W8 >> 3;
    for (int rb = rci * rc + wave * R; rb < r1; rb += nwave * R) {
        const int r = rb + sub;
        T acc = T(0);
        for (int k8 = 0; k8 < nch; ++k8) {
            Chunk8<E> q[R];
            bool any = false;
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int ru = min(rb + u, Dup - 1);
                q[u] = *reinterpret_cast<const Chunk8<E> *>(tab + (int64_t)ru * W8 + 8 * k8);
                any = any || (!is_pad<E>(entry(q[u], 0)) && rb + u < r1);
            }
            if (!any) break;   // ascending columns, padding at the end: the rest is padding too
            T v[8], sg[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                unsigned e = entry(q[0], k);
#pragma unroll
                for (int u = 1; u < R; ++u)
                    if (sub == u) e = entry(q[u], k);
                const bool pk = !is_pad<E>(e);
                sg[k] = pk ? ((e & 1u) ? T(-1) : T(1)) : T(0);
                v[k] = xc[(int64_t)(pk ? (e >> 1) : 0u) * Ddn];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) acc = fma_t(sg[k], v[k], acc);
        }
        if (cok && r < r1) __builtin_nontemporal_store(t * acc, out + (int64_t)r * Ddn + c);
    }
}

// Chunk count template parameter for a table of stride W8 (nch = W8/8 chunks
// of 8 entries): the smallest of 1, 2, 4, 8 that holds nch.
__host__ __device__ constexpr int nch_class(int nch) { return nch <= 1 ? 1 : (nch <= 2 ? 2 : (nch <= 4 ? 4 : 8)); }

// The NCH chunks of table row `row` (scalar loads when row is wave-uniform).
// Chunks at or beyond nch = W8/8 read as padding.  The loads themselves read
// NCH*8 entries from the row start, which stays inside the packed table: its
// second (interleaved) half of dim*W8 entries follows the row-major half and
// NCH*8 - W8 < W8.
template <int NCH, typename E>
__device__ __forceinline__ void row_chunks(const E *__restrict__ tab, int row, int W8, int nch,
                                           Chunk8<E> (&q)[NCH]) {
    const Chunk8<E> *p = reinterpret_cast<const Chunk8<E> *>(tab + (int64_t)row * W8);
#pragma unroll
    for (int k8 = 0; k8 < NCH; ++k8) {
        const Chunk8<E> v = p[k8];
        q[k8] = k8 < nch ? v : pad_chunk<E>();
    }
}

// One row of the up part with NL live chunks: every gather of the row is
// issued, then the previous row's result is stored (so the store does not
// sit ahead of these gathers in the in-order memory counter, and its data
// register is not reused while it is in flight), then the row is summed.
template <typename T, int NL, int NCH, typename E>
__device__ __forceinline__ void up_row(const T *__restrict__ xs, unsigned cc, int Ddn, const Chunk8<E> (&q)[NCH], T t,
                                       T &pend, T *&pend_ptr, T *row_out) {
    T v[NL > 0 ? NL : 1][8];
#pragma unroll
    for (int k8 = 0; k8 < NL; ++k8)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned e = entry(q[k8], k);
            // wave-uniform row base, 32-bit lane offset
            const T *xr = xs + (int64_t)(!is_pad<E>(e) ? (e >> 1) : 0u) * Ddn;
            v[k8][k] = xr[cc];
        }
    if (pend_ptr) __builtin_nontemporal_store(pend, pend_ptr);
    T acc = T(0);
#pragma unroll
    for (int k8 = 0; k8 < NL; ++k8)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned e = entry(q[k8], k);
            const T sg = is_pad<E>(e) ? T(0) : ((e & 1u) ? T(-1) : T(1));
            acc = fma_t(sg, v[k8][k], acc);
        }
    pend = t * acc;
    pend_ptr = row_out;
}

// Up part with 64-column stripes (one row per wave), all of a row's gathers
// in flight at once.  The row's table chunks arrive by scalar loads, fetched
// one row ahead; the number of live chunks (the columns in a row ascend, so
// padding is a suffix) selects straight-line code that issues every gather
// of the row before the first is consumed.  Padding inside the last live
// chunk re-reads x[0, c] and is multiplied by zero.
template <typename T, int NCH, typename E>
__device__ __forceinline__ void up_tile_wide(const T *__restrict__ x, T *__restrict__ out,
                                             const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc,
                                             int s, int rci, T t) {
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = s * 64 + lane;
    const bool cok = c < Ddn;
    const T *xs = x + s * 64;
    const unsigned cc = cok ? (unsigned)lane : 0u;
    const int r1 = min(Dup, (rci + 1) * rc);
    const int nch = W8 >> 3;
    int rb = rci * rc + wave;
    if (rb >= r1) return;
    Chunk8<E> q[NCH];
    row_chunks<NCH>(tab, rb, W8, nch, q);
    T pend = T(0);
    T *pend_ptr = nullptr;
    for (; rb < r1; rb += nwave) {
        int nl = 0;
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) nl += !is_pad<E>(entry(q[k8], 0)) ? 1 : 0;
        Chunk8<E> qn[NCH];
        row_chunks<NCH>(tab, min(rb + nwave, r1 - 1), W8, nch, qn);
        T *row_out = cok ? out + (int64_t)rb * Ddn + c : nullptr;
        switch (nl) {
        case 0: up_row<T, 0, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 1: up_row<T, 1, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 2: if constexpr (NCH >= 2) up_row<T, 2, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 3: if constexpr (NCH >= 4) up_row<T, 3, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 4: if constexpr (NCH >= 4) up_row<T, 4, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 5: if constexpr (NCH >= 8) up_row<T, 5, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 6: if constexpr (NCH >= 8) up_row<T, 6, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        case 7: if constexpr (NCH >= 8) up_row<T, 7, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        default: if constexpr (NCH >= 8) up_row<T, 8, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out); break;
        }
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) q[k8] = qn[k8];
    }
    if (pend_ptr) __builtin_nontemporal_store(pend, pend_ptr);
}

// Up part with 64*V-column stripes: the one-row kernel with V adjacent
// columns per lane (V = 2: float2 / double2, V = 4: float4), so each gather
// instruction moves V times the bytes and a row needs 1/V of the
// instructions (the up part is bound by gather instructions in flight, not by
// bytes).  Needs row starts aligned to V elements (row length a multiple of
// V); each column's terms are still added in ascending order with one fused
// multiply-add each.
template <typename T, int V> struct VecT;
template <> struct VecT<float, 2> { using type = float2; };
template <> struct VecT<double, 2> { using type = double2; };
template <> struct VecT<float, 4> { using type = float4; };

template <typename VT> __device__ __forceinline__ auto vcomp(const VT &v, int i) {
    if constexpr (sizeof(VT) / sizeof(v.x) == 2) return i == 0 ? v.x : v.y;
    else return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Gathers in flight per batch in up_rowv: a row's first 16 are issued
// together, the rest (rows of up to 32 entries) after the first batch is
// summed.  Holding all 32 in registers would cost the kernel a wave per SIMD.
constexpr int kUpBatch = 16;

// One row of the vector up tile with exactly NE entries (a row's entries come
// first, padding after them): every gather is a real row of x, then the
// previous row's result is stored, then the row is summed in ascending column
// order with one fused multiply-add per term.

template <typename T, int V, int NE, int NCH, typename E>
__device__ __forceinline__ void up_rowv(const T *__restrict__ xs, unsigned cc, int Ddn, const Chunk8<E> (&q)[NCH], T t,
                                        T (&pend)[V], T *&pend_ptr, T *row_out) {
    using VT = typename VecT<T, V>::type;
    constexpr int B0 = NE < kUpBatch ? NE : kUpBatch;
    VT v[B0 > 0 ? B0 : 1];
#pragma unroll
    for (int j = 0; j < B0; ++j) {
        const unsigned e = entry(q[j >> 3], j & 7);
        v[j] = *reinterpret_cast<const VT *>(xs + (int64_t)(e >> 1) * Ddn + cc);
    }
    if (pend_ptr) {
#pragma unroll
        for (int i = 0; i < V; ++i) __builtin_nontemporal_store(pend[i], pend_ptr + i);
    }
    T a[V];
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] = T(0);
#pragma unroll
    for (int j = 0; j < B0; ++j) {
        const unsigned e = entry(q[j >> 3], j & 7);
        const T sg = (e & 1u) ? T(-1) : T(1);
#pragma unroll
        for (int i = 0; i < V; ++i) a[i] = fma_t(sg, vcomp(v[j], i), a[i]);
    }
    // later batches: the scheduling barrier keeps their loads after the sums
    // above, so their registers reuse the first batch's
#pragma unroll
    for (int j0 = B0; j0 < NE; j0 += kUpBatch) {
        __builtin_amdgcn_sched_barrier(0);
        VT w[kUpBatch];
#pragma unroll
        for (int j = j0; j < NE && j < j0 + kUpBatch; ++j) {
            const unsigned e = entry(q[j >> 3], j & 7);
            w[j - j0] = *reinterpret_cast<const VT *>(xs + (int64_t)(e >> 1) * Ddn + cc);
        }
#pragma unroll
        for (int j = j0; j < NE && j < j0 + kUpBatch; ++j) {
            const unsigned e = entry(q[j >> 3], j & 7);
            const T sg = (e & 1u) ? T(-1) : T(1);
#pragma unroll
            for (int i = 0; i < V; ++i) a[i] = fma_t(sg, vcomp(w[j - j0], i), a[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < V; ++i) pend[i] = t * a[i];
    pend_ptr = row_out;
}

// Dispatch a row with ne entries (wave-uniform) to its exact-count variant,
// for tables of up to 8 * NCH <= 32 entries per row.
template <typename T, int V, int NCH, typename E, int NE = 0>
__device__ __forceinline__ void up_rowv_n(int ne, const T *__restrict__ xs, unsigned cc, int Ddn,
                                          const Chunk8<E> (&q)[NCH], T t, T (&pend)[V], T *&pend_ptr, T *row_out) {
    if constexpr (NE <= 8 * NCH) {
        if (ne == NE)
            up_rowv<T, V, NE, NCH, E>(xs, cc, Ddn, q, t, pend, pend_ptr, row_out);
        else
            up_rowv_n<T, V, NCH, E, NE + 1>(ne, xs, cc, Ddn, q, t, pend, pend_ptr, row_out);
    }
}

template <typename T, int V, int NCH, typename E>
__device__ __forceinline__ void up_tile_vec(const T *__restrict__ x, T *__restrict__ out,
                                            const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc,
                                            int s, int rci, T t) {
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = s * 64 * V + V * lane;
    const bool cok = c < Ddn;   // Ddn a multiple of V: the lane's other columns are valid too
    const T *xs = x + s * 64 * V;
    const unsigned cc = cok ? (unsigned)(V * lane) : 0u;
    const int r1 = min(Dup, (rci + 1) * rc);
    const int nch = W8 >> 3;
    int rb = rci * rc + wave;
    if (rb >= r1) return;
    Chunk8<E> q[NCH];
    row_chunks<NCH>(tab, rb, W8, nch, q);
    T pend[V];
#pragma unroll
    for (int i = 0; i < V; ++i) pend[i] = T(0);
    T *pend_ptr = nullptr;
    for (; rb < r1; rb += nwave) {
        // the row's entries: every entry of the row's chunks that is not padding (wave-uniform)
        int ne = 0;
#pragma unroll
        for (int j = 0; j < 8 * NCH; ++j) ne += !is_pad<E>(entry(q[j >> 3], j & 7)) ? 1 : 0;
        Chunk8<E> qn[NCH];
        row_chunks<NCH>(tab, min(rb + nwave, r1 - 1), W8, nch, qn);
        T *row_out = cok ? out + (int64_t)rb * Ddn + c : nullptr;
        up_rowv_n<T, V, NCH, E>(ne, xs, cc, Ddn, q, t, pend, pend_ptr, row_out);
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) q[k8] = qn[k8];
    }
    if (pend_ptr) {
#pragma unroll
        for (int i = 0; i < V; ++i) __builtin_nontemporal_store(pend[i], pend_ptr + i);
    }
}

// Up part with 32-column stripes, two rows per wave (lanes 0-31 row rb,
// lanes 32-63 row rb+1): half the stripe footprint of the one-row kernel, so
// a stripe of x stays in an XCD's L2, with the same latency tolerance.  Both
// rows' table chunks are scalar loads fetched one pair ahead; each lane picks
// its row's entry, and every gather of the pair is issued before the first is
// consumed (the chunk count is the larger of the two rows').  A row beyond the
// tile or the table reads as padding (its chunks are loaded from a valid row
// and discarded).  Used for tables of at most 4 chunks (scalar registers).
template <typename T, int NL, int NCH, typename E>
__device__ __forceinline__ void up_pair(const T *__restrict__ xc, int Ddn, bool hi, const Chunk8<E> (&qa)[NCH],
                                        const Chunk8<E> (&qb)[NCH], T t, T &pend, T *&pend_ptr, T *row_out) {
    T v[NL > 0 ? NL : 1][8];
#pragma unroll
    for (int k8 = 0; k8 < NL; ++k8)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned e = hi ? entry(qb[k8], k) : entry(qa[k8], k);
            v[k8][k] = xc[(int64_t)(!is_pad<E>(e) ? (e >> 1) : 0u) * Ddn];
        }
    if (pend_ptr) __builtin_nontemporal_store(pend, pend_ptr);
    T acc = T(0);
#pragma unroll
    for (int k8 = 0; k8 < NL; ++k8)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned e = hi ? entry(qb[k8], k) : entry(qa[k8], k);
            const T sg = is_pad<E>(e) ? T(0) : ((e & 1u) ? T(-1) : T(1));
            acc = fma_t(sg, v[k8][k], acc);
        }
    pend = t * acc;
    pend_ptr = row_out;
}

template <int NCH, typename E>
__device__ __forceinline__ int live_chunks(const Chunk8<E> (&q)[NCH]) {
    int n = 0;
#pragma unroll
    for (int k8 = 0; k8 < NCH; ++k8) n += !is_pad<E>(entry(q[k8], 0)) ? 1 : 0;
    return n;
}

template <typename T, int NCH, typename E>
__device__ __forceinline__ void up_tile_pair(const T *__restrict__ x, T *__restrict__ out,
                                             const E *__restrict__ tab, int Dup, int Ddn, int W8, int rc,
                                             int s, int rci, T t) {
    static_assert(NCH <= 4, "two rows of scalar table chunks");
    const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool hi = lane >= 32;
    const int c = s * 32 + (lane & 31);
    const bool cok = c < Ddn;
    const T *xc = x + (cok ? c : 0);
    const int r1 = min(Dup, (rci + 1) * rc);
    const int nch = W8 >> 3;
    int rb = rci * rc + 2 * wave;
    if (rb >= r1) return;
    Chunk8<E> qa[NCH], qb[NCH];
    row_chunks<NCH>(tab, rb, W8, nch, qa);
    row_chunks<NCH>(tab, min(rb + 1, Dup - 1), W8, rb + 1 < r1 ? nch : 0, qb);
    T pend = T(0);
    T *pend_ptr = nullptr;
    for (; rb < r1; rb += 2 * nwave) {
        const int nl = max(live_chunks(qa), live_chunks(qb));
        const int rn = min(rb + 2 * nwave, r1 - 1);
        Chunk8<E> qan[NCH], qbn[NCH];
        row_chunks<NCH>(tab, rn, W8, nch, qan);
        row_chunks<NCH>(tab, min(rn + 1, Dup - 1), W8, rn + 1 < r1 ? nch : 0, qbn);
        const int r = rb + (hi ? 1 : 0);
        T *row_out = (cok && r < r1) ? out + (int64_t)r * Ddn + c : nullptr;
        switch (nl) {
        case 0: up_pair<T, 0, NCH, E>(xc, Ddn, hi, qa, qb, t, pend, pend_ptr, row_out); break;
        case 1: up_pair<T, 1, NCH, E>(xc, Ddn, hi, qa, qb, t, pend, pend_ptr, row_out); break;
        case 2: if constexpr (NCH >= 2) up_pair<T, 2, NCH, E>(xc, Ddn, hi, qa, qb, t, pend, pend_ptr, row_out); break;
        case 3: if constexpr (NCH >= 4) up_pair<T, 3, NCH, E>(xc, Ddn, hi, qa, qb, t, pend, pend_ptr, row_out); break;
        default: if constexpr (NCH >= 4) up_pair<T, 4, NCH, E>(xc, Ddn, hi, qa, qb, t, pend, pend_ptr, row_out); break;
        }
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) {
            qa[k8] = qan[k8];
            qb[k8] = qbn[k8];
        }
    }
    if (pend_ptr) __builtin_nontemporal_store(pend, pend_ptr);
}

// Chunk k8 of column c in the 8-interleaved table; chunks at or beyond nch
// read as padding.  The load always goes to a valid table address (nch >= 1
// in every variant with NCH >= 1) and the value is selected afterwards:
// selecting between the table's address and a constant's would make the
// address space unknown and turn the 16-byte load into flat dword loads, and
// a branch around the load would make the wait counts inexact.  NCH = 0 is the
// variant for a species without hopping, which may pass no table at all.
template <int NCH, typename E>
__device__ __forceinline__ Chunk8<E> table_chunk(const Chunk8<E> *__restrict__ til, int k8, int nch, int Ddn,
                                                 int c) {
    if constexpr (NCH == 0) {
        return pad_chunk<E>();
    } else {
        // padding is all ones: OR it in, so the load is always consumed and
        // the compiler cannot sink it into a branch
        const unsigned m = k8 < nch ? 0u : ~0u;
        Chunk8<E> v = til[(int64_t)(k8 < nch ? k8 : 0) * Ddn + c];
#pragma unroll
        for (int i = 0; i < (int)(sizeof(E) / 2); ++i)
            v.q[i] = make_uint4(v.q[i].x | m, v.q[i].y | m, v.q[i].z | m, v.q[i].w | m);
        return v;
    }
}

// table_chunk with the chunk's element offset (k8 * Ddn) precomputed and a
// wave-uniform choice: chunk k8 when real, else padding read from chunk 0's
// address (the per-wavefront chunk counts of the one-species down part)
template <typename E>
__device__ __forceinline__ Chunk8<E> table_chunk_off(const Chunk8<E> *__restrict__ til, int64_t off, bool real,
                                                     int c) {
    const unsigned m = real ? 0u : ~0u;
    Chunk8<E> v = til[(real ? off : 0) + c];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(E) / 2); ++i)
        v.q[i] = make_uint4(v.q[i].x | m, v.q[i].y | m, v.q[i].z | m, v.q[i].w | m);
    return v;
}

// v if keep, else +0, without a branch (the loaded value is always consumed)
__device__ __forceinline__ double keep_or_zero(double v, bool keep) {
    return __longlong_as_double(__double_as_longlong(v) & (keep ? ~0ll : 0ll));
}
__device__ __forceinline__ float keep_or_zero(float v, bool keep) {
    return __int_as_float(__float_as_int(v) & (keep ? ~0 : 0));
}

// ---------------------------------------------------------------------------
// Down part (Eq. 5) on a block of rows:
//   q[r, c] = sig * (io[r, c] + t * sum_k sgn_k x[r, J_dn[c,k]] + U*Docc[r,c]*x[r,c])
//             (- cprev * p[r, c] in a Lanczos step, cprev = b_j / s_{j-1})
// io holds the up part on entry and q on exit.  The rows are staged in LDS
// with 16-byte loads by the caller; lane c reads its table row from the
// 8-interleaved layout (16 bytes per chunk, contiguous across lanes).  The
// column loop is software pipelined: the next column's table chunks, up part
// and f_{j-1} value are loaded while the current column gathers from the rows
// (branch-free: padding reads one broadcast address times zero).
// NCH = largest number of table chunks per row (W8 / 8 <= NCH) handled.
// MODE 0: plain H.v (sig = 1).  MODE 1: Lanczos, partial q.x.
// MODE 2: Lanczos mixed form, partials (q.x, q.p, x.x, x.p, p.p).
// P8: take 8-byte pieces where the source is 8- but not 16-byte aligned (the
// second row of a pair of float rows of even length); else element by element.
template <typename T, bool P8 = false>
__device__ __forceinline__ void stage_rows(const T *__restrict__ src, T *__restrict__ dst, int n) {
    // 16-byte pieces, four in flight per thread; the tail element by element
    constexpr int V = 16 / sizeof(T);
    const int nv = n / V;
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst);
    const bool aligned = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
    if (aligned) {
        int i = threadIdx.x;
        for (; i + 3 * (int)blockDim.x < nv; i += 4 * blockDim.x) {
            const uint4 a = s4[i], b = s4[i + blockDim.x], c = s4[i + 2 * blockDim.x], d = s4[i + 3 * blockDim.x];
            d4[i] = a;
            d4[i + blockDim.x] = b;
            d4[i + 2 * blockDim.x] = c;
            d4[i + 3 * blockDim.x] = d;
        }
        for (; i < nv; i += blockDim.x) d4[i] = s4[i];
        for (int k = nv * V + threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
    } else if (P8 && (reinterpret_cast<uintptr_t>(src) & 7) == 0 && (reinterpret_cast<uintptr_t>(dst) & 7) == 0) {
        constexpr int V2 = 8 / sizeof(T);
        const int n2 = n / V2;
        const uint2 *s2 = reinterpret_cast<const uint2 *>(src);
        uint2 *d2 = reinterpret_cast<uint2 *>(dst);
        int i = threadIdx.x;
        for (; i + 3 * (int)blockDim.x < n2; i += 4 * blockDim.x) {
            const uint2 a = s2[i], b = s2[i + blockDim.x], c = s2[i + 2 * blockDim.x], d = s2[i + 3 * blockDim.x];
            d2[i] = a;
            d2[i + blockDim.x] = b;
            d2[i + 2 * blockDim.x] = c;
            d2[i + 3 * blockDim.x] = d;
        }
        for (; i < n2; i += blockDim.x) d2[i] = s2[i];
        for (int k = n2 * V2 + threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
    } else {
        for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
    }
}

// The down-part sum of one column (Eq. 5): the row's elements at the column's
// table entries times their signs, in two interleaved partial sums (even
// entries in acc0, odd in acc1, each term added with one rounding).  Chunks
// from nch on, and chunks that are padding for every lane of the wave, are
// skipped.  Padding entries read element 0 and add it times zero.
template <typename T, int NCH, typename E>
__device__ __forceinline__ void down_gather(const T *__restrict__ xrow, const Chunk8<E> (&tq)[NCH > 0 ? NCH : 1],
                                            int nch, T &acc0, T &acc1) {
    acc0 = T(0);
    acc1 = T(0);
#pragma unroll
    for (int k8 = 0; k8 < NCH; ++k8) {
        if (k8 >= nch) break;
        // a chunk whose first entry is padding is padding throughout; skip it
        // when that holds for every lane of the wave
        if (!__any(!is_pad<E>(entry(tq[k8], 0)))) break;
        // likewise the chunk's second half (entries 4..7), in FP32: gather it only where some lane needs
        // it (in FP64 the extra branch cost more than the skipped gathers saved)
        bool upper = true;
        if constexpr (sizeof(T) == 4) upper = __any(!is_pad<E>(entry(tq[k8], 4)));
        T v[8], sg[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k >= 4 && !upper) {
                v[k] = T(0);
                sg[k] = T(0);
                continue;
            }
            const unsigned e = entry(tq[k8], k);
            const bool pk = !is_pad<E>(e);
            sg[k] = pk ? ((e & 1u) ? T(-1) : T(1)) : T(0);
            v[k] = xrow[pk ? (int)(e >> 1) : 0];   // padding: one broadcast address
        }
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            acc0 += sg[k] * v[k];
            acc1 += sg[k + 1] * v[k + 1];
        }
    }
}

// -v where the sign bit s31 (bit 31) is set, else v: one integer XOR on the
// word holding the sign
__device__ __forceinline__ double flip_sign(double v, unsigned s31) {
    uint2 u = __builtin_bit_cast(uint2, v);
    u.y ^= s31;
    return __builtin_bit_cast(double, u);
}
__device__ __forceinline__ float flip_sign(float v, unsigned s31) {
    return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) ^ s31);
}

// down_gather for a row staged in LDS with a zero at index zslot (= the row
// length): a padding entry's column (all ones) is clamped to zslot, so it adds
// a zero, and an entry's sign flips the loaded value's sign bit, so each
// entry costs a clamp, an address, a sign and an add instead of a selected
// sign factor and a selected address.  The terms and their order are
// down_gather's (x + (-v) is fma(-1, v, x)), so the results are the same bits.
template <typename T, int NCH, typename E, bool WIN = false>
__device__ __forceinline__ void down_gather_z(const T *__restrict__ xrow, const Chunk8<E> (&tq)[NCH > 0 ? NCH : 1],
                                             int nch, unsigned zslot, T &acc0, T &acc1,
                                             unsigned xlo = 0) {
    acc0 = T(0);
    acc1 = T(0);
#pragma unroll
    for (int k8 = 0; k8 < NCH; ++k8) {
        if (k8 >= nch) break;
        if (!__any(!is_pad<E>(entry(tq[k8], 0)))) break;
        bool upper = true;
        if constexpr (sizeof(T) == 4) upper = __any(!is_pad<E>(entry(tq[k8], 4)));
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k >= 4 && !upper) {
                v[k] = T(0);
                continue;
            }
            const unsigned e = entry(tq[k8], k);
            if constexpr (WIN)   // xrow holds the window from column xlo; padding clamps onto its zero
                v[k] = flip_sign(xrow[min((e >> 1) - xlo, zslot)], e << 31);
            else
                v[k] = flip_sign(xrow[min(e >> 1, zslot)], e << 31);
        }
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            acc0 += v[k];
            acc1 += v[k + 1];
        }
    }
}

// Elements [i0, iend) of a block of rows starting at row r0 of one instance
// (element i = row i / Ddn, column i % Ddn of the block): q = sig * (io + t *
// down-part + U Docc x) - cprev * p, in place on io; per-thread partial sums
// added to s[].  xrows: the rows (LDS copy or global); base: offset of row r0
// in the global vectors.  A workgroup takes whole rows (i0 = 0, iend = rows *
// Ddn) or, for one long row, a range of its columns.  IO = false: there is
// no up part (the up species cannot hop); io is written but not read.  ZS:
// one row in LDS followed by a zero (down_gather_z).  WIN (with ZS, one
// row): xrows is the window of the row from column xlo, its zero at index
// zs_win, and [i0, iend) a block of columns inside it; the table's columns
// are absolute (WIN 1) or relative to xlo already (WIN 2).  WCH (one row,
// i0 a multiple of 64): wch holds the table's chunk count per 64 columns; a
// wavefront reads only its own count of chunks, the rest as padding from
// chunk 0's address (the same bits: those chunks are padding for all of its
// columns).
template <typename T, int MODE, int NCH, bool MULTI, bool IO = true, bool ZS = false, typename E, int WIN = 0,
          bool WCH = false>
__device__ __forceinline__ void down_rows(const T *__restrict__ xrows, T *__restrict__ io, const T *__restrict__ p,
                                          const E *__restrict__ tab, const uint64_t *__restrict__ st_up_r0,
                                          const uint64_t *__restrict__ st_dn, int Ddn, int W8, int i0, int iend,
                                          int64_t base, T t, T U, T sig, T cprev, bool use_p,
                                          double (&s)[MODE == 2 ? 5 : 1], unsigned xlo = 0, unsigned zs_win = 0,
                                          const uint32_t *__restrict__ wch = nullptr) {
    const Chunk8<E> *til = reinterpret_cast<const Chunk8<E> *>(tab + (int64_t)Ddn * W8);   // 8-interleaved part
    const int nch = W8 >> 3;
    // the chunk count of column col's wavefront: one scalar load per wavefront
    // (its 64 columns share col / 64, so the first lane's index is every lane's),
    // issued a column ahead of its use: scalar loads complete on their own
    // counter, so waiting for it never waits for the vector loads
    auto chunks_of = [&](int col) -> int {
        if constexpr (WCH) return min((int)wch[__builtin_amdgcn_readfirstlane(col >> 6)], nch);
        else return nch;
    };
    const int n = iend;
    // Every global operand of a column (table chunks, up part, f_{j-1}, the
    // down state) is fetched one column ahead, so that the wait for the
    // current column's operands (memory counters complete in issue order)
    // never includes the next column's.
    // The loads are unconditional (the last column's prefetch re-reads a valid
    // element; f_{j-1} is read whenever a Lanczos step has one and zeroed when
    // it is not used) so that the wait count is exact on every path.
    // MULTI: the block holds several (short) rows and a thread's columns move
    // between them; else one row, whose up state is a wave-uniform constant.
    int i = i0 + threadIdx.x;
    if (i >= n) return;
    const uint64_t su0 = st_up_r0[0];
    Chunk8<E> tq[NCH > 0 ? NCH : 1];
    T iov, pv;
    uint64_t sdv, suv = su0;
    int c, rr;
    if constexpr (MULTI) { rr = i / Ddn; c = i - rr * Ddn; } else { rr = 0; c = i; }
    int ncw = chunks_of(c), ncwn = nch;
    int64_t koff[NCH > 0 ? NCH : 1];
    if constexpr (WCH) {
        ncwn = chunks_of(min(i + (int)blockDim.x, n - 1));
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) koff[k8] = (int64_t)k8 * Ddn;
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = table_chunk_off<E>(til, koff[k8], k8 < ncw, c);
    } else {
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = table_chunk<NCH, E>(til, k8, ncw, Ddn, c);
    }
    if constexpr (IO) iov = io[base + i]; else iov = T(0);
    if constexpr (MODE != 0) pv = keep_or_zero(p[base + i], use_p); else pv = T(0);
    sdv = st_dn[c];
    if constexpr (MULTI) suv = st_up_r0[rr];
    for (; i < n; i += blockDim.x) {
        const int in = min(i + (int)blockDim.x, n - 1);
        int cn, rrn;
        if constexpr (MULTI) { rrn = in / Ddn; cn = in - rrn * Ddn; } else { rrn = 0; cn = in; }
        Chunk8<E> tqn[NCH > 0 ? NCH : 1];
        int ncwn2 = nch;
        if constexpr (WCH) {
            ncwn2 = chunks_of(min(i + 2 * (int)blockDim.x, n - 1));
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) tqn[k8] = table_chunk_off<E>(til, koff[k8], k8 < ncwn, cn);
        } else {
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) tqn[k8] = table_chunk<NCH, E>(til, k8, ncwn, Ddn, cn);
        }
        T iovn;
        if constexpr (IO) iovn = io[base + in]; else iovn = T(0);
        T pvn;
        if constexpr (MODE != 0) pvn = keep_or_zero(p[base + in], use_p); else pvn = T(0);
        const uint64_t sdn = st_dn[cn];
        uint64_t sun = su0;
        if constexpr (MULTI) sun = st_up_r0[rrn];
        const T *xrow = xrows + (int64_t)rr * Ddn;
        T acc0, acc1;
        if constexpr (ZS && WIN == 1)
            down_gather_z<T, NCH, E, true>(xrow, tq, nch, zs_win, acc0, acc1, xlo);
        else if constexpr (ZS && WIN == 2)
            down_gather_z<T, NCH, E>(xrow, tq, nch, zs_win, acc0, acc1);
        else if constexpr (ZS)
            down_gather_z<T, NCH, E>(xrow, tq, nch, (unsigned)Ddn, acc0, acc1);
        else
            down_gather<T, NCH, E>(xrow, tq, ncw, acc0, acc1);
        T xv;
        if constexpr (WIN) xv = xrow[c - (int)xlo]; else xv = xrow[c];
        const T nd = static_cast<T>(__popcll(suv & sdv));
        T q = iov + t * (acc0 + acc1) + U * nd * xv;
        if (MODE != 0) {
            q *= sig;
            if (use_p) q -= cprev * pv;
        }
        io[base + i] = q;
        if (MODE != 0) {
            const double qd = q, xd = xv;
            s[0] += qd * xd;
            if constexpr (MODE == 2) {
                const double pd = pv;
                s[1] += qd * pd;
                s[2] += xd * xd;
                s[3] += xd * pd;
                s[4] += pd * pd;
            }
        }
        c = cn;
        rr = rrn;
        iov = iovn;
        pv = pvn;
        sdv = sdn;
        suv = sun;
        ncw = ncwn;
        ncwn = ncwn2;
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = tqn[k8];
    }
}


// down_gather_z for two rows staged in LDS (each followed by a zero at index
// zslot): one table decode per entry serves both rows.  Each row's terms are
// summed exactly as down_gather_z sums them.
template <typename T, int NCH, typename E>
__device__ __forceinline__ void down_gather_z2(const T *__restrict__ x0, const T *__restrict__ x1,
                                               const Chunk8<E> (&tq)[NCH > 0 ? NCH : 1], int nch, unsigned zslot,
                                               T &a00, T &a01, T &a10, T &a11) {
    a00 = T(0);
    a01 = T(0);
    a10 = T(0);
    a11 = T(0);
#pragma unroll
    for (int k8 = 0; k8 < NCH; ++k8) {
        if (k8 >= nch) break;
        if (!__any(!is_pad<E>(entry(tq[k8], 0)))) break;
        bool upper = true;
        if constexpr (sizeof(T) == 4) upper = __any(!is_pad<E>(entry(tq[k8], 4)));
        T v0[8], v1[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k >= 4 && !upper) {
                v0[k] = T(0);
                v1[k] = T(0);
                continue;
            }
            const unsigned e = entry(tq[k8], k);
            const unsigned at = min(e >> 1, zslot), sgn = e << 31;
            v0[k] = flip_sign(x0[at], sgn);
            v1[k] = flip_sign(x1[at], sgn);
        }
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            a00 += v0[k];
            a01 += v0[k + 1];
            a10 += v1[k];
            a11 += v1[k + 1];
        }
    }
}

// down_rows for two rows r0, r0 + 1 of one workgroup, staged in LDS at x0 and
// x1 (each followed by a zero): lane c takes column c of both rows, so each
// table chunk is loaded once for the two.  Per row the arithmetic is
// down_rows' (the same q bits); the partial sums take row 0's terms, then row
// 1's, column by column.  two = false: only row 0 exists (x1 = x0, nothing of
// row 1 is stored or summed).  WCH: per-wavefront chunk counts, as in
// down_rows.
template <typename T, int MODE, int NCH, typename E, bool WCH = false>
__device__ __forceinline__ void down_rows2(const T *__restrict__ x0, const T *__restrict__ x1, T *__restrict__ io,
                                           const T *__restrict__ p, const E *__restrict__ tab, uint64_t su0,
                                           uint64_t su1, bool two, const uint64_t *__restrict__ st_dn, int Ddn,
                                           int W8, int64_t base, T t, T U, T sig, T cprev, bool use_p,
                                           double (&s)[MODE == 2 ? 5 : 1],
                                           const uint32_t *__restrict__ wch = nullptr) {
    const Chunk8<E> *til = reinterpret_cast<const Chunk8<E> *>(tab + (int64_t)Ddn * W8);
    const int nch = W8 >> 3;
    const int64_t base1 = base + (two ? Ddn : 0);
    int c = threadIdx.x;
    if (c >= Ddn) return;
    auto chunks_of = [&](int col) -> int {
        if constexpr (WCH) return min((int)wch[__builtin_amdgcn_readfirstlane(col >> 6)], nch);
        else return nch;
    };
    Chunk8<E> tq[NCH > 0 ? NCH : 1];
    int ncwn = nch;
    int64_t koff[NCH > 0 ? NCH : 1];
    if constexpr (WCH) {
        const int ncw = chunks_of(c);
        ncwn = chunks_of(min(c + (int)blockDim.x, Ddn - 1));
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) koff[k8] = (int64_t)k8 * Ddn;
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = table_chunk_off<E>(til, koff[k8], k8 < ncw, c);
    } else {
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = table_chunk<NCH, E>(til, k8, nch, Ddn, c);
    }
    T io0 = io[base + c], io1 = io[base1 + c];
    T p0 = T(0), p1 = T(0);
    if constexpr (MODE != 0) {
        p0 = keep_or_zero(p[base + c], use_p);
        p1 = keep_or_zero(p[base1 + c], use_p);
    }
    uint64_t sdv = st_dn[c];
    for (; c < Ddn; c += blockDim.x) {
        const int cn = min(c + (int)blockDim.x, Ddn - 1);
        Chunk8<E> tqn[NCH > 0 ? NCH : 1];
        int ncwn2 = nch;
        if constexpr (WCH) {
            ncwn2 = chunks_of(min(c + 2 * (int)blockDim.x, Ddn - 1));
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) tqn[k8] = table_chunk_off<E>(til, koff[k8], k8 < ncwn, cn);
        } else {
#pragma unroll
            for (int k8 = 0; k8 < NCH; ++k8) tqn[k8] = table_chunk<NCH, E>(til, k8, nch, Ddn, cn);
        }
        const T io0n = io[base + cn], io1n = io[base1 + cn];
        T p0n = T(0), p1n = T(0);
        if constexpr (MODE != 0) {
            p0n = keep_or_zero(p[base + cn], use_p);
            p1n = keep_or_zero(p[base1 + cn], use_p);
        }
        const uint64_t sdn = st_dn[cn];
        T a00, a01, a10, a11;
        down_gather_z2<T, NCH, E>(x0, x1, tq, nch, (unsigned)Ddn, a00, a01, a10, a11);
        {
            const T xv = x0[c];
            const T nd = static_cast<T>(__popcll(su0 & sdv));
            T q = io0 + t * (a00 + a01) + U * nd * xv;
            if (MODE != 0) {
                q *= sig;
                if (use_p) q -= cprev * p0;
            }
            io[base + c] = q;
            if (MODE != 0) {
                const double qd = q, xd = xv;
                s[0] += qd * xd;
                if constexpr (MODE == 2) {
                    const double pd = p0;
                    s[1] += qd * pd;
                    s[2] += xd * xd;
                    s[3] += xd * pd;
                    s[4] += pd * pd;
                }
            }
        }
        if (two) {
            const T xv = x1[c];
            const T nd = static_cast<T>(__popcll(su1 & sdv));
            T q = io1 + t * (a10 + a11) + U * nd * xv;
            if (MODE != 0) {
                q *= sig;
                if (use_p) q -= cprev * p1;
            }
            io[base1 + c] = q;
            if (MODE != 0) {
                const double qd = q, xd = xv;
                s[0] += qd * xd;
                if constexpr (MODE == 2) {
                    const double pd = p1;
                    s[1] += qd * pd;
                    s[2] += xd * xd;
                    s[3] += xd * pd;
                    s[4] += pd * pd;
                }
            }
        }
        io0 = io0n;
        io1 = io1n;
        p0 = p0n;
        p1 = p1n;
        sdv = sdn;
        ncwn = ncwn2;
#pragma unroll
        for (int k8 = 0; k8 < NCH; ++k8) tq[k8] = tqn[k8];
    }
}
}  // namespace ed
