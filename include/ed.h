/*
 * ed.h -- C ABI of the MI355X exact-diagonalisation library.
 *
 * Ground-state energies of two-species lattice models H = -t sum_<ij>,sigma
 * (c+_i,s c_j,s + h.c.) + U sum_i n_i,up n_i,dn  (Eq. 1 and the on-site term of
 * Sec. 1) by the Lanczos iteration (Alg. 1) over the fixed-(N_up, N_dn)
 * occupation-bitstring basis (Sec. 2.1), with H applied matrix-free as
 * H_up x I + I x H_dn + diag(U n_up n_dn)  (Eq. 3, 4, 5).
 *
 * Conventions shared by every call:
 *  - Return value: ED_OK (0), a positive informational code, or a negative
 *    error code.  Nothing throws across this boundary.  On error,
 *    ed_last_error() gives a text for the calling thread.
 *  - "host" pointers are CPU memory, "device" pointers are GPU memory on the
 *    current HIP device.  Every buffer is allocated and owned by the caller;
 *    the library keeps no state between calls and never frees a caller
 *    buffer.  Device calls are asynchronous on `stream` (a hipStream_t passed
 *    as void*, NULL = the default stream) unless stated otherwise.
 *  - Basis states are uint64 bitmasks, bit i = site i (N_s <= 64).  Per-spin
 *    states are in ascending integer order; a two-species state has index
 *    i_up * dim_dn + i_dn, i.e. a vector is dim_up subvectors of length
 *    dim_dn (Sec. 4, Eq. 4-5).
 *  - Fermion signs: operators ordered by site index within a species, all up
 *    operators before all down operators.  A hop i <- j in state s carries
 *    (-1)^(number of occupied sites strictly between i and j); the two
 *    species then decouple exactly as Eq. 3 states.
 */
#ifndef ED_H
#define ED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    ED_OK = 0,
    ED_BREAKDOWN = 1,      /* b_{j+1} vanished (Alg. 1 stop): T_j is exact on an invariant subspace */
    ED_NOT_CONVERGED = 2,  /* max_steps reached before the convergence test passed */
    ED_EINVAL = -1,        /* bad argument (null pointer, bad size, zero/non-finite start vector...) */
    ED_ECAPACITY = -2,     /* caller buffer too small; the needed size is returned where stated */
    ED_EOVERFLOW = -3,     /* sizes beyond what the representation holds (N_s > 64, dims > 2^31-1 ...) */
    ED_EDEVICE = -4        /* a HIP runtime error; text via ed_last_error() */
};

/* Vector storage and H.v arithmetic.  Scalars (dots, norms, a_j, b_j, T) are float64 in both. */
enum { ED_F64 = 0, ED_F32 = 1 };

/* Flattening order of an exported ELL table (Fig. 2): row-major as the paper's
 * CPU code, column-major as its GPU code. */
enum { ED_ROW_MAJOR = 0, ED_COL_MAJOR = 1 };

/* Text of the last error on this thread; valid until the next ed_* call on it. */
const char *ed_last_error(void);

/* Library version string (static storage). */
const char *ed_version(void);

/* ---- host: basis and hopping tables ------------------------------------ */

/* Per-spin basis (Sec. 2.1, Eq. 2): every n_part-subset of n_sites sites as a
 * bitmask, in ascending order; *dim = C(n_sites, n_part).
 * states: host, capacity `cap` entries; states == NULL with cap == 0 only
 * queries *dim.  cap < dim -> ED_ECAPACITY (with *dim set).  n_sites > 64 or
 * dim > 2^31-1 -> ED_EOVERFLOW.  0 <= n_part <= n_sites, else ED_EINVAL. */
int ed_build_basis(int n_sites, int n_part, uint64_t *states, int64_t cap, int64_t *dim);

/* Index of each state in the ascending per-spin basis, by its colex rank
 * sum_k C(p_k, k+1) over the set bits p_0 < p_1 < ...  states/ranks: host,
 * n entries.  A state with the wrong popcount or bits >= n_sites -> ED_EINVAL. */
int ed_state_rank(int n_sites, int n_part, const uint64_t *states, int64_t n, int64_t *ranks);

/* Per-spin hopping matrix H_sigma for t = 1 (Sec. 2.1), exported in ELL form
 * (Fig. 2): row r holds, in ascending column order, the columns and values
 * of its nonzeros, then zero padding (value 0, index 0) up to the width.
 * bonds: host, n_bonds pairs (i, j), 0 <= i, j < n_sites, i != j, unordered
 * duplicates rejected (ED_EINVAL).  states: host, the basis of ed_build_basis.
 * Values are -sign in {-1, +1}; t scales them at H.v time.
 * layout: ED_ROW_MAJOR (entry [r * width + k]) or ED_COL_MAJOR ([k * dim + r]).
 * cols/vals: host, cap_width * dim entries each; nnz: host, dim entries.
 * *width gets the ELL width (max nonzeros in a row); cap_width < width ->
 * ED_ECAPACITY with *width set and nothing else written.  Pass cols == vals ==
 * nnz == NULL with cap_width == 0 to query the width. */
int ed_build_hopping(int n_sites, const int32_t *bonds, int n_bonds, const uint64_t *states,
                     int64_t dim, int layout, int32_t cap_width, int32_t *cols, double *vals,
                     int32_t *nnz, int32_t *width);

/* Convert an exported ELL table into the device table format: uint16
 * entries e = (col << 1) | (val < 0) in ascending column order with padding
 * 0xFFFF after the last nonzero of a row; the row stride W8 is the width
 * rounded up to a multiple of 8 (whole 16-byte chunks).  The table is stored
 * twice, one layout after the other:
 *   [0, dim*W8):       row-major, entry k of row r at [r*W8 + k]
 *                      (read by the up-part kernel, one row per wavefront);
 *   [dim*W8, 2*dim*W8): 8-interleaved, entry k of row r at
 *                      [dim*W8 + ((k/8)*dim + r)*8 + k%8]
 *                      (read by the down-part kernel, one row per lane).
 * Input values must be exactly +-1 for k < nnz[r] (ED_EINVAL otherwise);
 * dim > 32767 -> ED_EOVERFLOW.  packed: host, 2 * dim * W8 entries.  Copy it
 * to 16-byte aligned device memory for ed_ham, whose w_up/w_dn are then W8. */
int ed_pack_tables(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                   int32_t width, int layout, uint16_t *packed);

/* The same table with uint32 entries e = (col << 1) | (val < 0) and padding
 * 0xFFFFFFFF, for per-spin dimensions above 32767: the 18-site half-filled
 * sector that Sec. 4 places beyond the memory of any coprocessor has 48620
 * states per species.  Identical layouts and stride W8, 32-byte chunks.
 * dim > 2^30 -> ED_EOVERFLOW.  packed: host, 2 * dim * W8 entries;
 * ed_ham.eb_up/eb_dn = 4 selects it. */
int ed_pack_tables32(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                     int32_t width, int layout, uint32_t *packed);

/* Complex hopping amplitudes (the paper's checkerboard lattice has complex
 * nearest-neighbour hoppings, Sec. 2.1 and its lattice figure): H_sigma =
 * sum over bonds (i, j) of a_ij c+_i c_j + conj(a_ij) c+_j c_i, t = 1 (t
 * scales at H.v time).  amps: host, n_bonds (re, im) pairs, a_ij for the
 * bond as given (i first).  Output as ed_build_hopping, with vals holding
 * (re, im) pairs: the element <row| H_sigma |col>, that is a_ij times the
 * fermion sign when the row state has the particle at i, conj(a_ij) times it
 * when at j.  With every a_ij = -1 this is ed_build_hopping.  vals: host,
 * 2 * cap_width * dim doubles.  Non-finite amplitudes -> ED_EINVAL. */
int ed_build_hopping_complex(int n_sites, const int32_t *bonds, int n_bonds, const double *amps,
                             const uint64_t *states, int64_t dim, int layout, int32_t cap_width, int32_t *cols,
                             double *vals, int32_t *nnz, int32_t *width);

/* Device table for complex values: uint32 entries e = (col << 6) | index of
 * the value in amps (distinct values numbered in first-seen order, row by
 * row), padding 0xFFFFFFFF; the two layouts and stride W8 of ed_pack_tables.
 * amps: host, 128 doubles (64 (re, im) pairs) written with the n_amps
 * distinct values; copy all 128 (the unused ones zero) to the device for
 * ed_ham.amp_up / amp_dn.  More than 64 distinct values or dim > 2^26 - 1
 * -> ED_EOVERFLOW.  packed: host, 2 * dim * W8 entries. */
int ed_pack_tables_complex(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim,
                           int32_t width, int layout, uint32_t *packed, double *amps, int32_t *n_amps);

/* Basis orders.  The basis of Sec. 2.1 is ascending (colex rank order), and
 * that is the order of every vector unless a species is reordered here.  Any
 * order of a species' basis gives the same H up to a permutation P of the
 * vector elements, and the Lanczos run started from P f_1 yields the same
 * a_j, b_j and E0 (up to rounding).  Tables and state arrays fix the order the
 * device calls see; only the calls that find a state by its colex rank (spin-
 * flip and bond moments) need the ascending order (see ed_ham.order).
 *
 * ed_hop_order: perm such that position q of the reordered basis holds state
 * perm[q] of the given one, sorted by hop count (nonzeros per row, nnz from
 * ed_build_hopping) from most to fewest, equal counts in their given order.
 * The down-part kernel gives a wavefront 64 consecutive columns and pays for
 * the table chunks of its widest column; in this order the columns of a
 * wavefront have nearly equal hop counts, so whole padding chunks drop out.
 * nnz: host, dim entries (>= 0); perm: host, dim entries. */
int ed_hop_order(const int32_t *nnz, int64_t dim, int64_t *perm);

/* ed_wave_chunks: for each group of 64 consecutive rows of an ELL table
 * (nnz from ed_build_hopping, in the basis order the device sees), the number
 * of 8-entry table chunks its widest row needs: out[g] = max over rows r in
 * [64g, min(64g + 64, dim)) of ceil(nnz[r] / 8).  The chunks from out[g] on
 * are padding for every row of the group (Fig. 2's ELL rows padded to the
 * widest).  nnz: host, dim entries (>= 0); out: host, ceil(dim / 64)
 * entries. */
int ed_wave_chunks(const int32_t *nnz, int64_t dim, uint32_t *out);

/* ed_band_order: perm (position q holds state perm[q]) that numbers each
 * state close to its hopping neighbours: reverse Cuthill-McKee on the graph
 * whose edges are the table's nonzeros (a breadth-first sweep from a
 * pseudo-peripheral state of fewest neighbours, each state's new neighbours
 * taken fewest-neighbours first, then lowest index; one sweep per connected
 * part; the whole order reversed).  The up-part kernel gathers, for a tile of
 * consecutive rows, the rows of x at their neighbours; in this order those
 * rows are fewer and closer together, so more of them are L2 hits.
 * cols, nnz, width, layout: one species' ELL table as from ed_build_hopping
 * (host); perm: host, dim entries.  nnz or a column out of range -> ED_EINVAL. */
int ed_band_order(const int32_t *cols, const int32_t *nnz, int64_t dim, int32_t width, int layout, int64_t *perm);

/* Neighbour windows of column blocks (for rows too long for LDS): for block
 * b of block_cols consecutive states [b*block_cols, min((b+1)*block_cols,
 * dim)), lo_hi[2b] and lo_hi[2b+1] bound every state of the block and every
 * table column of its states, lo rounded down and hi up to multiples of 4
 * (hi at most dim).  The down part can then stage x[r, lo..hi) of a row in
 * LDS for that block (Eq. 5 reads a row only at the block's neighbours); in a
 * band order (ed_band_order) the windows are narrow.  *max_window: the
 * largest hi - lo.  cols, nnz, width, layout: one species' ELL table as from
 * ed_build_hopping (host); block_cols > 0 and a multiple of 64; lo_hi: host,
 * 2 * ceil(dim / block_cols) entries.  A column out of range -> ED_EINVAL. */
int ed_row_windows(const int32_t *cols, const int32_t *nnz, int64_t dim, int32_t width, int layout,
                   int32_t block_cols, int32_t *lo_hi, int32_t *max_window);

/* The down part's table of a species with neighbour windows, columns
 * relative to their block's window: the layout of ed_pack_tables (stride =
 * width rounded up to 8; a row-major part, here all padding and unused, then
 * the 8-interleaved part) with 16-bit entries ((col - lo_b) << 1) |
 * negative, b = row / block_cols, padding 0xFFFF.  Windows of up to 32,767
 * states thus take 16-bit entries at any species size.  cols, vals, nnz,
 * width, layout: the species' ELL table (host, values +-1); lo_hi: its
 * ed_row_windows output for block_cols; packed: host, 2 * stride * dim
 * entries.  A window wider than 32,767 or not holding a row or its columns
 * -> ED_EINVAL. */
int ed_pack_tables_windowed(const int32_t *cols, const double *vals, const int32_t *nnz, int64_t dim, int32_t width,
                            int layout, int32_t block_cols, const int32_t *lo_hi, uint16_t *packed);

/* Reorder one species' basis and its exported ELL table (Fig. 2 format, as
 * from ed_build_hopping or ed_build_hopping_complex): position q of the
 * output is state perm[q] of the input, and each row's columns are renumbered
 * into the new order and sorted ascending again (padding as in the input
 * format).  n_vals: 1 (real values) or 2 ((re, im) pairs).  All pointers
 * host; outputs have the input's sizes and must not overlap the inputs.  The
 * result packs with ed_pack_tables / ed_pack_tables32 / ed_pack_tables_complex.
 * perm not a permutation of [0, dim), nnz or a column out of range ->
 * ED_EINVAL (outputs then undefined). */
int ed_permute_basis(const uint64_t *states, const int32_t *cols, const double *vals, const int32_t *nnz,
                     int64_t dim, int32_t width, int layout, int32_t n_vals, const int64_t *perm,
                     uint64_t *states_out, int32_t *cols_out, double *vals_out, int32_t *nnz_out);

/* Lowest eigenvalue of the m-by-m symmetric tridiagonal T (Sec. 2.2) with
 * diagonal a[0..m-1] = a_1..a_m and off-diagonal b[0..m-2] = b_2..b_m, by
 * Sturm-sequence bisection in float64 to full precision.  host pointers. */
int ed_tridiag_lowest(const double *a, const double *b, int m, double *e0);

/* Lowest eigenvector y (unit norm, y[0] >= 0 unless it vanishes) of the same
 * T, by inverse iteration at the bisection eigenvalue.  y: host, m entries. */
int ed_tridiag_lowest_vector(const double *a, const double *b, int m, double *e0, double *y);

/* ---- device: the Hamiltonian and H.v ----------------------------------- */

/* One instance (lattice, fillings, t, U).  All pointers are device memory.
 * tab_up/tab_dn: ed_pack_tables (eb = 2, or 0) or ed_pack_tables32 (eb = 4)
 * output for H_up and H_dn, with row strides w_up/w_dn (multiples of 8; 0
 * when a species cannot hop); the two species may use different formats.
 * st_up/st_dn: the per-spin bases (for the U term).  dtype: ED_F64 or ED_F32
 * (vectors and H.v).  tile: 0 = default launch configuration, else an id
 * returned by ed_tune.  A species with 16-bit tables has dim <= 32767, one
 * with 32-bit tables dim <= 2^30 (ED_EOVERFLOW otherwise); eb other than 0,
 * 2, 4 -> ED_EINVAL.  The batched launch takes 16-bit tables only.
 * cplx = 1: complex amplitudes.  Both tables come from
 * ed_pack_tables_complex (eb = 4), amp_up/amp_dn are device arrays of 64
 * complex values (128 doubles, interleaved re, im) from it, and every vector
 * of the device calls holds dim_up*dim_dn complex numbers as interleaved
 * (re, im) pairs of dtype (so 2*dim_up*dim_dn reals).  a_j and b_j stay real
 * (H is Hermitian; a_j = Re f_j^dagger q).  Complex instances are accepted by
 * ed_hv, the Lanczos calls, ed_ground_state (gauge_index = -1 only) and
 * ed_tune; the batch, the start-vector network and the observables return
 * ED_EINVAL for them.  cplx = 0: amp_up/amp_dn are ignored.
 * order: 0 when both bases are ascending (ed_build_basis); set bit 0 / bit 1
 * when the up / down tables and states come from ed_permute_basis.  Every
 * call accepts reordered bases (tables and state arrays fix the order) except
 * ed_spin_flip_moments and ed_bond_moments, which find states by colex rank
 * and return ED_EINVAL unless order = 0; other values -> ED_EINVAL.
 * win_dn: NULL, or the down species' neighbour windows from ed_row_windows
 * (device, 2 * ceil(dim_dn / win_cols) int32) for blocks of win_cols states,
 * the largest win_max; the autotuner may then give rows too long for LDS a
 * down-part kernel that stages each block's window (real instances).  The
 * windows must hold every block's table columns (they come from this
 * species' table): a block whose pair is wider than win_max or does not
 * cover the block is gathered from global memory instead.  win_tab: NULL,
 * or the down table in the window-relative 16-bit form of
 * ed_pack_tables_windowed (device, with win_dn), which that kernel then
 * reads instead of tab_dn.
 * wch_dn: NULL, or the down table's chunk count per 64 consecutive states
 * from ed_wave_chunks (device, ceil(dim_dn / 64) uint32).  These down-part
 * kernels then read only those chunks of each wavefront's 64 columns: the
 * one- and two-row kernels that stage rows in LDS (tables of 3 or 4 chunks),
 * the windowed one on win_tab, and the one that gathers from global memory
 * for a species alone (w_up = 0, rows too long for LDS; in FP64 on 32-bit
 * tables of more than 4 chunks it reads every chunk, which measured faster
 * there).  Counts above w_dn / 8 are taken as w_dn / 8.  The results are the same bits as without it; a count below a
 * column's true chunk count drops that column's later hops. */
typedef struct ed_ham {
    int64_t dim_up, dim_dn;
    int32_t w_up, w_dn;
    const void *tab_up, *tab_dn;
    const uint64_t *st_up, *st_dn;
    double t, U;
    int32_t dtype;
    int32_t tile;
    int32_t eb_up, eb_dn;   /* bytes per table entry of each species */
    int32_t cplx;           /* 0: real hopping, 1: complex amplitudes and vectors */
    int32_t order;          /* bit 0 / bit 1: the up / down basis is not ascending (ed_permute_basis) */
    const double *amp_up, *amp_dn;
    const int32_t *win_dn;
    int32_t win_cols, win_max;
    const uint16_t *win_tab;
    const uint32_t *wch_dn;
} ed_ham;

/* Bytes of device workspace (`ws` below) the calls on this instance need
 * for runs of up to max_steps Lanczos steps.  Pass a 256-byte aligned buffer;
 * its contents are scratch between calls. */
int ed_workspace_size(const ed_ham *h, int32_t max_steps, int64_t *bytes);

/* y = H x (Eq. 3-5 plus the diagonal U term).  x, y: device, dim_up*dim_dn
 * elements of h->dtype, distinct buffers.  ws: device workspace of
 * ed_workspace_size(h, 0) bytes (work-queue counters of the up-part kernel). */
int ed_hv(const ed_ham *h, const void *x, void *y, void *ws, void *stream);

/* A vector in another basis order: y[p, q] = x[perm_up[p], perm_dn[q]] over
 * the dim_up x dim_dn element grid (Eq. 3), each element dtype (a (re, im)
 * pair when cplx = 1).  With perm the ed_hop_order output of a species, this
 * takes an ascending-order vector into the reordered one; its inverse
 * (inv[perm[q]] = q) takes it back.  perm_up / perm_dn: device int64 arrays of
 * dim_up / dim_dn entries, or NULL for the identity.  An entry outside its
 * range makes the affected elements NaN.  x, y: device, must not overlap
 * (ED_EINVAL).  Only dims, dtype and cplx of h are used; asynchronous on
 * `stream`. */
int ed_permute_vector(const ed_ham *h, const int64_t *perm_up, const int64_t *perm_dn, const void *x, void *y,
                      void *stream);

/* Launch-configuration autotuner (the paper tuned its CPU blocking and GPU
 * block size by experiment, Sec. 4-5; this searches the kernels' tiles).
 * Times every candidate tile of the up-part kernel (stripe width, rows per
 * tile, workgroup-to-XCD mapping) and of the down-part kernel (workgroup size,
 * rows per workgroup) on y = H x with h's sizes, `reps` timed launches each
 * after one warm-up, and returns in *tile the id of the fastest combination,
 * to be stored in ed_ham.tile.  The down-part kernel is timed as in a
 * Lanczos step, each timed launch after an untimed up part.  x, y: as for
 * ed_hv (y is overwritten); p: device vector of the same size standing in
 * for f_{j-1} (read only; not y), or NULL to let x stand in (its reads then
 * hit in cache and the down-part times come out short); ws: device
 * workspace of ed_workspace_size(h, 2) bytes.  For complex instances the
 * up-part kernel takes only the rows per tile and the down-part kernel only
 * the workgroup size (one row per workgroup), so one candidate per distinct
 * value is timed.
 * ms_up (n_up doubles) / ms_dn (n_dn doubles), may be NULL: average ms per
 * candidate index, -1 where a candidate does not apply or repeats an earlier
 * launch (see ed_tile_count).
 * Synchronises `stream`. */
int ed_tune(const ed_ham *h, const void *x, void *y, const void *p, void *ws, void *stream, int32_t reps,
            int32_t *tile, double *ms_up, double *ms_dn);

/* Number of up-part and down-part tile candidates; a tile id is
 * up_index | (down_index << 8), index 0 = built-in default. */
int ed_tile_count(int32_t *n_up, int32_t *n_dn);

/* The launch parameters a tile id resolves to for instance h: params[0..6] =
 * stripe width, rows per up tile, up workgroup size, up mapping (0 XCD
 * round-robin, 1 linear, 2 per-XCD work queues), down workgroup size, rows
 * per down workgroup, and the down kernel's form: 0 rows (or column blocks
 * of long rows) per workgroup, 1 two rows per workgroup that share each
 * table chunk (both in LDS), 2 column blocks of long rows with their
 * neighbour windows in LDS (ed_ham.win_dn).  params: host, 7 ints. */
int ed_tile_params(int32_t tile, const ed_ham *h, int32_t *params);

/* ---- device: the Lanczos iteration (Alg. 1) ---------------------------- */

/* Lanczos state.  f_prev, f_cur, f_next: device vectors (h->dtype, dim
 * elements, distinct); a: device, >= max_steps doubles (a[j-1] = a_j);
 * b: device, >= max_steps + 1 doubles (b[j-1] = b_j, b[0] = b_1 = 0).
 * j: steps launched so far (host side).  The library rotates the three
 * vector pointers after every step, so f_cur always holds the newest vector.
 * Vectors are stored unnormalised: after j steps f_cur = b_{j+1} f_{j+1}
 * (that is Alg. 1's q_j after its line 6), and right after init f_cur is a
 * copy of f1, i.e. |f1| f_1; the kernels apply the scale on the fly, which is
 * what lets b_{j+1} be the norm of the stored vector itself. */
typedef struct ed_lanczos {
    void *f_prev, *f_cur, *f_next;
    double *a, *b;
    int32_t j;
    int32_t max_steps;
} ed_lanczos;

/* Start the iteration (Alg. 1 requires a start vector of norm 1): f_cur =
 * f1 / |f1| with the norm accumulated in float64, b_1 = 0, j = 0.
 * f1: device, h->dtype, dim elements (it may alias f_prev or f_next, not
 * f_cur).  Synchronises `stream`; a zero or non-finite norm -> ED_EINVAL. */
int ed_lanczos_init(const ed_ham *h, ed_lanczos *st, const void *f1, void *ws, void *stream);

/* One iteration of Alg. 1, asynchronous:
 *   q = H f_j - b_j f_{j-1};  a_j = q.f_j;  q -= a_j f_j;  b_{j+1} = |q|;
 *   f_{j+1} = q / b_{j+1}  (the division is deferred, see ed_lanczos).
 * ED_F64 follows that order in float64.  ED_F32 stores vectors in float32
 * and adds local re-orthogonalisation: q is projected off both f_j and
 * f_{j-1} with float64 coefficients from their Gram matrix, the f_j
 * coefficient is a_j and b_{j+1} is the norm of the projected q.
 * All scalars stay on the device.  A vanishing b_{j+1} (<= 64 eps max|a|,b,
 * eps = 2^-52 or 2^-24) or j == max_steps freezes the state: further steps are
 * no-ops.  ed_lanczos_read reports it. */
int ed_lanczos_step(const ed_ham *h, ed_lanczos *st, void *ws, void *stream);

/* ed_lanczos_step with a HIP event recorded before each of its five kernels
 * and after the last: ms[0..4] = durations in milliseconds of the up-part
 * kernel (Eq. 4), the down-part/diagonal/recurrence kernel (Eq. 5 and Alg. 1
 * line 4, with the partial dot products), the a_j reduction (line 5), the
 * vector update with its partial norms (line 6) and the b_{j+1} reduction
 * (lines 7-8).  Synchronises on the last event.  ms: host, 5 doubles. */
int ed_lanczos_step_timed(const ed_ham *h, ed_lanczos *st, void *ws, void *stream, double *ms);

/* Synchronise `stream` and report the device-side state: *steps = number of
 * completed steps j, *status = ED_OK (running), ED_BREAKDOWN or
 * ED_NOT_CONVERGED (max_steps reached).  a_host (steps doubles) and b_host
 * (steps + 1 doubles, b_host[0] = b_1 = 0) may be NULL. */
int ed_lanczos_read(const ed_ham *h, const ed_lanczos *st, void *ws, void *stream, int32_t *steps,
                    int32_t *status, double *a_host, double *b_host);

/* The whole ground-state-energy run: init from f1, then Alg. 1 steps (launched
 * `check_every` at a time from a captured HIP graph) until
 *   tol > 0: |E0(j) - E0(j-1)| < tol at two consecutive j, where E0(j) is the
 *            lowest eigenvalue of T_j (Sec. 2.2, host bisection), or
 *   tol <= 0: exactly st->max_steps steps (the paper's fixed-m protocol),
 * or a breakdown.  Synchronises.  *e0 = E0 at the stopping step, *steps = j.
 * a_host/b_host as in ed_lanczos_read (may be NULL).  Returns ED_OK,
 * ED_BREAKDOWN (E0 exact on the invariant subspace) or ED_NOT_CONVERGED. */
int ed_ground_energy(const ed_ham *h, ed_lanczos *st, const void *f1, double tol,
                     int32_t check_every, void *ws, void *stream, double *e0, int32_t *steps,
                     double *a_host, double *b_host);

/* ed_ground_energy for callers that cannot allocate (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): the same run and
 * the same results, with no workspace argument, no captured graph and no
 * stream of its own.  The run's workspace (header, partial sums, queue
 * counters) is a 4 MiB array in device memory that the library holds on
 * every GPU it runs on until the process ends; runs needing more than that
 * (ed_workspace_size above 4 MiB: roughly dim_up + 2048 above 45,000 at
 * max_steps 2048), or max_steps above 2048, return ED_ECAPACITY and launch
 * nothing.  Steps are launched on `stream` `check_every` at a time.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU race,
 * whatever their streams.  Other arguments, results and errors as
 * ed_ground_energy. */
int ed_ground_energy_noalloc(const ed_ham *h, ed_lanczos *st, const void *f1, double tol, int32_t check_every,
                             void *stream, double *e0, int32_t *steps, double *a_host, double *b_host);

/* Ground-state vector by two passes: pass 1 runs m steps from f1 (as
 * ed_ground_energy with tol <= 0) or, with tol > 0, the steps until
 * |E0(j) - E0(j-1)| < tol at two consecutive j (ed_ground_energy's rule)
 * plus `extra` (>= 0) more, at most m; the lowest eigenvector y of T_m (m
 * the pass's step count) is found on the host, pass 2 replays the identical
 * steps and accumulates v = sum_k y_k f_k, then v is normalised (float64
 * norm).  A run to a tolerance therefore needs no separate ed_ground_energy
 * call to fix m.  v: device, h->dtype,
 * dim elements, distinct from the three Lanczos vectors.  gauge_index >= 0
 * fixes the arbitrary global sign: v[gauge_index] >= 0 afterwards, or, when
 * |v[gauge_index]| is below 1e-3 of max |v_i| (its sign then carries no
 * information), the largest-magnitude element (the lowest index among equal
 * magnitudes) is made positive instead; -1: no gauge.  ws must hold
 * ed_workspace_size(h, m).  *e0 = lowest eigenvalue of T_m, *steps = the
 * pass's step count (fewer than asked on breakdown).  m outside
 * [1, st->max_steps] or extra < 0 -> ED_EINVAL. */
int ed_ground_state(const ed_ham *h, ed_lanczos *st, const void *f1, int32_t m, double tol, int32_t extra,
                    int64_t gauge_index, void *v, void *ws, void *stream, double *e0, int32_t *steps);

/* ---- device: batched ground-state runs --------------------------------- */

/* One instance of a batch: its Hamiltonian (dtype must be ED_F32: float32
 * vectors and H.v, float64 scalars), its start vector f1 (device, dim
 * floats, any nonzero norm), three device work vectors of dim floats, and
 * device arrays a (max_steps doubles) and b (max_steps + 1 doubles) that
 * receive its Lanczos coefficients.  Tables may be shared between items. */
typedef struct ed_batch_item {
    ed_ham h;
    const void *f1;
    void *vec[3];
    double *a, *b;
} ed_batch_item;

/* Device workspace bytes for ed_ground_energy_batch on these items with
 * this solo_dim. */
int ed_batch_workspace_size(const ed_batch_item *items, int32_t n, int32_t max_steps, int64_t solo_dim,
                            int64_t *bytes);

/* Run n independent Lanczos ground-state computations (Alg. 1 with the mixed
 * form of ed_lanczos_step).  The items below solo_dim states (all of them
 * when solo_dim <= 0) run in ONE persistent cooperative kernel launch, which
 * is captured in a HIP graph when use_graph != 0 and the runtime accepts the
 * capture (*graph_used reports it; otherwise the kernel is launched
 * directly).  The instances may differ in U, t and fillings (uneven
 * dimensions).  Each instance stops on its own when |E0(j) - E0(j-1)| < tol
 * at two consecutive steps, E0(j) being the lowest eigenvalue of T_j found
 * on the device by Sturm-count multisection; or on breakdown; or at
 * max_steps.  Launch tiles follow each item's h.tile (see ed_tune).  Items
 * of at least solo_dim states (solo_dim > 0) then run one after another on
 * `stream` through ed_ground_energy (the same stopping rule, checked every 9
 * steps on the host, steps launched from a captured graph): one step of such
 * an instance fills the GPU by itself, and its tuned one-instance kernels
 * beat the persistent kernel's shared tiles.
 * Per item (host arrays of n): e0 = lowest eigenvalue of T at the stopping
 * step (host bisection of the returned coefficients), steps, status (ED_OK =
 * converged, ED_BREAKDOWN, ED_NOT_CONVERGED); e0_device (may be NULL) = the
 * device's value at that step (for an item run on its own, the host value).
 * phase_ms (6 doubles, may be NULL): time the persistent launch spent in the
 * phases start-up, up part, down part, a_j, update, b_j (summed over the
 * steps, barrier waits included; zero without one).  ws:
 * ed_batch_workspace_size bytes for the same solo_dim, 256-byte aligned.
 * Synchronises `stream`.  Returns ED_NOT_CONVERGED if any item did not
 * converge.  Limits (every item): per-spin dims <= 32767, rows (dim_dn) of
 * at most 8192 floats, table strides <= 32 (both species), both species
 * must hop. */
int ed_ground_energy_batch(const ed_batch_item *items, int32_t n, int32_t max_steps, double tol, int64_t solo_dim,
                           void *ws, int64_t ws_bytes, void *stream, int32_t use_graph, double *e0, int32_t *steps,
                           int32_t *status, double *e0_device, int32_t *graph_used, double *phase_ms);

/* ---- device: observables of a state -------------------------------------- */

/* Occupation moments of a state psi, e.g. the ground-state vector of
 * ed_ground_state: G[a][b] = sum_x |psi_x|^2 n_a(x) n_b(x) / sum_x |psi_x|^2
 * over the 2*n_sites occupation numbers, a = i for n_i,up and a = n_sites + i
 * for n_i,dn.  The basis states of Sec. 2.1 fix every occupation number, so
 * all diagonal observables (double occupancy, density and spin correlations)
 * follow from G; see ed_occupation_correlations.  Two passes over psi, float64
 * sums in a fixed order.
 * psi: device, dim_up*dim_dn elements of h->dtype, any nonzero norm (a zero
 * vector gives G = 0).  n_sites: 1..32, the number of lattice sites (the bits
 * of the per-spin states; higher bits are ignored).  ws: device, 256-byte
 * aligned, ws_bytes >= ed_occupation_moments_ws(h, n_sites).  g: host,
 * (2*n_sites)^2 doubles, row-major.  Synchronises stream. */
int ed_occupation_moments_ws(const ed_ham *h, int32_t n_sites, int64_t *bytes);
int ed_occupation_moments(const ed_ham *h, int32_t n_sites, const void *psi, void *ws, int64_t ws_bytes,
                          void *stream, double *g);

/* Diagonal observables from G (ed_occupation_moments): double occupancy
 * docc[i] = <n_i,up n_i,dn>, density correlations nn[i*n_sites+j] = <n_i n_j>
 * with n = n_up + n_dn, spin correlations szsz[i*n_sites+j] = <S^z_i S^z_j>
 * with S^z = (n_up - n_dn)/2.  host; each output may be NULL. */
int ed_occupation_correlations(const double *g, int32_t n_sites, double *docc, double *nn, double *szsz);

/* Spin-flip moments of a state: c[i * n_sites + j] = <S+_i S-_j> / <psi|psi>
 * with S+_i = c+_i,up c_i,dn and S-_j = c+_j,dn c_j,up: an up particle moves
 * j -> i and a down particle i -> j, both staying in the sector; the
 * diagonal is <n_i,up (1 - n_i,dn)>.  With the occupation moments they give
 * the full spin correlation <S_i . S_j> (ed_spin_correlations); the
 * observable of the ground state, which the paper's Lanczos vector gives
 * (Sec. 2.2).  psi: device, dim_up*dim_dn real values of h->dtype; ws:
 * device, ed_spin_flip_moments_ws bytes, 256-byte aligned; c: host, n_sites^2
 * doubles.  One pass over psi per site i, with the target of each hop found
 * by its colex rank; sums in float64 in a fixed order.  Synchronises
 * `stream`.  n_sites outside 1..32 or complex amplitudes -> ED_EINVAL. */
int ed_spin_flip_moments_ws(const ed_ham *h, int32_t n_sites, int64_t *bytes);
int ed_spin_flip_moments(const ed_ham *h, int32_t n_sites, const void *psi, void *ws, int64_t ws_bytes,
                         void *stream, double *c);

/* <S_i . S_j> (host, n_sites^2 doubles) from the normalised occupation
 * moments g (ed_occupation_moments) and spin-flip moments c: <S^z_i S^z_j> +
 * (c[i][j] + c[j][i]) / 2 off the diagonal, and <S_i^2> = (3/4) <(n_i,up -
 * n_i,dn)^2> on it.  All host pointers. */
int ed_spin_correlations(const double *g, const double *c, int32_t n_sites, double *ss);

/* Bond moments of a state: k[2 * b + sigma] = <c+_i,sigma c_j,sigma + c+_j,sigma
 * c_i,sigma> / <psi|psi> for bond b = (i, j) of `bonds` (host, n_bonds
 * pairs, 0 <= i, j < n_sites, i != j) and species sigma (0 up, 1 down).  The
 * hopping energy is -t times their sum (Eq. 1), so <H> = -t sum k + U sum_i
 * <n_i,up n_i,dn>.  psi: device, real values of h->dtype; ws: device,
 * ed_bond_moments_ws bytes, 256-byte aligned; k: host, 2 * n_bonds doubles.
 * One pass over psi per 16 bonds; sums in float64 in a fixed order.
 * Synchronises `stream`.  Bad bonds, n_sites outside 1..32 or complex
 * amplitudes -> ED_EINVAL. */
int ed_bond_moments_ws(const ed_ham *h, int32_t n_sites, int32_t n_bonds, int64_t *bytes);
int ed_bond_moments(const ed_ham *h, int32_t n_sites, const int32_t *bonds, int32_t n_bonds, const void *psi,
                    void *ws, int64_t ws_bytes, void *stream, double *k);

/* ---- device: the start-vector network ---------------------------------- */

/* psi(bits): 32 inputs (bits 0..15 of the up state, then of the down state,
 * as +-1) -> 128 -> 128 -> 128 (ReLU) -> 1.  It proposes the Lanczos start
 * vector (Alg. 1 requires only a vector of norm 1).  Parameters: one float32
 * array of ED_MLP_NPARAM values, W1[128x32] b1[128] W2[128x128] b2 W3[128x128]
 * b3 W4[1x128] b4, each W row-major [out][in].  Every matrix product runs on
 * bfloat16 matrix cores (operands rounded to nearest even), accumulating in
 * float32.  Minibatch calls keep their activations in `ws`
 * (ed_mlp_workspace_size bytes for n samples, 256-byte aligned). */
#define ED_MLP_NPARAM 37377
int ed_mlp_workspace_size(int64_t n, int64_t *bytes);

/* Forward pass on n samples; sample k is the state (st_up[idx[2k]],
 * st_dn[idx[2k+1]]).  out: device, n floats (may be NULL).  All device
 * pointers; the activations stay in ws for ed_mlp_backward. */
int ed_mlp_forward(const float *params, const uint64_t *st_up, const uint64_t *st_dn, const int32_t *idx,
                   int64_t n, float *out, void *ws, void *stream);

/* Gradient of the mean squared error (1/n) sum_k (psi_k - target_k)^2 of
 * the last ed_mlp_forward on ws: grad (device, ED_MLP_NPARAM floats) is
 * overwritten; loss (device double, may be NULL) receives the loss. */
int ed_mlp_backward(const float *params, const float *target, int64_t n, float *grad, double *loss, void *ws,
                    void *stream);

/* One Adam step (bias-corrected, step >= 1) on the float32 parameters with
 * moments m, v (device, ED_MLP_NPARAM floats each, zero before step 1). */
int ed_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, float beta1,
                float beta2, float eps, void *stream);

/* psi over every state of instance h: f1[i_up * dim_dn + i_dn] (h->dtype). */
int ed_mlp_start_vector(const float *params, const ed_ham *h, void *f1, void *stream);

/* Row distribution of a vector psi of instance h for ed_mlp_sample:
 * cdf[r] = (sum_{r' <= r} sum_c psi[r', c]^2) / |psi|^2 (float64).  cdf: device,
 * dim_up + 1 doubles (the last receives |psi|^2). */
int ed_mlp_row_cdf(const void *psi, const ed_ham *h, double *cdf, void *stream);

/* Draw n training samples from a ground-state vector psi of h: with
 * uniforms[2k] < 1/2 the state is drawn with probability |psi|^2 (the row
 * through row_cdf from ed_mlp_row_cdf, then the column inside the row),
 * otherwise uniformly;
 * uniforms[2k+1] is the position.  idx: device, 2n ints (i_up, i_dn);
 * target: device, n floats = sqrt(dim) psi[state]. */
int ed_mlp_sample(const void *psi, const ed_ham *h, const double *row_cdf, const double *uniforms, int32_t n,
                  int32_t *idx, float *target, void *stream);

#ifdef __cplusplus
}
#endif
#endif
