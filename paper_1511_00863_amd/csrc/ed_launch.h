// Host-side launch helpers shared by the device translation units: tile
// tables and their resolution, argument checks, HIP error mapping.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/ed.h"
#include "ed_internal.h"

namespace ed {

struct Tile {
    int up_wlog2;   // stripe width = 2^up_wlog2 columns (16..256; 128/256 = 2/4 columns per lane)
    int up_rc;      // rows per k_up tile
    int up_block;   // k_up threads per workgroup
    int up_map;     // 0 XCD round-robin remap, 1 linear, 2 per-XCD queues
    int dn_block;   // k_down threads per workgroup
    int dn_rpb;     // rows per k_down workgroup (0 = derive from LDS and block)
    int dn_pair;    // 1: two rows per workgroup sharing each table chunk (k_down2), where both fit LDS
    int dn_win;     // 1: rows too long for LDS by column blocks with their neighbour windows (k_down_win)
};

struct UpTile { int wlog2, rc, block, map; };
struct DnTile { int block, rpb, pair, win; };

// Candidates searched by ed_tune.  A tile id is up_index | (dn_index << 8);
// index 0 means "heuristic default" for that kernel.
static const UpTile kUpTiles[] = {
    {0, 0, 0, 0},
    {6, 16, 256, 0}, {5, 16, 256, 0}, {4, 16, 256, 0},
    {6, 32, 256, 0}, {5, 32, 256, 0}, {4, 32, 256, 0},
    {6, 64, 256, 0}, {5, 64, 256, 0}, {4, 64, 256, 0},
    {6, 128, 256, 0}, {5, 128, 256, 0}, {4, 128, 256, 0},
    {6, 256, 256, 0}, {5, 256, 256, 0}, {4, 256, 256, 0},
    {6, 32, 256, 1}, {5, 32, 256, 1}, {4, 32, 256, 1},
    {6, 128, 256, 1}, {5, 128, 256, 1}, {4, 128, 256, 1},
    {6, 32, 256, 2}, {5, 32, 256, 2}, {4, 32, 256, 2},
    {6, 128, 256, 2}, {5, 128, 256, 2}, {4, 128, 256, 2},
    {6, 64, 512, 0}, {5, 64, 512, 0}, {6, 128, 512, 0}, {5, 128, 512, 0},
    {7, 16, 256, 0}, {7, 32, 256, 0}, {7, 64, 256, 0}, {7, 128, 256, 0}, {7, 64, 512, 0},
    {7, 8, 256, 0}, {7, 16, 512, 0}, {8, 8, 256, 0}, {8, 16, 256, 0}, {8, 32, 256, 0}, {8, 16, 512, 0},
};
static const DnTile kDnTiles[] = {
    {0, 0, 0, 0},    {1024, 0, 0, 0}, {512, 0, 0, 0}, {256, 0, 0, 0}, {1024, 1, 0, 0}, {512, 1, 0, 0},
    {256, 1, 0, 0},  {1024, 2, 0, 0}, {512, 2, 0, 0}, {256, 4, 0, 0}, {1024, 2, 1, 0}, {512, 2, 1, 0},
    {256, 2, 1, 0},  {1024, 0, 0, 1}, {512, 0, 0, 1}, {256, 0, 0, 1},
};
constexpr int kNumUp = sizeof(kUpTiles) / sizeof(kUpTiles[0]);
constexpr int kNumDn = sizeof(kDnTiles) / sizeof(kDnTiles[0]);
constexpr int kLdsBudget = 152 * 1024;
constexpr int kMaxWideDim = 1 << 30;   // per-spin dimension limit of the 32-bit table format
constexpr int kComplexMaxDim = (1 << 26) - 1;   // columns of a complex table entry: 26 bits
constexpr int kAmpSlots = 64;                    // complex amplitude values per species (6-bit index)
constexpr int kDownBlocks = 2048;      // workgroups a k_down launch of long rows is split into, at least

static inline int elem_size(const ed_ham *h) { return h->dtype == ED_F64 ? 8 : 4; }

// 32-bit table entries (ed_pack_tables32) for a species; 16-bit otherwise
static inline bool wide_up(const ed_ham *h) { return h->eb_up == 4; }
static inline bool wide_dn(const ed_ham *h) { return h->eb_dn == 4; }

static inline Tile resolve_tile_id(const ed_ham *h, int id) {
    const int ui = id & 0xFF, di = (id >> 8) & 0xFF;
    const int es = elem_size(h);
    Tile t;
    if (ui > 0 && ui < kNumUp) {
        t.up_wlog2 = kUpTiles[ui].wlog2;
        t.up_rc = kUpTiles[ui].rc;
        t.up_block = kUpTiles[ui].block;
        t.up_map = kUpTiles[ui].map;
    } else {   // two columns per lane on 128-column stripes, 16-row tiles (falls back below)
        t.up_wlog2 = 7;
        t.up_rc = 16;
        t.up_block = 256;
        t.up_map = 0;
    }
    if (di > 0 && di < kNumDn) {
        t.dn_block = kDnTiles[di].block;
        t.dn_rpb = kDnTiles[di].rpb;
        t.dn_pair = kDnTiles[di].pair;
        t.dn_win = kDnTiles[di].win;
    } else {
        t.dn_block = h->dim_dn >= 1024 ? 1024 : 256;
        t.dn_rpb = 0;
        t.dn_pair = 0;
        t.dn_win = 0;
    }
    if (wide_dn(h)) t.dn_block = std::min(t.dn_block, 512);   // the 32-bit table variants' launch bound
    // V = 2 or 4 columns per lane need row starts aligned to V elements (a row
    // length that is a multiple of V) and at most 4 table chunks; 4 columns
    // per lane is float only (16-byte loads)
    if (t.up_wlog2 == 8 && (es != 4 || (h->dim_dn & 3) || h->w_up > 32 || wide_up(h))) t.up_wlog2 = 7;
    if (t.up_wlog2 == 7 && ((h->dim_dn & 1) || h->w_up > 32)) t.up_wlog2 = 6;
    // stripes much wider than the row are pointless
    while (t.up_wlog2 > 4 && (1 << (t.up_wlog2 - 1)) >= h->dim_dn) --t.up_wlog2;
    if (t.up_wlog2 < 4) t.up_wlog2 = 4;
    const int64_t row_bytes = h->dim_dn * es;
    if (t.dn_rpb == 0) {
        int64_t by_lds = std::max<int64_t>(1, kLdsBudget / row_bytes);
        int64_t by_fill = std::max<int64_t>(1, (2 * t.dn_block + h->dim_dn - 1) / h->dim_dn);
        t.dn_rpb = (int)std::min<int64_t>(std::min(by_lds, by_fill), h->dim_up);
    }
    t.dn_rpb = (int)std::max<int64_t>(1, std::min<int64_t>(t.dn_rpb, h->dim_up));
    return t;
}

static inline Tile resolve_tile(const ed_ham *h) { return resolve_tile_id(h, h->tile); }

static inline bool valid_tile_id(int id) {
    return id >= 0 && (id & 0xFF) < kNumUp && ((id >> 8) & 0xFF) < kNumDn && (id >> 16) == 0;
}

static inline int check_ham(const ed_ham *h, const char *who) {
    if (!h) return set_error(ED_EINVAL, "%s: ham is NULL", who);
    if (h->dim_up < 1 || h->dim_dn < 1) return set_error(ED_EINVAL, "%s: bad dims", who);
    if ((h->eb_up != 0 && h->eb_up != 2 && h->eb_up != 4) || (h->eb_dn != 0 && h->eb_dn != 2 && h->eb_dn != 4))
        return set_error(ED_EINVAL, "%s: table entry bytes must be 0, 2 or 4", who);
    if ((!wide_up(h) && h->dim_up > 32767) || (!wide_dn(h) && h->dim_dn > 32767))
        return set_error(ED_EOVERFLOW, "%s: per-spin dims above 32767 need 32-bit tables", who);
    if (h->dim_up > kMaxWideDim || h->dim_dn > kMaxWideDim)
        return set_error(ED_EOVERFLOW, "%s: per-spin dims must be <= %d", who, kMaxWideDim);
    if (h->w_up < 0 || h->w_dn < 0 || (h->w_up && !h->tab_up) || (h->w_dn && !h->tab_dn) || !h->st_up ||
        !h->st_dn)
        return set_error(ED_EINVAL, "%s: missing tables or states", who);
    if ((h->w_up & 7) || (h->w_dn & 7)) return set_error(ED_EINVAL, "%s: table strides must be multiples of 8", who);
    if (h->w_up > 64 || h->w_dn > 64) return set_error(ED_EOVERFLOW, "%s: table strides above 64 unsupported", who);
    if (h->dtype != ED_F64 && h->dtype != ED_F32) return set_error(ED_EINVAL, "%s: bad dtype %d", who, h->dtype);
    if (h->cplx != 0 && h->cplx != 1) return set_error(ED_EINVAL, "%s: cplx must be 0 or 1", who);
    if (h->order < 0 || h->order > 3) return set_error(ED_EINVAL, "%s: order must be 0..3", who);
    if (h->cplx) {
        if ((h->w_up && (!wide_up(h) || !h->amp_up)) || (h->w_dn && (!wide_dn(h) || !h->amp_dn)))
            return set_error(ED_EINVAL, "%s: complex amplitudes need 32-bit complex tables and amplitude arrays", who);
        if (h->dim_up > kComplexMaxDim || h->dim_dn > kComplexMaxDim)
            return set_error(ED_EOVERFLOW, "%s: per-spin dims above %d with complex tables", who, kComplexMaxDim);
    }
    if (!valid_tile_id(h->tile)) return set_error(ED_EINVAL, "%s: bad tile id %d", who, h->tile);
    if (h->win_dn && (h->win_cols <= 0 || (h->win_cols & 63) || h->win_max <= 0 || h->win_max > h->dim_dn))
        return set_error(ED_EINVAL, "%s: bad neighbour windows (win_cols %d, win_max %d)", who, h->win_cols, h->win_max);
    if (h->win_tab && (!h->win_dn || h->win_max > 32767))
        return set_error(ED_EINVAL, "%s: a window-relative table needs windows of at most 32767 states", who);
    if (!std::isfinite(h->t) || !std::isfinite(h->U)) return set_error(ED_EINVAL, "%s: non-finite t or U", who);
    return ED_OK;
}

// calls that take real instances only
static inline int check_real(const ed_ham *h, const char *who) {
    int rc = check_ham(h, who);
    if (rc) return rc;
    if (h->cplx) return set_error(ED_EINVAL, "%s: complex amplitudes are not supported by this call", who);
    return ED_OK;
}

static inline int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return ED_OK;
    return set_error(ED_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace ed

#define ED_HIP(call)                                          \
    do {                                                      \
        int rc_ = ::ed::hip_check((call), #call);             \
        if (rc_) return rc_;                                  \
    } while (0)

#define ED_LAUNCHED(name)                                     \
    do {                                                      \
        int rc_ = ::ed::hip_check(hipGetLastError(), name);   \
        if (rc_) return rc_;                                  \
    } while (0)
