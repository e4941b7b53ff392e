// Host-side internals shared by the library's translation units: the
// lattice handle, parameter checks, lane-draw shapes, launch shapes and the
// step arguments.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/okpz.h"
#include "db_rows.hpp"
#include "dt_rows.hpp"
#include "kernels.hpp"
#include "philox.hpp"

namespace okpz_host {

using namespace okpz;

// HIP error text of the calling thread (okpz_last_error)
int hip_fail(hipError_t e, const char *what);
// any other status with an explanation for okpz_last_error
int fail_with(int status, const char *what);

#define HIP_TRY(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

inline bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

inline uint32_t ilog2(uint64_t v)
{
    uint32_t r = 0;
    while ((uint64_t(1) << r) < v) ++r;
    return r;
}

constexpr uint32_t kMaxL = 1u << 17;
constexpr uint32_t kMaxLds = 160u * 1024u;  // gfx950 LDS per workgroup
constexpr uint64_t kMcsLimit = uint64_t(1) << 30;

struct TimedPair {
    hipEvent_t start, stop;
    int kind;  // 0 step, 1 measure
};

}  // namespace okpz_host

struct okpz_lattice {
    okpz_params prm;
    hipStream_t stream = nullptr;
    uint32_t *words = nullptr;
    bool external = false;
    uint64_t nwords = 0;
    uint64_t mcs = 0;
    // measurement
    int32_t *h0 = nullptr;
    int32_t *h0s = nullptr;
    uint32_t *snap = nullptr;
    int64_t *partial = nullptr;
    int64_t *reduced = nullptr;
    int64_t *host_out = nullptr;  // pinned
    bool has_snap = false;
    uint64_t snap_mcs = 0;
    __int128 snap_s1 = 0;
    uint32_t threads = 0;  // device-step workgroup size (0: by the number of tiles per step)
    uint32_t cus = 0;      // compute units of the device
    // timing
    bool timing = false;
    std::vector<okpz_host::TimedPair> pairs;
};

namespace okpz_host {

// ---------------------------------------------------------------- validation
struct WindowShape {
    uint32_t NWX, NB, P, NR, PY, shared_edges;
};

// The window of a domain: Dx + 1 sites starting at any column of a block
// span Dx/32 + 1 blocks (2 for Dx < 32); Dy + 1 rows starting at any row of
// a band span Dy/4 + 1 bands.
inline WindowShape window_shape(const okpz_params &p)
{
    WindowShape w;
    w.NWX = (p.dom_x + 31) / 32 + 1;
    w.NB = p.dom_y / 4 + 1;
    w.P = (w.NWX + 1) | 1u;  // odd pitches spread random accesses over the LDS banks
    w.NR = 4 * w.NB;
    w.PY = (w.NR + 1) | 1u;
    w.shared_edges = p.dom_x < 32 ? 1u : 0u;
    return w;
}

inline uint32_t cells_of(const okpz_params &p) { return (p.dom_x / p.cell_x) * (p.dom_y / p.cell_y); }

// LDS bytes of one device-step workgroup with nslot = lanes x cells per lane
// (0: the largest any workgroup shape uses, max(cells, 256)).
inline uint64_t step_lds_bytes(const okpz_params &p, uint32_t nslot = 0)
{
    const WindowShape w = window_shape(p);
    if (nslot == 0) nslot = std::max<uint32_t>(cells_of(p), 256u);
    return 4ull * step_lds_words(w.NR, w.P, w.NWX, w.PY, w.NB, w.shared_edges, nslot, p.block_scheme == OKPZ_BLOCK_DB,
                                 p.device_layer == OKPZ_DEVICE_DB ? 1u : 0u);
}

inline int check_params(const okpz_params *p)
{
    if (!p) return OKPZ_EINVAL;
    if (!is_pow2(p->L) || p->L < 64 || p->L > kMaxL) return OKPZ_EINVAL;
    if (!is_pow2(p->dom_x) || !is_pow2(p->dom_y) || p->dom_x < 4 || p->dom_y < 4) return OKPZ_EINVAL;
    if (2 * p->dom_x > p->L || 2 * p->dom_y > p->L) return OKPZ_EINVAL;
    if (!is_pow2(p->cell_x) || !is_pow2(p->cell_y) || p->cell_x < 2 || p->cell_y < 2) return OKPZ_EINVAL;
    if (p->cell_x > 64 || p->cell_y > 64 || p->cell_x > p->dom_x || p->cell_y > p->dom_y) return OKPZ_EINVAL;
    if (p->block_scheme < OKPZ_BLOCK_DT || p->block_scheme > OKPZ_BLOCK_DTR) return OKPZ_EINVAL;
    if (p->origin_mode < OKPZ_ORIGIN_RANDOM || p->origin_mode > OKPZ_ORIGIN_COARSE) return OKPZ_EINVAL;
    if (p->device_layer != OKPZ_DEVICE_DT && p->device_layer != OKPZ_DEVICE_DB) return OKPZ_EINVAL;
    if (step_lds_bytes(*p) > kMaxLds) return OKPZ_EINVAL;
    const uint64_t ncell = uint64_t(p->dom_x / p->cell_x) * (p->dom_y / p->cell_y);
    if (ncell > 4096u) return OKPZ_EINVAL;  // at most 16 cells per lane of a 256-thread workgroup

    return OKPZ_OK;
}

// ---------------------------------------------------------------- exact rounding
// Correctly rounded (nearest, ties to even) conversion of a 128-bit integer.
inline double i128_to_double(__int128 v)
{
    if (v == 0) return 0.0;
    const bool neg = v < 0;
    unsigned __int128 m = neg ? (unsigned __int128)(-(v + 1)) + 1 : (unsigned __int128)v;
    int msb = 127;
    while (!((m >> msb) & 1)) --msb;
    double r;
    if (msb <= 52) {
        r = (double)(uint64_t)m;
    } else {
        const int drop = msb - 52;  // keep 53 significant bits
        unsigned __int128 keep = m >> drop;
        const unsigned __int128 rem = m & (((unsigned __int128)1 << drop) - 1);
        const unsigned __int128 half = (unsigned __int128)1 << (drop - 1);
        if (rem > half || (rem == half && (keep & 1))) ++keep;
        r = std::ldexp((double)(uint64_t)keep, drop);  // keep <= 2^53, exact
    }
    return neg ? -r : r;
}

inline __int128 pair_to_i128(const int64_t *p) { return ((__int128)p[1] << 64) | (uint64_t)p[0]; }

inline okpz_i128 to_abi(__int128 v)
{
    okpz_i128 r;
    r.lo = (uint64_t)v;
    r.hi = (int64_t)(v >> 64);
    return r;
}

// ---------------------------------------------------------------- MCS draw
// Origin uniform over all sites and one of the 24 orders of the four domain
// sets (Sec. 3: DT shuffles the set order each MCS; DTr moves the origin),
// from the Philox block (0, 0xFFFFFFFF, 0xFFFFFFFF, 4*MCS); the order is
// entry floor(24 w2 / 2^32) of the permutations in lexicographic order.
struct McsDraw {
    uint32_t ox, oy;
    int perm[4];
};

inline McsDraw mcs_draw(const okpz_params &p, uint64_t m)
{
    const u32x4 w = philox4x32_10(p.seed, p.stream, 0u, 0xFFFFFFFFu, 0xFFFFFFFFu, (uint32_t)(m << 2));
    McsDraw d;
    d.ox = w.x & (p.L - 1);
    d.oy = w.y & (p.L - 1);
    if (p.origin_mode == OKPZ_ORIGIN_FIXED) d.ox = d.oy = 0;
    if (p.origin_mode == OKPZ_ORIGIN_COARSE) {
        d.ox &= ~3u;
        d.oy &= ~3u;
    }
    const uint32_t pick = (uint32_t)(((uint64_t)w.z * 24u) >> 32);
    int perm[4] = {0, 1, 2, 3};
    for (uint32_t i = 0; i < pick; ++i) std::next_permutation(perm, perm + 4);
    std::memcpy(d.perm, perm, sizeof(perm));
    return d;
}

// ---------------------------------------------------------------- lane-draw shape
struct LaneShape {
    uint32_t s_bits, F_log2;
    bool accept;
    uint64_t P, Q;  // thresholds on the (A+32)-bit acceptance variate
};

inline bool prob01(double v) { return v == 0.0 || v == 1.0; }

inline LaneShape lane_shape(const okpz_params &p, double pd, double qr)
{
    LaneShape ls;
    const uint32_t sites = p.block_scheme == OKPZ_BLOCK_DB ? p.cell_x * p.cell_y : p.cell_x * p.cell_y / 4;
    ls.s_bits = ilog2(sites);
    ls.accept = !(prob01(pd) && prob01(qr));
    if (ls.accept) {
        const uint32_t F = 1u << ilog2(ls.s_bits + 8);
        ls.F_log2 = ilog2(F);
        const uint32_t A = F - ls.s_bits;
        const double scale = std::ldexp(1.0, (int)(A + 32));
        const uint64_t full = uint64_t(1) << (A + 32);
        const double pp = std::floor(pd * scale + 0.5), qq = std::floor(qr * scale + 0.5);
        ls.P = pp >= (double)full ? full : (uint64_t)pp;
        ls.Q = qq >= (double)full ? full : (uint64_t)qq;
    } else {
        ls.F_log2 = ilog2(std::max<uint32_t>(ls.s_bits, 1));
        ls.P = ls.Q = 0;
    }
    return ls;
}

// ---------------------------------------------------------------- launch helpers
inline void begin_timed(okpz_lattice *lat, int kind, TimedPair &tp)
{
    tp.kind = kind;
    if (!lat->timing) return;
    (void)hipEventCreate(&tp.start);
    (void)hipEventCreate(&tp.stop);
    (void)hipEventRecord(tp.start, lat->stream);
}

inline void end_timed(okpz_lattice *lat, TimedPair &tp)
{
    if (!lat->timing) return;
    (void)hipEventRecord(tp.stop, lat->stream);
    lat->pairs.push_back(tp);
}

// Workgroup shape of the device step: `threads` lanes (64, 128 or 256; 0
// picks 256) with ncell / threads cells each (at most 16), fewer lanes when
// the domain has fewer cells.  Results do not depend on the shape.
// Lanes per device-step workgroup when none is configured: 256, or 512 when a
// step has fewer than 4 tiles per compute unit (more lanes then share the few
// tiles; with more tiles 256-lane workgroups keep more of them resident);
// at most half the domain's cells once it has 256 or more, so that every lane
// holds two cells or more: the row-paired DB kernel needs two, and the other
// kernels then pay one barrier per two attempts of a lane instead of one.
inline uint32_t default_threads(uint64_t ntiles, uint32_t cus, uint32_t ncell)
{
    const uint32_t nt = ntiles < 4ull * cus ? 512u : 256u;
    return ncell >= 256u ? std::min(nt, ncell / 2u) : nt;
}

inline void step_shape(uint32_t ncell, uint32_t threads, uint32_t &cpt, uint32_t &nt)
{
    nt = threads ? threads : 256u;
    if (ncell <= nt) {
        cpt = 1;
        nt = std::max<uint32_t>(64, ncell);
    } else {
        cpt = ncell / nt;
    }
}

inline StepArgs base_args(const okpz_lattice *lat, const LaneShape &ls, double pd, double qr)
{
    const okpz_params &p = lat->prm;
    const WindowShape ws = window_shape(p);
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.words = lat->words;
    a.nbx_log2 = ilog2(p.L / 32);
    a.nbx_mask = p.L / 32 - 1;
    a.nby_mask = p.L / 4 - 1;
    a.L_mask = p.L - 1;
    a.Dx = p.dom_x;
    a.Dy = p.dom_y;
    a.log2Cx = ilog2(p.cell_x);
    a.log2Cy = ilog2(p.cell_y);
    a.log2ncx = ilog2(p.dom_x / p.cell_x);
    a.ncell = (p.dom_x / p.cell_x) * (p.dom_y / p.cell_y);
    a.dev_db = p.device_layer == OKPZ_DEVICE_DB ? 1u : 0u;
    a.log2ntx = ilog2(p.L / ((2 - a.dev_db) * p.dom_x));
    a.key0 = p.seed;
    a.key1 = p.stream;
    a.s_bits = ls.s_bits;
    a.F_log2 = ls.F_log2;
    a.rounds = p.cell_x * p.cell_y;
    a.NWX = ws.NWX;
    a.NB = ws.NB;
    a.P = ws.P;
    a.NR = ws.NR;
    a.PY = ws.PY;
    a.shared_edges = ws.shared_edges;
    a.flip_table = (pd == 1.0 ? kFlipMin : 0u) | (qr == 1.0 ? kFlipMax : 0u);
    a.P_hi = (uint32_t)(ls.P >> 32);
    a.P_lo = (uint32_t)ls.P;
    a.Q_hi = (uint32_t)(ls.Q >> 32);
    a.Q_lo = (uint32_t)ls.Q;
    a.pq_delta = (int32_t)a.P_hi - (int32_t)a.Q_hi;
    return a;
}

// Moments (and correlation, against the snapshot) from the 128-bit totals in
// lat->host_out.
void fill_moments(const okpz_lattice *lat, okpz_moments *out);
// the same from the exact totals of the moments pass (S1 even, S1 odd, S2
// even, S2 odd as (lo, hi) int64 pairs) of a lattice of size L at MCS mcs
void moments_from_totals(uint64_t L, uint64_t mcs, const int64_t *totals, okpz_moments *out);
void fill_correlation(const okpz_lattice *lat, okpz_correlation *out);

}  // namespace okpz_host
