/*
 * CPU oracle for the random-sequential (RS) octahedron model and its DTr
 * domain-decomposition schedule (Kelling, Odor, Gemming, "Suppressing
 * correlations in massively parallel simulations of lattice models",
 * arXiv:1705.01022).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow, obviously correct C
 * that the tests, the smoke check and the CPU-baseline leg of the benchmark
 * compare the GPU library against.  It shares no code, header, table or
 * constant with the GPU path and must never be linked into it.
 *
 * State convention (one byte per site, index y*L + x, x fast, periodic):
 *   bit 0 = sx[x,y] = 1  <=>  h(x,y) - h(x-1,y) = +1
 *   bit 1 = sy[x,y] = 1  <=>  h(x,y) - h(x,y-1) = +1
 * Each site stores its x and y slopes towards its left and lower neighbours
 * (Sec. 3, DB scheme), so an update at (x,y) reads and writes sx[x,y],
 * sx[x+1,y], sy[x,y], sy[x,y+1] only.
 *
 * Contents
 *   1. Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 *      SC'11, "Parallel random numbers: as easy as 1, 2, 3").
 *   2. The update rule (Sec. 2.1, Kawasaki dimer-exchange equation).
 *   3. Sequential RS dynamics, the paper's correlation-free reference
 *      (Sec. 1 and Sec. 4.3), driven by its own generator (xoshiro256**),
 *      unrelated to Philox.
 *   4. Step-by-step emulation of DTr at device level (Sec. 3, DTr) with
 *      single-hit DT / DB (delayed borders) / DTr at block level (Sec. 3.1),
 *      under the counter-based random-number contract described at
 *      dtr_lane_draw() below; the negative controls: a fixed or coarse
 *      origin, and dead borders at device level (Sec. 3 DB, cDB of
 *      Sec. 4.1).  Optional window mode for sampled checks.
 *   5. Heights and exact integer moments for W^2 (Sec. 2.1, roughness
 *      definition), the height autocorrelation C_h and the slope
 *      autocorrelation C_s (Sec. 2.1).
 *
 * Parity status: every function here is pinned by the CPU tests
 * (brute force over all 990 states of the 4x4 torus, the exact master
 * equation, invariants, symmetry, third-party Philox).  Nothing is
 * "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* 1. Philox4x32-10 (SC'11): 10 rounds of the 4x32 S-P network, key bumped   */
/*    by the Weyl constants between rounds.                                  */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_call(uint32_t seed, uint32_t stream,
                        uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                        uint32_t w[4])
{
    const uint32_t key[2] = {seed, stream};
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    orc_philox4x32_10(key, ctr, w);
}

/* ------------------------------------------------------------------------ */
/* 2. State helpers and the update rule                                      */
/* ------------------------------------------------------------------------ */
static int get_sx(const uint8_t *s, uint32_t L, uint32_t x, uint32_t y)
{
    return s[(size_t)(y % L) * L + (x % L)] & 1;
}

static int get_sy(const uint8_t *s, uint32_t L, uint32_t x, uint32_t y)
{
    return (s[(size_t)(y % L) * L + (x % L)] >> 1) & 1;
}

/* Flat zig-zag surface h = (x+y) mod 2: every slope is +1 on odd sites. */
void orc_init_flat(uint8_t *s, uint32_t L)
{
    for (uint32_t y = 0; y < L; ++y)
        for (uint32_t x = 0; x < L; ++x) {
            uint8_t odd = (uint8_t)((x + y) & 1u);
            s[(size_t)y * L + x] = (uint8_t)(odd | (odd << 1));
        }
}

/*
 * A slope state is a valid periodic octahedron surface iff the height
 * function it defines closes around both periodic cycles (per row the
 * number of +1 x-slopes is L/2, per column the number of +1 y-slopes is
 * L/2) and around every elementary plaquette.
 * Returns 0 if valid, 1 row balance, 2 column balance, 3 plaquette, 4 bad bits.
 */
int orc_check_state(const uint8_t *s, uint32_t L)
{
    for (size_t i = 0; i < (size_t)L * L; ++i)
        if (s[i] & ~3u) return 4;
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t n = 0;
        for (uint32_t x = 0; x < L; ++x) n += (uint32_t)get_sx(s, L, x, y);
        if (2 * n != L) return 1;
    }
    for (uint32_t x = 0; x < L; ++x) {
        uint32_t n = 0;
        for (uint32_t y = 0; y < L; ++y) n += (uint32_t)get_sy(s, L, x, y);
        if (2 * n != L) return 2;
    }
    /* going (x-1,y-1) -> (x,y-1) -> (x,y) and (x-1,y-1) -> (x-1,y) -> (x,y)
       must give the same height difference */
    for (uint32_t y = 0; y < L; ++y)
        for (uint32_t x = 0; x < L; ++x) {
            int path_a = get_sx(s, L, x, y + L - 1) + get_sy(s, L, x, y);
            int path_b = get_sy(s, L, x + L - 1, y) + get_sx(s, L, x, y);
            if (path_a != path_b) return 3;
        }
    return 0;
}

/*
 * One update attempt at site (x,y) (Sec. 2.1, Kawasaki rule): the four
 * slopes around the site are a = sx[x,y], b = sx[x+1,y], c = sy[x,y],
 * d = sy[x,y+1].  (a,b,c,d) = (0,1,0,1) is a local minimum: depositing an
 * octahedron (probability p) turns it into (1,0,1,0), raising h by 2.
 * (1,0,1,0) is a local maximum: removal (probability q) turns it into
 * (0,1,0,1).  Every other configuration is left alone.
 * dep_ok / rem_ok carry the outcome of the acceptance draw.
 * Returns +1 on deposition, -1 on removal, 0 otherwise.
 */
int orc_attempt(uint8_t *s, uint32_t L, uint32_t x, uint32_t y, int dep_ok, int rem_ok)
{
    uint32_t xr = (x + 1) % L, yd = (y + 1) % L;
    uint8_t *here = &s[(size_t)y * L + x];
    uint8_t *right = &s[(size_t)y * L + xr];
    uint8_t *down = &s[(size_t)yd * L + x];
    int a = *here & 1, b = *right & 1, c = (*here >> 1) & 1, d = (*down >> 1) & 1;
    int is_min = (a == 0 && b == 1 && c == 0 && d == 1);
    int is_max = (a == 1 && b == 0 && c == 1 && d == 0);
    if ((is_min && dep_ok) || (is_max && rem_ok)) {
        *here ^= 3u;  /* sx[x,y] and sy[x,y] */
        *right ^= 1u; /* sx[x+1,y] */
        *down ^= 2u;  /* sy[x,y+1] */
        return is_min ? +1 : -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3. Sequential RS with its own generator                                   */
/* ------------------------------------------------------------------------ */
/* splitmix64 (Steele, Lea, Flood 2014) seeds xoshiro256** (Blackman, Vigna). */
static uint64_t splitmix64_next(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t rotl64(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }

static uint64_t xoshiro_next(uint64_t st[4])
{
    uint64_t result = rotl64(st[1] * 5u, 7) * 9u;
    uint64_t t = st[1] << 17;
    st[2] ^= st[0];
    st[3] ^= st[1];
    st[1] ^= st[2];
    st[0] ^= st[3];
    st[2] ^= t;
    st[3] = rotl64(st[3], 45);
    return result;
}

void orc_seq_init(uint64_t st[4], uint64_t seed, uint64_t stream)
{
    uint64_t sm = seed * 0x100000001B3ull ^ (stream + 0x632BE59BD9B4E019ull);
    for (int i = 0; i < 4; ++i) st[i] = splitmix64_next(&sm);
}

/* uniform integer in [0, n) by rejection, n >= 1 */
static uint64_t xoshiro_below(uint64_t st[4], uint64_t n)
{
    uint64_t lim = UINT64_MAX - (UINT64_MAX % n);
    uint64_t v;
    do v = xoshiro_next(st); while (v >= lim);
    return v % n;
}

/*
 * n_mcs Monte Carlo steps of sequential RS (Sec. 1; the CPU reference of
 * Sec. 4.3): each MCS is L*L attempts, each at a site drawn uniformly
 * from the whole lattice, accepted with probability p (deposit) or q
 * (removal).  Returns the net number of depositions minus removals.
 */
int64_t orc_seq_mcs(uint8_t *s, uint32_t L, uint64_t n_mcs, double p, double q, uint64_t st[4])
{
    int64_t net = 0;
    uint64_t attempts = n_mcs * (uint64_t)L * (uint64_t)L;
    for (uint64_t i = 0; i < attempts; ++i) {
        uint32_t x = (uint32_t)xoshiro_below(st, L);
        uint32_t y = (uint32_t)xoshiro_below(st, L);
        double u = (double)(xoshiro_next(st) >> 11) * 0x1.0p-53;
        net += orc_attempt(s, L, x, y, u < p, u < q);
    }
    return net;
}

/* ------------------------------------------------------------------------ */
/* 4. DTr emulation                                                          */
/* ------------------------------------------------------------------------ */
enum { ORC_DT = 0, ORC_DB = 1, ORC_DTR = 2 };
enum { ORC_ORIGIN_RANDOM = 0, ORC_ORIGIN_FIXED = 1, ORC_ORIGIN_COARSE = 2 };
/* device layer: double tiling (four domain sets per MCS; DTr with a random
 * origin) or dead border (Sec. 3 DB: every tile at once, its rim inactive) */
enum { ORC_DEVICE_DT = 0, ORC_DEVICE_DB = 1 };

typedef struct {
    uint32_t L;        /* lateral size, power of two                        */
    uint32_t Dx, Dy;   /* device domain (sub-tile) size; tile is 2Dx x 2Dy  */
    uint32_t Cx, Cy;   /* block-level thread-cell size in sites             */
    int32_t scheme;    /* block-level scheme: ORC_DT, ORC_DB, ORC_DTR       */
    uint32_t seed;     /* Philox key word 0                                 */
    uint32_t stream;   /* Philox key word 1 (one per realization)           */
    double p, q;       /* deposition / removal probabilities                */
    uint32_t wx0, wy0; /* window origin (global, periodic)                  */
    uint32_t W, H;     /* window size; W = H = L means the whole lattice    */
    int32_t order;     /* 0 natural, 1 reversed, 2 shuffled within phases   */
    uint64_t order_seed;
    int32_t check_adjacency; /* 1: fail if two same-phase attempts touch   */
    int32_t origin_mode;     /* ORC_ORIGIN_*: random (DTr), fixed (DT), 4x4 grid */
    int32_t device;          /* ORC_DEVICE_*: double tiling or dead border      */
} orc_dtr_cfg;

static int is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

static uint32_t ilog2(uint32_t v)
{
    uint32_t r = 0;
    while ((1u << r) < v) ++r;
    return r;
}

static uint32_t next_pow2(uint32_t v)
{
    uint32_t r = 1;
    while (r < v) r <<= 1;
    return r;
}

int orc_dtr_validate(const orc_dtr_cfg *cfg)
{
    if (!is_pow2(cfg->L) || cfg->L < 4) return -1;
    if (!is_pow2(cfg->Dx) || !is_pow2(cfg->Dy) || cfg->Dx < 2 || cfg->Dy < 2) return -1;
    if (cfg->device != ORC_DEVICE_DT && cfg->device != ORC_DEVICE_DB) return -1;
    /* double tiling: tiles of 2Dx x 2Dy; dead border: tiles of Dx x Dy */
    if (cfg->device == ORC_DEVICE_DT && (2 * cfg->Dx > cfg->L || 2 * cfg->Dy > cfg->L)) return -1;
    if (cfg->Dx > cfg->L || cfg->Dy > cfg->L) return -1;
    if (!is_pow2(cfg->Cx) || !is_pow2(cfg->Cy) || cfg->Cx < 2 || cfg->Cy < 2) return -1;
    if (cfg->Cx > 64 || cfg->Cy > 64 || cfg->Cx > cfg->Dx || cfg->Cy > cfg->Dy) return -1;
    if (cfg->scheme < ORC_DT || cfg->scheme > ORC_DTR) return -1;
    if (!(cfg->p >= 0.0 && cfg->p <= 1.0 && cfg->q >= 0.0 && cfg->q <= 1.0)) return -1;
    if (cfg->W == 0 || cfg->H == 0 || cfg->W > cfg->L || cfg->H > cfg->L) return -1;
    if (cfg->origin_mode < ORC_ORIGIN_RANDOM || cfg->origin_mode > ORC_ORIGIN_COARSE) return -1;
    return 0;
}

/*
 * MCS draw (Sec. 3 DT: the order of the 2^d = 4 domain sets is a uniformly
 * shuffled permutation each MCS; Sec. 3 DTr: the decomposition origin is
 * moved to a uniformly random site each MCS).  Philox counter
 * (0, 0xFFFFFFFF, 0xFFFFFFFF, 4m); origin = low bits of words 0 and 1,
 * permutation = entry floor(24 * w2 / 2^32) of the 24 permutations of
 * {0,1,2,3} in lexicographic order.  origin_mode selects the negative
 * controls: fixed origin (plain DT) or origin on the 4x4-site grid (cDB-like).
 */
void orc_mcs_draw(const orc_dtr_cfg *cfg, uint32_t m, uint32_t out[6])
{
    uint32_t w[4];
    philox_call(cfg->seed, cfg->stream, 0u, 0xFFFFFFFFu, 0xFFFFFFFFu, m << 2, w);
    uint32_t ox = w[0] & (cfg->L - 1), oy = w[1] & (cfg->L - 1);
    if (cfg->origin_mode == ORC_ORIGIN_FIXED) { ox = 0; oy = 0; }
    if (cfg->origin_mode == ORC_ORIGIN_COARSE) { ox &= ~3u; oy &= ~3u; }
    uint32_t pick = (uint32_t)(((uint64_t)w[2] * 24u) >> 32);
    /* enumerate permutations of {0,1,2,3} in lexicographic order */
    uint32_t n = 0;
    for (uint32_t a = 0; a < 4; ++a)
        for (uint32_t b = 0; b < 4; ++b)
            for (uint32_t c = 0; c < 4; ++c)
                for (uint32_t d = 0; d < 4; ++d) {
                    if (a == b || a == c || a == d || b == c || b == d || c == d) continue;
                    if (n == pick) {
                        out[0] = ox; out[1] = oy;
                        out[2] = a; out[3] = b; out[4] = c; out[5] = d;
                    }
                    ++n;
                }
}

/*
 * Block draw for round rho of the domain of tile t in step k of MCS m:
 * one 16-bit field, eight per Philox call, counter
 * (rho/8, 0xFFFFFFFF, t, 4m+k).  Bits 0-1: the block-level domain set
 * (DT, DTr; chosen at random each round, not by permutation, Sec. 3.1);
 * bits 2-7 / 8-13: the cell-origin offset (DB, DTr; moved after every
 * collective single-hit update).
 */
static void dtr_block_draw(const orc_dtr_cfg *cfg, uint32_t m, uint32_t k, uint32_t t,
                           uint32_t rho, uint32_t *sigma, uint32_t *bx, uint32_t *by)
{
    uint32_t w[4];
    philox_call(cfg->seed, cfg->stream, rho >> 3, 0xFFFFFFFFu, t, (m << 2) | k, w);
    uint32_t f = rho & 7u;
    uint32_t field = (w[f >> 1] >> (16u * (f & 1u))) & 0xFFFFu;
    *sigma = field & 3u;
    *bx = (field >> 2) & (cfg->Cx - 1);
    *by = (field >> 8) & (cfg->Cy - 1);
    if (cfg->scheme == ORC_DT) { *bx = 0; *by = 0; }
}

/* Parameters of the lane draw that depend only on the configuration. */
typedef struct {
    uint32_t s;      /* site-index bits                                     */
    uint32_t F;      /* field width per attempt                             */
    uint32_t A;      /* acceptance-prefix bits, F - s                       */
    int accept;      /* 1 if p or q is strictly between 0 and 1             */
    uint64_t P, Q;   /* thresholds on the (A+32)-bit acceptance variate     */
} lane_shape;

static int prob_is_01(double v) { return v == 0.0 || v == 1.0; }

static lane_shape lane_shape_of(const orc_dtr_cfg *cfg)
{
    lane_shape ls;
    uint32_t sites = cfg->scheme == ORC_DB ? cfg->Cx * cfg->Cy : cfg->Cx * cfg->Cy / 4;
    ls.s = ilog2(sites);
    ls.accept = !(prob_is_01(cfg->p) && prob_is_01(cfg->q));
    if (ls.accept) {
        ls.F = next_pow2(ls.s + 8);
        ls.A = ls.F - ls.s;
        double scale = ldexp(1.0, (int)(ls.A + 32));
        uint64_t full = (uint64_t)1 << (ls.A + 32);
        double pp = floor(cfg->p * scale + 0.5), qq = floor(cfg->q * scale + 0.5);
        ls.P = pp >= (double)full ? full : (uint64_t)pp;
        ls.Q = qq >= (double)full ? full : (uint64_t)qq;
    } else {
        ls.F = next_pow2(ls.s > 1 ? ls.s : 1);
        ls.A = 0;
        ls.P = ls.Q = 0;
    }
    return ls;
}

/*
 * Lane draw for cell c in round rho.  The paper does not specify its
 * generator; this is the build's counter-based contract:
 *   F-bit field f = rho mod (128/F) of the Philox block with counter
 *   (floor(rho / (128/F)), c, t, 4m+k); the low s bits pick the site in the
 *   cell (its active quadrant for DT/DTr), the next A = F-s bits are the
 *   top of the acceptance variate.  When acceptance is needed, the variate
 *   is the (A+32)-bit integer U = (prefix << 32) | r with r = word 0 of the
 *   Philox block (rho, c | 0x80000000, t, 4m+k); deposition is accepted iff
 *   U < P = min(2^(A+32), floor(p 2^(A+32) + 1/2)), removal iff U < Q.
 */
static void dtr_lane_draw(const orc_dtr_cfg *cfg, const lane_shape *ls, uint32_t m, uint32_t k,
                          uint32_t t, uint32_t rho, uint32_t c,
                          uint32_t *idx, int *dep_ok, int *rem_ok)
{
    uint32_t per_call = 128u / ls->F, per_word = 32u / ls->F;
    uint32_t w[4];
    philox_call(cfg->seed, cfg->stream, rho / per_call, c, t, (m << 2) | k, w);
    uint32_t f = rho % per_call;
    uint32_t mask = ls->F == 32 ? 0xFFFFFFFFu : ((1u << ls->F) - 1u);
    uint32_t field = (w[f / per_word] >> (ls->F * (f % per_word))) & mask;
    *idx = field & ((1u << ls->s) - 1u);
    if (ls->accept) {
        uint32_t r[4];
        philox_call(cfg->seed, cfg->stream, rho, c | 0x80000000u, t, (m << 2) | k, r);
        uint64_t U = ((uint64_t)(field >> ls->s) << 32) | r[0];
        *dep_ok = U < ls->P;
        *rem_ok = U < ls->Q;
    } else {
        *dep_ok = cfg->p == 1.0;
        *rem_ok = cfg->q == 1.0;
    }
}

/* window helpers: global periodic site -> index into the window, or -1 */
static int64_t win_index(const orc_dtr_cfg *cfg, uint32_t gx, uint32_t gy)
{
    uint32_t lx = (gx + cfg->L - cfg->wx0 % cfg->L) % cfg->L;
    uint32_t ly = (gy + cfg->L - cfg->wy0 % cfg->L) % cfg->L;
    if (lx >= cfg->W || ly >= cfg->H) return -1;
    return (int64_t)ly * cfg->W + lx;
}

/* the update rule on a window-indexed state (same rule as orc_attempt) */
static int win_attempt(uint8_t *s, const orc_dtr_cfg *cfg, uint32_t gx, uint32_t gy,
                       int dep_ok, int rem_ok)
{
    int64_t ih = win_index(cfg, gx, gy);
    int64_t ir = win_index(cfg, (gx + 1) % cfg->L, gy);
    int64_t id = win_index(cfg, gx, (gy + 1) % cfg->L);
    int a = s[ih] & 1, b = s[ir] & 1, c = (s[ih] >> 1) & 1, d = (s[id] >> 1) & 1;
    int is_min = (a == 0 && b == 1 && c == 0 && d == 1);
    int is_max = (a == 1 && b == 0 && c == 1 && d == 0);
    if ((is_min && dep_ok) || (is_max && rem_ok)) {
        s[ih] ^= 3u;
        s[ir] ^= 1u;
        s[id] ^= 2u;
        return is_min ? +1 : -1;
    }
    return 0;
}

typedef struct {
    uint32_t gx, gy;
    int phase, dep_ok, rem_ok;
} attempt_rec;

/*
 * Footprint of a domain: its Dx x Dy sites plus the column at u = Dx (whose
 * sx bits rim updates flip) and the row at v = Dy (whose sy bits they
 * flip).  Returns 1 if the whole footprint is inside the window and valid.
 * Otherwise marks the part inside the window invalid and returns 0.
 */
static int footprint_ok(const orc_dtr_cfg *cfg, uint8_t *valid, uint32_t X0, uint32_t Y0)
{
    /* footprint entirely outside the window: nothing to check or invalidate */
    uint32_t lx0 = (X0 + cfg->L - cfg->wx0 % cfg->L) % cfg->L;
    uint32_t ly0 = (Y0 + cfg->L - cfg->wy0 % cfg->L) % cfg->L;
    if ((lx0 >= cfg->W && lx0 + cfg->Dx < cfg->L) || (ly0 >= cfg->H && ly0 + cfg->Dy < cfg->L))
        return 0;
    int ok = 1;
    for (uint32_t v = 0; v <= cfg->Dy && ok; ++v)
        for (uint32_t u = 0; u <= cfg->Dx; ++u) {
            if (u == cfg->Dx && v == cfg->Dy) continue;
            int64_t i = win_index(cfg, (X0 + u) % cfg->L, (Y0 + v) % cfg->L);
            if (i < 0 || (valid && !valid[i])) { ok = 0; break; }
        }
    if (ok) return 1;
    for (uint32_t v = 0; v <= cfg->Dy; ++v)
        for (uint32_t u = 0; u <= cfg->Dx; ++u) {
            if (u == cfg->Dx && v == cfg->Dy) continue;
            int64_t i = win_index(cfg, (X0 + u) % cfg->L, (Y0 + v) % cfg->L);
            if (i >= 0 && valid) valid[i] = 0;
        }
    return 0;
}

/* Fisher-Yates shuffle with splitmix64, used only by the order-invariance tests. */
static void shuffle_u32(uint32_t *a, uint32_t n, uint64_t *rs)
{
    for (uint32_t i = n; i > 1; --i) {
        uint32_t j = (uint32_t)(splitmix64_next(rs) % i);
        uint32_t tmp = a[i - 1]; a[i - 1] = a[j]; a[j] = tmp;
    }
}

/*
 * One device step: a full single-hit sweep of the domain of tile t
 * (Sec. 3.1).  Rounds rho = 0 .. Cx*Cy-1; each round gives every cell
 * exactly one attempt ("collective single-hit update"), so the domain
 * receives Dx*Dy attempts.
 *   DT  : cells split 2x2; each round picks one quadrant sigma at random;
 *         the attempt falls in that quadrant.
 *   DTr : as DT, with the cell grid shifted by a random (bx,by) each round.
 *   DB  : random cell-grid shift each round; attempts may fall anywhere in
 *         the cell.  Delayed borders: bulk attempts first, then those on the
 *         right or bottom rim of their cell, then the corner ones.
 * Attempts of one phase never touch a shared slope, so they commute; the
 * emulation applies them in cell order (or a test-chosen order) and, if
 * asked, verifies that no two of them are equal or nearest neighbours.
 * Returns attempts made, or -2 on an adjacency violation.
 */
static int64_t sweep_domain(uint8_t *s, const orc_dtr_cfg *cfg, const lane_shape *ls,
                            uint32_t m, uint32_t k, uint32_t t, uint32_t X0, uint32_t Y0,
                            attempt_rec *rec, uint32_t *order, int32_t *stamp, int32_t *stamp_ctr,
                            uint32_t *hits, uint64_t *rs)
{
    /* dead border at device level: the domain's last column and last row
     * are inactive; an attempt drawn there is not carried out (Sec. 3 DB) */
    const int dead_rim = cfg->device == ORC_DEVICE_DB;
    const uint32_t ncx = cfg->Dx / cfg->Cx, ncy = cfg->Dy / cfg->Cy;
    const uint32_t ncell = ncx * ncy, rounds = cfg->Cx * cfg->Cy;
    int64_t attempts = 0;
    for (uint32_t rho = 0; rho < rounds; ++rho) {
        uint32_t sigma, bx, by;
        dtr_block_draw(cfg, m, k, t, rho, &sigma, &bx, &by);
        for (uint32_t c = 0; c < ncell; ++c) {
            uint32_t cx = c % ncx, cy = c / ncx, idx, du, dv;
            int dep_ok, rem_ok;
            dtr_lane_draw(cfg, ls, m, k, t, rho, c, &idx, &dep_ok, &rem_ok);
            if (cfg->scheme == ORC_DB) {
                du = idx % cfg->Cx;
                dv = idx / cfg->Cx;
            } else {
                uint32_t hw = cfg->Cx / 2;
                du = (sigma & 1u) * (cfg->Cx / 2) + idx % hw;
                dv = (sigma >> 1) * (cfg->Cy / 2) + idx / hw;
            }
            uint32_t u = (bx + cx * cfg->Cx + du) % cfg->Dx;
            uint32_t v = (by + cy * cfg->Cy + dv) % cfg->Dy;
            rec[c].gx = (X0 + u) % cfg->L;
            rec[c].gy = (Y0 + v) % cfg->L;
            rec[c].phase = cfg->scheme == ORC_DB
                               ? (int)(du == cfg->Cx - 1) + (int)(dv == cfg->Cy - 1)
                               : 0;
            if (dead_rim && (u == cfg->Dx - 1 || v == cfg->Dy - 1)) {
                rec[c].phase = 3; /* never carried out, but drawn */
                ++attempts;
            }
            rec[c].dep_ok = dep_ok;
            rec[c].rem_ok = rem_ok;
        }
        for (int phase = 0; phase < 3; ++phase) {
            for (uint32_t i = 0; i < ncell; ++i) order[i] = i;
            if (cfg->order == 1)
                for (uint32_t i = 0; i < ncell; ++i) order[i] = ncell - 1 - i;
            if (cfg->order == 2) shuffle_u32(order, ncell, rs);
            int32_t mark = ++(*stamp_ctr);
            for (uint32_t i = 0; i < ncell; ++i) {
                const attempt_rec *a = &rec[order[i]];
                if (a->phase != phase) continue;
                if (stamp) {
                    /* no other attempt of this phase at the site or a nearest neighbour */
                    uint32_t L = cfg->L;
                    uint32_t nb[5][2] = {{a->gx, a->gy},
                                         {(a->gx + 1) % L, a->gy},
                                         {(a->gx + L - 1) % L, a->gy},
                                         {a->gx, (a->gy + 1) % L},
                                         {a->gx, (a->gy + L - 1) % L}};
                    for (int j = 0; j < 5; ++j) {
                        int64_t wi = win_index(cfg, nb[j][0], nb[j][1]);
                        if (wi >= 0 && stamp[wi] == mark) return -2;
                    }
                    stamp[win_index(cfg, a->gx, a->gy)] = mark;
                }
                win_attempt(s, cfg, a->gx, a->gy, a->dep_ok, a->rem_ok);
                if (hits) ++hits[win_index(cfg, a->gx, a->gy)];
                ++attempts;
            }
        }
    }
    return attempts;
}

/*
 * One MCS of DTr at device level (Sec. 3, DTr; Sec. 3.1): draw the origin
 * and the set permutation, then for each of the four steps k sweep every
 * domain of set perm[k] (domains of one set are independent, so tile order
 * is irrelevant).  Tile (tx,ty) has id t = ty*(L/2Dx) + tx and its active
 * domain starts at (ox + 2Dx tx + a Dx, oy + 2Dy ty + b Dy) mod L, where
 * (a,b) = (set & 1, set >> 1).
 *
 * Dead border at device level (cfg->device = ORC_DEVICE_DB; Sec. 3 DB, with
 * origin_mode COARSE the paper's cDB): one step, k = 0, in which every tile
 * of Dx x Dy sites, t = ty*(L/Dx) + tx starting at (ox + Dx tx, oy + Dy ty)
 * mod L, gets its sweep, attempts on its last column or last row not
 * carried out.  An active site's update reads and writes slopes of itself
 * and of its right and lower neighbours only, all inside its own tile, so
 * the tiles are independent and their order is irrelevant.  The set
 * permutation is drawn but unused.
 *
 * s: window state (W*H bytes).  valid: per-site validity flags for window
 * mode (NULL for the whole lattice).  stamp: W*H int32 scratch for the
 * adjacency check (NULL to skip).  hits: W*H counters incremented at every
 * attempted site (NULL to skip).  Returns attempts drawn (L*L for the whole
 * lattice) or a negative error.
 */
int64_t orc_dtr_mcs(uint8_t *s, uint8_t *valid, const orc_dtr_cfg *cfg, uint32_t m, int32_t *stamp,
                    uint32_t *hits)
{
    if (orc_dtr_validate(cfg) != 0) return -1;
    if (m >= (1u << 30)) return -1;
    if ((cfg->W < cfg->L || cfg->H < cfg->L) && !valid) return -1;
    const lane_shape ls = lane_shape_of(cfg);
    const int dead = cfg->device == ORC_DEVICE_DB;
    const uint32_t span = dead ? 1u : 2u, nsteps = dead ? 1u : 4u;
    const uint32_t ntx = cfg->L / (span * cfg->Dx), nty = cfg->L / (span * cfg->Dy);
    const uint32_t ncell = (cfg->Dx / cfg->Cx) * (cfg->Dy / cfg->Cy);
    attempt_rec *rec = (attempt_rec *)malloc(sizeof(attempt_rec) * ncell);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * ncell);
    uint32_t *tiles = (uint32_t *)malloc(sizeof(uint32_t) * ntx * nty);
    if (!rec || !order || !tiles) {
        free(rec); free(order); free(tiles);
        return -3;
    }
    uint64_t rs = cfg->order_seed ^ ((uint64_t)m << 32);
    int32_t stamp_ctr = 0;
    if (stamp) memset(stamp, 0, sizeof(int32_t) * (size_t)cfg->W * cfg->H);
    uint32_t draw[6];
    orc_mcs_draw(cfg, m, draw);
    int64_t total = 0;
    for (uint32_t k = 0; k < nsteps; ++k) {
        uint32_t set = dead ? 0u : draw[2 + k], a = set & 1u, b = set >> 1;
        for (uint32_t i = 0; i < ntx * nty; ++i) tiles[i] = cfg->order == 1 ? ntx * nty - 1 - i : i;
        if (cfg->order == 2) shuffle_u32(tiles, ntx * nty, &rs);
        for (uint32_t i = 0; i < ntx * nty; ++i) {
            uint32_t t = tiles[i], tx = t % ntx, ty = t / ntx;
            uint32_t X0 = (draw[0] + span * cfg->Dx * tx + a * cfg->Dx) % cfg->L;
            uint32_t Y0 = (draw[1] + span * cfg->Dy * ty + b * cfg->Dy) % cfg->L;
            if (!footprint_ok(cfg, valid, X0, Y0)) continue;
            int64_t n = sweep_domain(s, cfg, &ls, m, k, t, X0, Y0, rec, order,
                                     cfg->check_adjacency ? stamp : NULL, &stamp_ctr, hits, &rs);
            if (n < 0) {
                free(rec); free(order); free(tiles);
                return n;
            }
            total += n;
        }
    }
    free(rec); free(order); free(tiles);
    return total;
}

/* ------------------------------------------------------------------------ */
/* 5. Heights and exact moments                                              */
/* ------------------------------------------------------------------------ */
/*
 * Heights from slopes with the gauge h(0,0) = 0: walk down column 0 with
 * the y slopes, then along each row with the x slopes (a slope bit of 1 is
 * a +1 step, 0 a -1 step).
 */
void orc_heights(const uint8_t *s, uint32_t L, int64_t *h)
{
    for (uint32_t y = 0; y < L; ++y) {
        int64_t col0 = y == 0 ? 0 : h[(size_t)(y - 1) * L] + 2 * get_sy(s, L, 0, y) - 1;
        h[(size_t)y * L] = col0;
        for (uint32_t x = 1; x < L; ++x)
            h[(size_t)y * L + x] = h[(size_t)y * L + x - 1] + 2 * get_sx(s, L, x, y) - 1;
    }
}

static void put_i128(__int128 v, int64_t *out)
{
    out[0] = (int64_t)(uint64_t)(unsigned __int128)v;        /* low 64 bits  */
    out[1] = (int64_t)(v >> 64);                             /* high 64 bits */
}

/*
 * Parity-split integer moments of the height field: for the even (x+y even)
 * and odd classes, N = number of sites, S1 = sum h, S2 = sum h^2.
 * out = {N_e, N_o, S1_e(lo,hi), S1_o(lo,hi), S2_e(lo,hi), S2_o(lo,hi)};
 * the sums are 128-bit two's complement split into (low, high) 64-bit words.
 * W^2 (Sec. 2.1, roughness) = (N S2 - S1^2) / N^2 over all sites.
 */
int orc_moments(const uint8_t *s, uint32_t L, int64_t out[10])
{
    int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)L * L);
    if (!h) return -3;
    orc_heights(s, L, h);
    __int128 n[2] = {0, 0}, s1[2] = {0, 0}, s2[2] = {0, 0};
    for (uint32_t y = 0; y < L; ++y)
        for (uint32_t x = 0; x < L; ++x) {
            int cls = (int)((x + y) & 1u);
            __int128 v = h[(size_t)y * L + x];
            n[cls] += 1;
            s1[cls] += v;
            s2[cls] += v * v;
        }
    free(h);
    out[0] = (int64_t)n[0];
    out[1] = (int64_t)n[1];
    put_i128(s1[0], out + 2);
    put_i128(s1[1], out + 4);
    put_i128(s2[0], out + 6);
    put_i128(s2[1], out + 8);
    return 0;
}

/*
 * Cross moment sum_r h_t(r) h_s(r) of two states (same gauge convention),
 * used for the height autocorrelation C_h(t,s) = <h_t h_s> - <h_t><h_s>
 * (Sec. 2.1; at t = s it equals W^2).  out = {lo, hi}.
 */
int orc_cross(const uint8_t *st, const uint8_t *ss, uint32_t L, int64_t out[2])
{
    int64_t *ht = (int64_t *)malloc(sizeof(int64_t) * (size_t)L * L);
    int64_t *hs = (int64_t *)malloc(sizeof(int64_t) * (size_t)L * L);
    if (!ht || !hs) {
        free(ht); free(hs);
        return -3;
    }
    orc_heights(st, L, ht);
    orc_heights(ss, L, hs);
    __int128 acc = 0;
    for (size_t i = 0; i < (size_t)L * L; ++i) acc += (__int128)ht[i] * hs[i];
    free(ht); free(hs);
    put_i128(acc, out);
    return 0;
}

/*
 * Slope (lattice-gas) overlap of two states: the number of slope variables,
 * over both directions of every site, that are 1 in both,
 * sum_r [sx_t sx_s + sy_t sy_s].  The slope autocorrelation (Sec. 2.1)
 * C_s(t,s) = <n_t n_s> - <n_t><n_s> averages n over the 2 L^2 slope variables;
 * particle conservation fixes <n> = 1/2 in every state, so
 * C_s = overlap / (2 L^2) - 1/4.
 */
int64_t orc_slope_overlap(const uint8_t *st, const uint8_t *ss, uint32_t L)
{
    int64_t acc = 0;
    for (size_t i = 0; i < (size_t)L * L; ++i) {
        const uint8_t both = (uint8_t)(st[i] & ss[i]);
        acc += (both & 1) + ((both >> 1) & 1);
    }
    return acc;
}

/* size of the config struct, so the Python side can check its layout */
uint32_t orc_cfg_size(void) { return (uint32_t)sizeof(orc_dtr_cfg); }
