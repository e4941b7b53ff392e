// Device kernels of the octahedron-model simulator (gfx950).
//
// Lattice layout in HBM ("block words"): the L x L sites are cut into blocks
// of 32 x 4 sites; block (bx, by) = (x / 32, y / 4) has index by * (L/32) + bx
// and owns 8 consecutive uint32 words: words 0..3 hold the sx slope bits of
// its rows y%4 = 0..3, words 4..7 the sy bits, bit x%32 of each word.  sx = 1
// means the slope to the left neighbour is +1, sy = 1 the slope to the
// neighbour at y-1 is +1.  Two bits per site as in the paper's bit-coded
// lattice (Sec. 3.1), arranged as row bit-planes so that one funnel shift
// yields a site's two x-slopes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "philox.hpp"

namespace okpz {

// h = (x+y) mod 2: slopes +1 on odd sites; rows with y even read 1010..,
// odd rows 0101.., for both bit planes
constexpr uint32_t kFlatEvenRow = 0xAAAAAAAAu;
constexpr uint32_t kFlatOddRow = 0x55555555u;

enum : int { kDT = 0, kDB = 1, kDTR = 2 };

// ---------------------------------------------------------------- init
// Flat state: word i of the lattice belongs to row i % 4 of its block, so
// its parity is that of i.
static __global__ void fill_flat_kernel(uint32_t *__restrict__ words, uint64_t n)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        words[i] = (i & 1u) ? kFlatOddRow : kFlatEvenRow;
}

// ---------------------------------------------------------------- Philox test
static __global__ void philox_kernel(uint32_t k0, uint32_t k1, const uint32_t *__restrict__ ctr,
                              uint32_t *__restrict__ out, uint64_t n)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32x4 r = philox4x32_10_lane(k0, k1, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

// ---------------------------------------------------------------- device step
// Arguments of one device step: sweep every active domain of one domain set
// (Sec. 3 DTr; Sec. 3.1 application on GPUs).  One workgroup per tile.
struct StepArgs {
    uint32_t *words;
    uint32_t nbx_log2;          // log2(blocks per band) = log2(L/32)
    uint32_t nbx_mask;          // L/32 - 1
    uint32_t nby_mask;          // L/4 - 1 (bands)
    uint32_t L_mask;            // L - 1
    uint32_t Dx, Dy;            // domain size (sites)
    uint32_t log2Cx, log2Cy;    // cell size (sites), log2
    uint32_t log2ncx;           // log2(cells per domain row)
    uint32_t ncell;             // cells per domain
    uint32_t log2ntx;           // log2(tiles per lattice row)
    uint32_t ox, oy;            // tiling origin of this MCS
    uint32_t set_a, set_b;      // active sub-tile (set & 1, set >> 1)
    uint32_t key0, key1;        // Philox key (seed, stream)
    uint32_t c3;                // 4*MCS + step
    uint32_t s_bits;            // site-index bits of the lane draw
    uint32_t F_log2;            // log2 of the lane-draw field width
    uint32_t rounds;            // Cx*Cy single-hit rounds per step
    uint32_t NWX;               // window width in blocks
    uint32_t NB;                // window height in bands
    uint32_t P;                 // LDS sx plane: row pitch in words (odd, > NWX)
    uint32_t NR;                // window rows (4 NB)
    uint32_t PY;                // LDS sy plane: column pitch in words (odd, > NR)
    uint32_t shared_edges;      // Dx < 32: edge blocks may be shared with another domain
    uint32_t flip_table;        // no acceptance draw: kFlipMin / kFlipMax for the patterns that flip
    uint32_t P_hi, P_lo, Q_hi, Q_lo;  // acceptance thresholds on the (A+32)-bit variate
    int32_t pq_delta;           // P_hi - Q_hi (row-paired DB kernel)
    uint32_t dev_db;            // dead border at device level: every Dx x Dy tile in one step,
                                // attempts on its last column / row not carried out
};


// LDS staging.  The window covers bands by0 .. by0+NB-1 and blocks
// bx0 .. bx0+NWX-1 (periodic) of the lattice, i.e. the domain plus the column
// to its right and the row below.  In LDS it becomes two bit planes of
// NR = 4 NB rows: sx row-major (word row * P + k, so a site's word and the
// next one are adjacent) and sy column-major (word sy_base + k * PY + row, so
// rows y and y+1 are adjacent); P > NWX and PY > NR are odd, the padding is
// never written back.  Each wave copies whole bands: contiguous runs of 8 NWX words.
// When the domain is narrower than a block (Dx < 32) the first and last block
// of a band may also belong to another domain of the same set; their bits
// are then written back as an XOR with what was loaded (the two domains
// change disjoint bits), using the copy kept in `orig`.
template <bool LOAD>
__device__ __forceinline__ void copy_window(const StepArgs &A, uint32_t *lds, uint32_t *orig, uint32_t bx0,
                                            uint32_t by0)
{
    const uint32_t nwaves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t sy_base = A.NR * A.P;
    for (uint32_t b = wave; b < A.NB; b += nwaves) {
        const uint64_t band = static_cast<uint64_t>((by0 + b) & A.nby_mask) << A.nbx_log2;
        for (uint32_t t = lane; t < 8u * A.NWX; t += 64) {
            const uint32_t k = t >> 3, wib = t & 7u, row = 4u * b + (wib & 3u);
            const uint64_t g = ((band + ((bx0 + k) & A.nbx_mask)) << 3) + wib;
            const uint32_t li = wib < 4u ? row * A.P + k : sy_base + k * A.PY + row;
            // dead border: the tiles of one launch border each other, so the
            // blocks of the first and last two columns and bands -- which
            // may hold a neighbour's sites -- go back as XORs of the change
            const bool edge = A.dev_db ? (k == 0 || k + 2u >= A.NWX || b == 0 || b + 2u >= A.NB)
                                       : A.shared_edges && (k == 0 || k == A.NWX - 1);
            const uint32_t oi = A.dev_db ? (b * A.NWX + k) * 8u + wib : (b * 2u + (k == 0 ? 0u : 1u)) * 8u + wib;
            if (LOAD) {
                const uint32_t v = A.words[g];
                lds[li] = v;
                if (edge) orig[oi] = v;
            } else {
                if (edge)
                    atomicXor(&A.words[g], lds[li] ^ orig[oi]);
                else
                    A.words[g] = lds[li];
            }
        }
    }
}

// Slope pattern of an attempt: bit 0 sy(x,y+1), bit 1 sy(x,y), bit 2 sx(x,y),
// bit 3 sx(x+1,y).  Local minimum (sx(x), sx(x+1), sy(x), sy(y+1)) = (0,1,0,1)
// is 0x9, local maximum (1,0,1,0) is 0x6.  A flip mask holds bit k for
// pattern k twice, at k and k + 16, so that a pattern index with garbage in
// bit 4 selects the same bit (the bit-field extract reads 5 offset bits).
constexpr uint32_t kPatternMin = 0x9u, kPatternMax = 0x6u;
constexpr uint32_t kFlipMin = (1u << kPatternMin) | (1u << (kPatternMin + 16u));
constexpr uint32_t kFlipMax = (1u << kPatternMax) | (1u << (kPatternMax + 16u));

// 8 (w mod 256) in one instruction (a shift of the low byte selected as the
// operand; the compiler forms this itself for the other three bytes).
__device__ __forceinline__ uint32_t byte0_x8(uint32_t w)
{
    uint32_t r;
    asm("v_lshlrev_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(3u), "v"(w));
    return r;
}

// a + b + c in one instruction; c uniform.
__device__ __forceinline__ uint32_t add3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// a * b + c for a, b below 2^24 (one full-rate multiply-add); b uniform.
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// One cell's attempt in one round, decoded from its lane draw.
struct Draw {
    uint32_t ix;    // byte offset of the site's sx-plane word: 4 (row * P + column / 32)
    uint32_t iy;    // byte offset of its sy-plane word: 4 (sy_base + (column / 32) * PY + row)
    uint32_t sh;    // site bit in those words (column % 32)
    uint32_t mask;  // flip mask: kFlipMin set iff a local minimum here
                    // deposits, kFlipMax iff a local maximum is removed
    uint32_t pos;   // domain-local u | v << 16
    uint32_t rim;   // bit 0: right column of its cell, bit 1: bottom row (DB)
};

// Consumes the next F-bit field of a cell's lane-draw stream for round rho
// (rounds must be drawn in increasing order): field f = rho mod (128/F) of
// Philox block (rho / (128/F), cell, tile, 4*MCS+step), lowest bits first.
__device__ __forceinline__ uint32_t next_field(const StepArgs &A, uint32_t (&rw)[4], uint32_t rho, uint32_t cell,
                                               uint32_t tile)
{
    const uint32_t per_word_mask = (32u >> A.F_log2) - 1u;
    const uint32_t per_call_mask = (128u >> A.F_log2) - 1u;
    const uint32_t F = 1u << A.F_log2;
    if ((rho & per_call_mask) == 0u) {
        const u32x4 r = philox4x32_10_lane(A.key0, A.key1, rho >> (7u - A.F_log2), cell, tile, A.c3);
        rw[0] = r.x; rw[1] = r.y; rw[2] = r.z; rw[3] = r.w;
    }
    // field f of the current word: bits F*f .. F*f+F-1 (the offset is uniform;
    // the bit-field extract takes its width mod 32, so F = 32 is the word)
    const uint32_t field = F == 32u ? rw[0] : __builtin_amdgcn_ubfe(rw[0], (rho & per_word_mask) << A.F_log2, F);
    if (((rho + 1u) & per_word_mask) == 0u) {  // word used up: move to the next one
        rw[0] = rw[1];
        rw[1] = rw[2];
        rw[2] = rw[3];
    }
    return field;
}

// Block draw of round rho: 16-bit field rho mod 8 of Philox block
// (rho / 8, 0xFFFFFFFF, tile, 4*MCS+step): bits 0-1 the block-level domain
// set (DT, DTr), bits 2-7 and 8-13 the shift of the cell grid (DB, DTr).
struct BlockDraw {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ uint32_t next_block_field(const StepArgs &A, BlockDraw &b, uint32_t rho, uint32_t tile)
{
    if ((rho & 7u) == 0u) {
        const u32x4 r = philox4x32_10(A.key0, A.key1, rho >> 3, 0xFFFFFFFFu, tile, A.c3);
        b.w0 = r.x; b.w1 = r.y; b.w2 = r.z; b.w3 = r.w;
    }
    const uint32_t f16 = b.w0 & 0xFFFFu;
    if (rho & 1u) {
        b.w0 = b.w1; b.w1 = b.w2; b.w2 = b.w3;
    } else {
        b.w0 >>= 16;
    }
    return f16;
}

// Site of a cell's attempt from its field (low s_bits) and the round's block
// field f16.  base_u, base_v: the cell's corner in the domain; offx, offy:
// the domain's offset inside its first block / band.
template <int SCHEME, bool ACCEPT>
__device__ __forceinline__ Draw decode(const StepArgs &A, uint32_t field, uint32_t f16, uint32_t base_u,
                                       uint32_t base_v, uint32_t offx, uint32_t offy)
{
    const uint32_t idx = field & ((1u << A.s_bits) - 1u);
    uint32_t du, dv, u, v;
    if (SCHEME == kDB) {
        du = idx & ((1u << A.log2Cx) - 1u);
        dv = idx >> A.log2Cx;
    } else {
        const uint32_t hw = A.log2Cx - 1u;  // quadrant of the cell chosen by bits 0-1
        du = ((f16 & 1u) << hw) + (idx & ((1u << hw) - 1u));
        dv = (((f16 >> 1) & 1u) << (A.log2Cy - 1u)) + (idx >> hw);
    }
    if (SCHEME == kDT) {
        u = base_u + du;  // cell grid fixed: never wraps
        v = base_v + dv;
    } else {
        const uint32_t shx = (f16 >> 2) & ((1u << A.log2Cx) - 1u), shy = (f16 >> 8) & ((1u << A.log2Cy) - 1u);
        u = (shx + base_u + du) & (A.Dx - 1u);
        v = (shy + base_v + dv) & (A.Dy - 1u);
    }
    const uint32_t lx = u + offx, ly = v + offy;
    Draw d;
    if (SCHEME == kDB) {
        d.ix = __umul24(ly, A.P << 2) + ((lx >> 3) & ~3u);
        d.iy = ((A.NR * A.P) << 2) + __umul24(lx >> 5, A.PY << 2) + (ly << 2);
    } else {
        // the same addresses with both multiply-adds in one instruction each
        // (faster for DT and DTr; the DB kernels measured slower with them)
        const uint32_t hx = lx >> 5;  // the site's word column
        d.ix = mad24(ly, A.P << 2, hx << 2);
        d.iy = mad24(hx, A.PY << 2, (A.NR * A.P + ly) << 2);
    }
    d.sh = lx & 31u;
    d.mask = ACCEPT ? field >> A.s_bits : A.flip_table;  // acceptance prefix until accept_draws()
    if (A.dev_db && (u == A.Dx - 1u || v == A.Dy - 1u))
        d.mask = ACCEPT ? 0xFFFFFFFFu : 0u;  // dead border: a prefix no threshold accepts
    d.pos = SCHEME == kDB ? u | (v << 16) : 0u;
    d.rim = SCHEME == kDB ? ((du == (1u << A.log2Cx) - 1u) ? 1u : 0u) | ((dv == (1u << A.log2Cy) - 1u) ? 2u : 0u)
                          : 0u;
    return d;
}

// DB: what a cell keeps of its drawn attempt between the draw (one round
// ahead) and the attempt: the domain-local site, the flip mask (bits
// kPatternMin and kPatternMax) and the rim bits; the LDS addresses are derived
// again when the attempt runs.
struct CDraw {
    uint32_t pos;  // u | v << 16
    uint32_t ur;   // flip mask | rim (bit 0 right column, bit 1 bottom row); before
                   // accept_draws(): acceptance prefix << 2 | rim
};

template <bool ACCEPT>
__device__ __forceinline__ CDraw decode_db(const StepArgs &A, uint32_t field, uint32_t f16, uint32_t base_u,
                                           uint32_t base_v)
{
    const uint32_t idx = field & ((1u << A.s_bits) - 1u);
    const uint32_t cxm = (1u << A.log2Cx) - 1u, cym = (1u << A.log2Cy) - 1u;
    const uint32_t du = idx & cxm, dv = idx >> A.log2Cx;
    const uint32_t shx = (f16 >> 2) & cxm, shy = (f16 >> 8) & cym;
    const uint32_t u = (shx + base_u + du) & (A.Dx - 1u);
    const uint32_t v = (shy + base_v + dv) & (A.Dy - 1u);
    CDraw c;
    c.pos = u | (v << 16);
    c.ur = (ACCEPT ? (field >> A.s_bits) << 2 : 0u) | (du == cxm ? 1u : 0u) | (dv == cym ? 2u : 0u);
    // dead border at device level: no threshold accepts the prefix; without
    // acceptance draws bit 2 marks the attempt void for expand()
    if (A.dev_db && (u == A.Dx - 1u || v == A.Dy - 1u)) c.ur = (ACCEPT ? 0xFFFFFFFCu : 4u) | (c.ur & 3u);
    return c;
}

// Acceptance (Sec. 2.1 rates) of every cell's attempt of round rho, turned
// into flip masks.  The acceptance variate is U = prefix * 2^32 + r: a
// deposition is accepted iff U < P, a removal iff U < Q.  The prefix decides
// unless it equals the top bits of P or Q (probability about 2^(1-A)); only
// then r, word 0 of Philox block (rho, cell | 0x80000000, tile, 4*MCS+step),
// is drawn -- by a branch the whole wave skips when no lane needs it.
// pre[j]: the prefixes in, the masks out; cell[j]: the cells' ids.
template <int CPT>
__device__ __forceinline__ void accept_draws(const StepArgs &A, uint32_t (&pre)[CPT], const uint32_t (&cell)[CPT],
                                             uint32_t rho, uint32_t tile)
{
    bool tie[CPT];
    bool any = false;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        tie[j] = pre[j] == A.P_hi || pre[j] == A.Q_hi;
        any |= tie[j];
    }
    uint32_t mask[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j)
        mask[j] = (pre[j] < A.P_hi ? kFlipMin : 0u) | (pre[j] < A.Q_hi ? kFlipMax : 0u);
    if (__ballot(any)) {
#pragma unroll
        for (int j = 0; j < CPT; ++j)
            if (tie[j]) {
                const uint32_t r = philox4x32_10_lane(A.key0, A.key1, rho, cell[j] | 0x80000000u, tile, A.c3).x;
                if (pre[j] == A.P_hi && r < A.P_lo) mask[j] |= kFlipMin;
                if (pre[j] == A.Q_hi && r < A.Q_lo) mask[j] |= kFlipMax;
            }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) pre[j] = mask[j];
}

// The full attempt of a DB cell from its compact draw.
template <bool ACCEPT>
__device__ __forceinline__ Draw expand(const StepArgs &A, const CDraw &c, uint32_t offx, uint32_t offy)
{
    const uint32_t lx = (c.pos & 0xFFFFu) + offx, ly = (c.pos >> 16) + offy;
    Draw d;
    d.ix = __umul24(ly, A.P << 2) + ((lx >> 3) & ~3u);
    d.iy = ((A.NR * A.P) << 2) + __umul24(lx >> 5, A.PY << 2) + (ly << 2);
    d.sh = lx & 31u;
    d.mask = ACCEPT ? c.ur & ~3u : ((c.ur & 4u) ? 0u : A.flip_table);
    d.pos = c.pos;
    d.rim = c.ur & 3u;
    return d;
}

// One update attempt (Sec. 2.1 rule) at the site of d.  With the window as
// bit planes, a = sx(x,y) and b = sx(x+1,y) are two adjacent bits of the sx
// row (a funnel shift over the word and the next one, which leaves further
// bits above them: they reach bit 4 of the pattern index only), c = sy(x,y)
// and d = sy(x,y+1) the same bit of two consecutive sy rows.  A local minimum
// (0,1,0,1) may deposit, a local maximum (1,0,1,0) may be removed (as the
// draw's flip mask says); both flip the same four bits with LDS atomic XORs,
// because attempts of different cells may share a word (never a bit).  All
// decisions are bitwise; lanes that flip nothing (or whose `enable` is false)
// skip the XORs, and the flip of sx(x+1) in the next word (x at bit 31) is a
// further branch.
__device__ __forceinline__ void attempt(uint32_t *lds, const Draw &d, bool enable = true)
{
    char *base = reinterpret_cast<char *>(lds);
    uint32_t *px = reinterpret_cast<uint32_t *>(base + d.ix);
    uint32_t *py = reinterpret_cast<uint32_t *>(base + d.iy);
    const uint32_t w0 = px[0], w1 = px[1];
    const uint32_t y0 = py[0], y1 = py[1];
    const uint32_t ab = __builtin_amdgcn_alignbit(w1, w0, d.sh);
    const uint32_t cd = (__builtin_amdgcn_ubfe(y0, d.sh, 1) << 1) | __builtin_amdgcn_ubfe(y1, d.sh, 1);
    const uint32_t key = (ab << 2) | cd;
    // Most attempts flip nothing: their lanes sit out the atomics, which
    // leaves fewer active lanes to conflict on the LDS banks.
    if (enable && __builtin_amdgcn_ubfe(d.mask, key, 1) != 0u) {
        const uint32_t m = 1u << d.sh;
        atomicXor(&px[0], m | (m << 1));  // sx(x), and sx(x+1) unless x is bit 31
        atomicXor(&py[0], m);             // sy(x, y)
        atomicXor(&py[1], m);             // sy(x, y+1)
        if (d.sh == 31u) atomicXor(&px[1], 1u);  // sx(x+1) in the next word
    }
}

// A cell's published-site slot: cell c of thread c / CPT is stored at
// (c % CPT) * NT + c / CPT, so the lanes of one instruction touch
// consecutive words (no bank conflicts); nb_r, nb_d are the slots of the
// cells to the right and below.
struct CellGeom {
    uint32_t base;  // cell corner in the domain: base_u | base_v << 16
    uint32_t nb;    // published-site slots of the cells to the right (low 16 bits) and below
};

// Orders the LDS accesses of one wave: everything before completes, in
// program order, before anything after (a wave's LDS instructions execute in
// issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// DB: draw round rho+1 for every cell of the thread into nxt and publish
// the sites (buffer (rho+1) & 1), then run round rho whose draws are in cur.
//
// Delayed borders apply a round's attempts as bulk (phase 0), then edges
// (phase 1: right column or bottom row of the cell), then the corner
// (phase 2).  Only a rim attempt whose right or lower neighbour site holds the
// neighbouring cell's attempt depends on that order ("deferred"); all other
// attempts run in the first pass.  Dependencies point right (same cell row)
// or down (next cell row).  With `inwave`, every wave holds whole cell rows,
// at least two of them (or all of them), so the only deferred attempts with a
// dependency in another wave are bottom-row and corner attempts in a wave's
// last cell row ("remote"); their dependents are remote too.  Every other
// deferred attempt runs in its own wave right after the first pass, edges
// before corners, without a workgroup barrier; remote ones run after the
// round's barrier (edges, then corners, in program order), followed by one
// more barrier.  Without `inwave`, all deferred edges, then all deferred
// corners, run after barriers.
template <bool ACCEPT, int CPT>
__device__ __forceinline__ void db_round(const StepArgs &A, uint32_t *lds, uint32_t *cpos, uint32_t *flags,
                                         const CellGeom (&g)[CPT], uint32_t (&rw)[CPT][4], BlockDraw &bd,
                                         CDraw (&cur)[CPT], CDraw (&nxt)[CPT], uint32_t rho, uint32_t tile,
                                         uint32_t offx, uint32_t offy, const bool (&act)[CPT],
                                         const bool (&border)[CPT], bool inwave)
{
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    if (rho + 1u < A.rounds) {
        const uint32_t f16 = next_block_field(A, bd, rho + 1u, tile);
        const uint32_t nbuf = ((rho + 1u) & 1u) * (NT * CPT);
        uint32_t pre[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const uint32_t field = next_field(A, rw[j], rho + 1u, tid * CPT + j, tile);
            nxt[j] = decode_db<ACCEPT>(A, field, f16, g[j].base & 0xFFFFu, g[j].base >> 16);
            if (act[j]) cpos[nbuf + j * NT + tid] = nxt[j].pos;
            pre[j] = nxt[j].ur >> 2;
        }
        if (ACCEPT) {
            uint32_t ids[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) ids[j] = tid * CPT + j;
            accept_draws<CPT>(A, pre, ids, rho + 1u, tile);
#pragma unroll
            for (int j = 0; j < CPT; ++j) nxt[j].ur = pre[j] | (nxt[j].ur & 3u);
        }
    }
    // A rim attempt waits if the neighbouring cell's attempt sits on the site
    // to its right (right column / corner) or below it (bottom row / corner).
    // A target one past the domain edge is never a published site.
    const uint32_t buf = (rho & 1u) * (NT * CPT);
    bool def[CPT], remote[CPT];
    bool any1 = false, any2 = false;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const uint32_t pr = cpos[buf + (g[j].nb & 0xFFFFu)], pd = cpos[buf + (g[j].nb >> 16)];
        const uint32_t rim = cur[j].ur & 3u;
        const uint32_t want_r = (rim & 1u) ? cur[j].pos + 1u : 0xFFFFFFFFu;
        const uint32_t want_d = (rim & 2u) ? cur[j].pos + 0x10000u : 0xFFFFFFFFu;
        def[j] = act[j] && (pr == want_r || pd == want_d);
        remote[j] = inwave ? def[j] && border[j] && (rim & 2u) : def[j];
        any1 |= remote[j] && rim != 3u;
        any2 |= remote[j] && rim == 3u;
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j)
        attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy), !def[j] && act[j]);
    if (inwave) {
        wave_order();
#pragma unroll
        for (int j = 0; j < CPT; ++j)  // local deferred edges
            if (def[j] && !remote[j] && (cur[j].ur & 3u) != 3u)
                attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy));
        wave_order();
#pragma unroll
        for (int j = 0; j < CPT; ++j)  // local deferred corners
            if (def[j] && !remote[j] && (cur[j].ur & 3u) == 3u)
                attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy));
    }
    const uint64_t b1 = __ballot(any1), b2 = __ballot(any2);
    if ((tid & 63u) == 0u && (b1 | b2)) atomicOr(&flags[rho % 3u], (b1 ? 1u : 0u) | (b2 ? 2u : 0u));
    if (tid == 0) flags[(rho + 1u) % 3u] = 0u;
    __syncthreads();
    const uint32_t f = flags[rho % 3u];
    if (inwave) {
        if (f) {  // remote edges, then remote corners of the same waves
#pragma unroll
            for (int j = 0; j < CPT; ++j)
                if (remote[j] && (cur[j].ur & 3u) != 3u)
                    attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy));
            wave_order();
#pragma unroll
            for (int j = 0; j < CPT; ++j)
                if (remote[j] && (cur[j].ur & 3u) == 3u)
                    attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy));
            __syncthreads();
        }
        return;
    }
    if (f & 1u) {  // deferred edge attempts
#pragma unroll
        for (int j = 0; j < CPT; ++j)
            if (def[j] && (cur[j].ur & 3u) != 3u)
                attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy));
        __syncthreads();
    }
    if (f & 2u) {  // deferred corner attempts
#pragma unroll
        for (int j = 0; j < CPT; ++j)
            if (def[j] && (cur[j].ur & 3u) == 3u)
                attempt(lds, expand<ACCEPT>(A, cur[j], offx, offy));
        __syncthreads();
    }
}

// LDS words of one device-step workgroup (see sweep_tile); nslot = lanes x
// cells per lane.
// Words of the loaded copy kept for XOR write-back: two edge blocks per band
// for narrow domains, every block under a dead border at device level.
__host__ __device__ inline uint32_t orig_words(uint32_t NWX, uint32_t NB, uint32_t shared_edges, uint32_t dev_db)
{
    return dev_db ? 8u * NWX * NB : (shared_edges ? 16u * NB : 0u);
}

__host__ __device__ inline uint32_t step_lds_words(uint32_t NR, uint32_t P, uint32_t NWX, uint32_t PY, uint32_t NB,
                                                   uint32_t shared_edges, uint32_t nslot, bool db, uint32_t dev_db)
{
    return NR * P + (NWX + 1u) * PY + orig_words(NWX, NB, shared_edges, dev_db) + (db ? 2u * nslot + 4u : 0u);
}

// One domain sweep (device step of one tile).  The tile's active domain
// (sub-tile set (set_a, set_b)) is staged with its +x column and +y row in
// LDS, swept by Cx*Cy single-hit rounds (every cell gets exactly one attempt
// per round, Sec. 3.1) and written back.  Same-set domains of at least 32
// sites never share a block, so their write-back is plain; narrower ones XOR
// their changes into the two edge blocks of each band.  Lane `tid` owns cells
// tid*CPT .. tid*CPT+CPT-1; cells at or past A.ncell are idle (a domain with
// fewer cells than the workgroup has slots); FULL: the caller guarantees
// ncell = lanes x CPT.
//
// DT / DTr: the attempts of one round never touch each other, so a round is
// one pass.  DB (delayed borders: bulk attempts first, then those on the
// right column or bottom row of their cell, the corner last): only a rim
// attempt whose right or lower neighbour site holds an earlier-phase attempt
// of the neighbouring cell depends on the order, so every other attempt of
// the round runs in the first pass and the few dependent ones in one or two
// later passes.  All attempts of the first pass are pairwise non-adjacent
// and commute with the deferred ones they precede in phase order, so the
// result equals bulk -> edges -> corners exactly.  Attempt sites depend only
// on the random stream, so each cell publishes its next round's site one
// round ahead (double-buffered in LDS) and the check needs no extra barrier.
template <int SCHEME, bool ACCEPT, int CPT, bool FULL>
__device__ __forceinline__ void sweep_tile(const StepArgs &A, uint32_t *smem, uint32_t tile)
{
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    uint32_t *lds = smem;                                              // sx plane, then sy plane
    uint32_t *orig = smem + A.NR * A.P + (A.NWX + 1u) * A.PY;          // edge blocks as loaded
    uint32_t *cpos = orig + orig_words(A.NWX, A.NB, A.shared_edges, A.dev_db);  // DB: 2 x NT*CPT published sites
    uint32_t *flags = cpos + 2u * NT * CPT;                            // DB: 3 round flags

    const uint32_t tx = tile & ((1u << A.log2ntx) - 1u), ty = tile >> A.log2ntx;
    // tiles of 2D x 2D (double tiling) or D x D (dead border, one step per MCS)
    const uint32_t X0 = (A.ox + (2u - A.dev_db) * A.Dx * tx + A.set_a * A.Dx) & A.L_mask;
    const uint32_t Y0 = (A.oy + (2u - A.dev_db) * A.Dy * ty + A.set_b * A.Dy) & A.L_mask;
    const uint32_t offx = X0 & 31u, offy = Y0 & 3u;

    copy_window<true>(A, lds, orig, X0 >> 5, Y0 >> 2);

    const uint32_t ncx_mask = (1u << A.log2ncx) - 1u;
    const uint32_t ncy_mask = (A.ncell >> A.log2ncx) - 1u;
    // a cell's published-site slot: cell c of thread c / CPT is stored at
    // (c % CPT) * NT + c / CPT, so the lanes of one instruction touch
    // consecutive words (no LDS bank conflicts)
    auto slot_of = [&](uint32_t c) { return (c % CPT) * NT + c / CPT; };
    CellGeom g[CPT];
    uint32_t rw[CPT][4];
    bool act[CPT], border[CPT];
    // DB: waves hold whole cell rows, at least two of them or all of them
    const uint32_t cpw = 64u * CPT, ncx = 1u << A.log2ncx;
    const bool inwave = A.ncell <= cpw || (ncx <= cpw / 2u);
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        // a thread's cells are horizontal neighbours, so the lanes of one
        // instruction hit different LDS words
        const uint32_t cell = tid * CPT + j;
        const uint32_t cx = cell & ncx_mask, cy = (cell >> A.log2ncx) & ncy_mask;
        act[j] = FULL || cell < A.ncell;
        border[j] = ((cell + ncx) & (A.ncell - 1u)) / cpw != cell / cpw;  // the cell below is in another wave
        g[j].base = (cx << A.log2Cx) | ((cy << A.log2Cy) << 16);
        g[j].nb = slot_of((cy << A.log2ncx) | ((cx + 1u) & ncx_mask)) |
                  (slot_of((((cy + 1u) & ncy_mask) << A.log2ncx) | cx) << 16);
        rw[j][0] = rw[j][1] = rw[j][2] = rw[j][3] = 0u;
    }
    BlockDraw bd = {0u, 0u, 0u, 0u};

    if (SCHEME != kDB) {
        __syncthreads();
        for (uint32_t rho = 0; rho < A.rounds; ++rho) {
            const uint32_t f16 = next_block_field(A, bd, rho, tile);
            Draw d[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const uint32_t field = next_field(A, rw[j], rho, tid * CPT + j, tile);
                d[j] = decode<SCHEME, ACCEPT>(A, field, f16, g[j].base & 0xFFFFu, g[j].base >> 16, offx, offy);
            }
            if (ACCEPT) {
                uint32_t pre[CPT];
#pragma unroll
                for (int j = 0; j < CPT; ++j) pre[j] = d[j].mask;
                uint32_t ids[CPT];
#pragma unroll
                for (int j = 0; j < CPT; ++j) ids[j] = tid * CPT + j;
                accept_draws<CPT>(A, pre, ids, rho, tile);
#pragma unroll
                for (int j = 0; j < CPT; ++j) d[j].mask = pre[j];
            }
#pragma unroll
            for (int j = 0; j < CPT; ++j) attempt(lds, d[j], act[j]);
            __syncthreads();
        }
    } else {
        CDraw da[CPT], db[CPT];
        const uint32_t f16 = next_block_field(A, bd, 0u, tile);
        uint32_t pre[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const uint32_t field = next_field(A, rw[j], 0u, tid * CPT + j, tile);
            da[j] = decode_db<ACCEPT>(A, field, f16, g[j].base & 0xFFFFu, g[j].base >> 16);
            if (act[j]) cpos[j * NT + tid] = da[j].pos;
            pre[j] = da[j].ur >> 2;
        }
        if (ACCEPT) {
            uint32_t ids[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) ids[j] = tid * CPT + j;
            accept_draws<CPT>(A, pre, ids, 0u, tile);
#pragma unroll
            for (int j = 0; j < CPT; ++j) da[j].ur = pre[j] | (da[j].ur & 3u);
        }
        if (tid < 3) flags[tid] = 0u;
        __syncthreads();
        // Cx*Cy rounds, an even number: alternate the two draw buffers
        for (uint32_t rho = 0; rho < A.rounds; rho += 2) {
            db_round<ACCEPT, CPT>(A, lds, cpos, flags, g, rw, bd, da, db, rho, tile, offx, offy, act, border, inwave);
            db_round<ACCEPT, CPT>(A, lds, cpos, flags, g, rw, bd, db, da, rho + 1u, tile, offx, offy, act, border,
                                  inwave);
        }
    }
    copy_window<false>(A, lds, orig, X0 >> 5, Y0 >> 2);
}

// DB device step with each lane holding a column of CPT vertically stacked
// cells: lane t owns the cells (t mod ncx, CPT (t / ncx) + j), j = 0 .. CPT-1
// (needs cells = lanes x CPT, CPT >= 2 and at most 64 cells per row, so a
// wave holds whole rows of lanes).  The attempts, their random draws (keyed by
// cell id) and the delayed-border order are those of sweep_tile; only the
// bookkeeping differs.  Each round every cell draws its own attempt, except
// the top cell of each column, which is drawn one round ahead and published
// in LDS for the column above.  The dependency checks of the delayed borders
// (does the attempt of the cell to the right / below sit on the site right of /
// below mine?) read the cell below from the same lane (or, for the bottom
// cell, the published top cell of the column below), and the cell to the
// right from the neighbouring lane by a cross-lane permute.  A deferred
// attempt is "remote" only in a bottom cell whose column below lies in
// another wave, and only on the cell's bottom row; all others run in their
// own wave right after the first pass (edges, then corners), remote ones
// after the round's barrier, exactly as in db_round.
// One round of the column-mapped DB sweep.  field[j], j >= 1: the lane-draw
// fields of round rho; field[0]: the top cell's field of round rho + 1
// (has_next), drawn with the block field f16_next and published.
template <bool ACCEPT, int CPT>
__device__ __forceinline__ void db_columns_round(const StepArgs &A, uint32_t *lds, uint32_t *cpos, uint32_t *flags,
                                                 CDraw &top, const uint32_t (&field)[CPT], uint32_t f16,
                                                 uint32_t f16_next, bool has_next, uint32_t rho, uint32_t tile,
                                                 uint32_t offx, uint32_t offy, uint32_t base_u,
                                                 const uint32_t (&base_v)[CPT], const uint32_t (&cell)[CPT],
                                                 uint32_t below_lane, bool border, int rsrc)
{
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    // this round's attempts: the top cell's from the last round, the others drawn now
    Draw d[CPT];
    d[0] = expand<ACCEPT>(A, top, offx, offy);
    {
        uint32_t pre[CPT - 1], ids[CPT - 1];
#pragma unroll
        for (int j = 1; j < CPT; ++j) {
            d[j] = decode<kDB, ACCEPT>(A, field[j], f16, base_u, base_v[j], offx, offy);
            pre[j - 1] = d[j].mask;
            ids[j - 1] = cell[j];
        }
        if (ACCEPT) {
            accept_draws<CPT - 1>(A, pre, ids, rho, tile);
#pragma unroll
            for (int j = 1; j < CPT; ++j) d[j].mask = pre[j - 1];
        }
    }
    // the top cell's attempt of the next round, published for the column above
    if (has_next) {
        top = decode_db<ACCEPT>(A, field[0], f16_next, base_u, base_v[0]);
        if (ACCEPT) {
            uint32_t pre[1] = {top.ur >> 2};
            const uint32_t ids[1] = {cell[0]};
            accept_draws<1>(A, pre, ids, rho + 1u, tile);
            top.ur = pre[0] | (top.ur & 3u);
        }
        cpos[((rho + 1u) & 1u) * NT + tid] = top.pos;
    }
    // Order dependencies of the delayed borders: the attempt of the cell to
    // the right sits on the site right of mine, or the one of the cell below
    // on the site below mine.  Either implies that mine lies on my cell's
    // right column / bottom row (the neighbouring cell's sites can touch mine
    // only there; a site one past the domain edge is never a neighbour's), so
    // the rim needs no separate test; it is worked out only for deferred
    // attempts (a corner goes after the edges).
    //
    // The first pass takes a lane's cells bottom to top, so the attempt of the
    // cell below in the same lane has already run when mine runs: that
    // dependency needs no deferral, unless the attempt below is itself
    // deferred (it then sits on its cell's right column, so mine is a corner
    // and goes after it).  The dependency on the cell to the right (another
    // lane, same instruction) and on the cell below the lane's bottom cell
    // (another lane) always defers.
    const uint32_t cxm = (1u << A.log2Cx) - 1u, cym = (1u << A.log2Cy) - 1u;
    const uint32_t shx = (f16 >> 2) & cxm, shy = (f16 >> 8) & cym;  // this round's cell-grid shift
    auto bottom_row = [&](int j) { return (((d[j].pos >> 16) - shy - base_v[j]) & (A.Dy - 1u)) == cym; };
    auto corner = [&](int j) {
        return bottom_row(j) && (((d[j].pos & 0xFFFFu) - shx - base_u) & (A.Dx - 1u)) == cxm;
    };
    const uint32_t pbot = cpos[(rho & 1u) * NT + below_lane];
    bool def[CPT], remote[CPT];
    bool any = false;
#pragma unroll
    for (int j = CPT - 1; j >= 0; --j) {
        const uint32_t pr = (uint32_t)__builtin_amdgcn_ds_bpermute(rsrc, (int)d[j].pos);
        const uint32_t pd = j + 1 < CPT ? d[j + 1 < CPT ? j + 1 : j].pos : pbot;
        const bool below = pd == d[j].pos + 0x10000u && (j == CPT - 1 || def[j + 1 < CPT ? j + 1 : j]);
        def[j] = pr == d[j].pos + 1u || below;
        // remote: a bottom-row attempt of a bottom cell whose column below is in another wave
        remote[j] = j == CPT - 1 && border && def[j] && bottom_row(j);
        any |= remote[j];
    }
#pragma unroll
    for (int j = CPT - 1; j >= 0; --j) attempt(lds, d[j], !def[j]);
    wave_order();
    bool cor[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {  // deferred edges of this wave
        cor[j] = false;
        if (def[j] && !remote[j]) {
            cor[j] = corner(j);
            if (!cor[j]) attempt(lds, d[j]);
        }
    }
    wave_order();
#pragma unroll
    for (int j = 0; j < CPT; ++j)  // deferred corners of this wave
        if (def[j] && !remote[j] && cor[j]) attempt(lds, d[j]);
    const uint64_t wave_any = __ballot(any);  // every lane takes part in the ballot
    if ((tid & 63u) == 0u && wave_any) atomicOr(&flags[rho % 3u], 1u);
    if (tid == 0) flags[(rho + 1u) % 3u] = 0u;
    __syncthreads();
    if (flags[rho % 3u]) {  // remote edges, then remote corners of the same waves
        const bool rc = remote[CPT - 1] && corner(CPT - 1);
        if (remote[CPT - 1] && !rc) attempt(lds, d[CPT - 1]);
        wave_order();
        if (rc) attempt(lds, d[CPT - 1]);
        __syncthreads();
    }
}

// Field k (0 .. 128/F - 1) of a Philox block w, F = 2^FL bits, lowest first.
template <int FL>
__device__ __forceinline__ uint32_t block_field(const uint32_t (&w)[4], int k)
{
    constexpr int F = 1 << FL, FPW = 32 / F;
    if (F == 32) return w[k];
    return (w[k / FPW] >> (F * (k % FPW))) & ((1u << (F & 31)) - 1u);
}

// DB device step with each lane holding a column of CPT vertically stacked
// cells: lane t owns the cells (t mod ncx, CPT (t / ncx) + j), j = 0 .. CPT-1
// (needs cells = lanes x CPT, CPT >= 2 and at most 64 cells per row, so a
// wave holds whole rows of lanes).  The attempts, their random draws (keyed by
// cell id) and the delayed-border order are those of sweep_tile; only the
// bookkeeping differs.  Each round every cell draws its own attempt, except
// the top cell of each column, which is drawn one round ahead and published
// in LDS for the column above.  The dependency checks of the delayed borders
// (does the attempt of the cell to the right / below sit on the site right of /
// below mine?) read the cell below from the same lane (or, for the bottom
// cell, the published top cell of the column below), and the cell to the
// right from the neighbouring lane by a cross-lane permute.  A deferred
// attempt is "remote" only in a bottom cell whose column below lies in
// another wave, and only on the cell's bottom row; all others run in their
// own wave right after the first pass (edges, then corners), remote ones
// after the round's barrier, exactly as in db_round.
//
// FL > 0: the lane-draw field width is 2^FL bits (known at compile time) and
// the rounds are a multiple of the 128 / 2^FL fields of one Philox block; the
// rounds of one block are unrolled, so every field is a fixed shift of a
// fixed word.  FL = 0: the width is taken from A at run time.
template <bool ACCEPT, int CPT, int FL>
__device__ __forceinline__ void sweep_db_columns(const StepArgs &A, uint32_t *smem, uint32_t tile)
{
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    uint32_t *lds = smem;                                              // sx plane, then sy plane
    uint32_t *orig = smem + A.NR * A.P + (A.NWX + 1u) * A.PY;          // edge blocks as loaded
    uint32_t *cpos = orig + orig_words(A.NWX, A.NB, A.shared_edges, A.dev_db);  // 2 x NT published top-cell sites
    uint32_t *flags = cpos + 2u * NT;                                  // 3 round flags

    const uint32_t tx = tile & ((1u << A.log2ntx) - 1u), ty = tile >> A.log2ntx;
    // tiles of 2D x 2D (double tiling) or D x D (dead border, one step per MCS)
    const uint32_t X0 = (A.ox + (2u - A.dev_db) * A.Dx * tx + A.set_a * A.Dx) & A.L_mask;
    const uint32_t Y0 = (A.oy + (2u - A.dev_db) * A.Dy * ty + A.set_b * A.Dy) & A.L_mask;
    const uint32_t offx = X0 & 31u, offy = Y0 & 3u;

    copy_window<true>(A, lds, orig, X0 >> 5, Y0 >> 2);

    const uint32_t ncx = 1u << A.log2ncx;
    const uint32_t cx = tid & (ncx - 1u), grp = tid >> A.log2ncx;
    const uint32_t below_lane = (tid + ncx) & (NT - 1u);  // lane holding the column below
    const bool border = (below_lane >> 6) != (tid >> 6);   // ... in another wave
    const int rsrc = (int)((cx == ncx - 1u ? tid + 1u - ncx : tid + 1u) & 63u) << 2;  // lane of the column right
    const uint32_t base_u = cx << A.log2Cx;
    uint32_t cell[CPT], base_v[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const uint32_t cy = grp * CPT + j;
        cell[j] = (cy << A.log2ncx) | cx;
        base_v[j] = cy << A.log2Cy;
    }
    BlockDraw bd = {0u, 0u, 0u, 0u};
    uint32_t f16 = next_block_field(A, bd, 0u, tile);
    CDraw top;
    auto draw_top0 = [&](uint32_t field) {  // the top cell's draw for round 0
        top = decode_db<ACCEPT>(A, field, f16, base_u, base_v[0]);
        if (ACCEPT) {
            uint32_t pre[1] = {top.ur >> 2};
            const uint32_t ids[1] = {cell[0]};
            accept_draws<1>(A, pre, ids, 0u, tile);
            top.ur = pre[0] | (top.ur & 3u);
        }
        cpos[tid] = top.pos;
        if (tid < 3) flags[tid] = 0u;
        __syncthreads();
    };

    if constexpr (FL == 0) {
        uint32_t rw[CPT][4];
#pragma unroll
        for (int j = 0; j < CPT; ++j) rw[j][0] = rw[j][1] = rw[j][2] = rw[j][3] = 0u;
        draw_top0(next_field(A, rw[0], 0u, cell[0], tile));
        for (uint32_t rho = 0; rho < A.rounds; ++rho) {
            uint32_t field[CPT];
#pragma unroll
            for (int j = 1; j < CPT; ++j) field[j] = next_field(A, rw[j], rho, cell[j], tile);
            const bool has_next = rho + 1u < A.rounds;
            uint32_t f16n = 0u;
            field[0] = 0u;
            if (has_next) {
                f16n = next_block_field(A, bd, rho + 1u, tile);
                field[0] = next_field(A, rw[0], rho + 1u, cell[0], tile);
            }
            db_columns_round<ACCEPT, CPT>(A, lds, cpos, flags, top, field, f16, f16n, has_next, rho, tile, offx,
                                          offy, base_u, base_v, cell, below_lane, border, rsrc);
            f16 = f16n;
        }
    } else {
        constexpr int RPB = 128 >> FL;  // rounds per Philox block
        uint32_t w0[4];                 // the top cell's current block
        {
            const u32x4 r = philox4x32_10_lane(A.key0, A.key1, 0u, cell[0], tile, A.c3);
            w0[0] = r.x; w0[1] = r.y; w0[2] = r.z; w0[3] = r.w;
        }
        draw_top0(block_field<FL>(w0, 0));
        const uint32_t nblk = A.rounds / RPB;
        for (uint32_t blk = 0; blk < nblk; ++blk) {
            uint32_t w[CPT][4];
#pragma unroll
            for (int j = 1; j < CPT; ++j) {
                const u32x4 r = philox4x32_10_lane(A.key0, A.key1, blk, cell[j], tile, A.c3);
                w[j][0] = r.x; w[j][1] = r.y; w[j][2] = r.z; w[j][3] = r.w;
            }
#pragma unroll
            for (int k = 0; k < RPB; ++k) {
                const uint32_t rho = blk * RPB + k;
                uint32_t field[CPT];
#pragma unroll
                for (int j = 1; j < CPT; ++j) field[j] = block_field<FL>(w[j], k);
                const bool has_next = rho + 1u < A.rounds;
                uint32_t f16n = 0u;
                if (k == RPB - 1) {
                    if (has_next) {
                        const u32x4 r = philox4x32_10_lane(A.key0, A.key1, blk + 1u, cell[0], tile, A.c3);
                        w0[0] = r.x; w0[1] = r.y; w0[2] = r.z; w0[3] = r.w;
                    }
                    field[0] = block_field<FL>(w0, 0);
                } else {
                    field[0] = block_field<FL>(w0, k + 1 < RPB ? k + 1 : 0);
                }
                if (has_next) f16n = next_block_field(A, bd, rho + 1u, tile);
                db_columns_round<ACCEPT, CPT>(A, lds, cpos, flags, top, field, f16, f16n, has_next, rho, tile, offx,
                                              offy, base_u, base_v, cell, below_lane, border, rsrc);
                f16 = f16n;
            }
        }
    }
    copy_window<false>(A, lds, orig, X0 >> 5, Y0 >> 2);
}

// Largest device-step workgroup: 512 lanes (two cells each for 1024-cell
// domains), used when a step has few tiles, so that more lanes share them.
constexpr int kMaxStepThreads = 512;

// Without acceptance draws and with at most 4 cells per lane the kernel fits
// 80 VGPRs and so six waves per SIMD (its LDS, sized as step_lds_bytes with
// one slot per lane, allows six workgroups per compute unit): 5 % faster at
// p = 1.  With acceptance draws 80 VGPRs would spill, and five waves it is.
template <bool ACCEPT, int CPT, int FL>
__global__ void __launch_bounds__(kMaxStepThreads) __attribute__((amdgpu_waves_per_eu(!ACCEPT && CPT <= 4 ? 6 : 1)))
step_db_columns_kernel(StepArgs A)
{
    extern __shared__ uint32_t smem[];
    sweep_db_columns<ACCEPT, CPT, FL>(A, smem, blockIdx.x);
}

// One device step of a single lattice: one workgroup per tile.  With more
// than one cell per lane the workgroup shape divides the domain's cells
// exactly; one cell per lane may leave lanes idle.
template <int SCHEME, bool ACCEPT, int CPT>
__global__ void __launch_bounds__(kMaxStepThreads) step_kernel(StepArgs A)
{
    extern __shared__ uint32_t smem[];
    sweep_tile<SCHEME, ACCEPT, CPT, (CPT > 1)>(A, smem, blockIdx.x);
}

// ---------------------------------------------------------------- measurement
// Heights (gauge h(0,0) = 0): h(0,y) = sum_{y'=1..y} (2 sy[0,y'] - 1);
// h(x,y) = h(0,y) + sum_{x'=1..x} (2 sx[x',y] - 1).

// Column-0 bits of band b: bit r = sy of row 4b + r at x = 0 (the sy words
// of the band's block 0).
__device__ __forceinline__ uint32_t col0_bits(const uint32_t *__restrict__ words, uint32_t nbx_log2, uint32_t b)
{
    const uint4 sy = *reinterpret_cast<const uint4 *>(words + ((static_cast<uint64_t>(b) << nbx_log2) << 3) + 4);
    return (sy.x & 1u) | (sy.y & 1u) << 1 | (sy.z & 1u) << 2 | (sy.w & 1u) << 3;
}

// Column-0 anchors h(0,y) in one workgroup: each thread owns a run of up to 32
// consecutive bands (L <= 2^17 with 1024 threads) whose column-0 bits it
// holds in registers (bit 4k + r: row r of the run's band k, from `fetch(b)`,
// eight fetches in flight at a time); a block scan joins the runs and each
// thread writes its rows' heights, four at a time.
template <typename Fetch>
__device__ __forceinline__ void anchors_scan(Fetch fetch, uint32_t L, int32_t *__restrict__ h0, int32_t *part)
{
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    const uint32_t nband = L >> 2;
    const uint32_t chunk = (nband + T - 1) / T;  // at most 32
    const uint32_t b0 = tid * chunk;
    const uint32_t nb = b0 < nband ? min(chunk, nband - b0) : 0u;
    uint32_t bits[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (uint32_t g = 0; g < 4; ++g) {
        if (8u * g >= nb) break;
        uint32_t v = 0u;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
            const uint32_t k = 8u * g + i;
            if (k < nb) v |= fetch(b0 + k) << (4u * i);
        }
        bits[g] = v;
    }
    // height change over the run: +1 per bit, -1 per row, row 0 of the lattice has no step
    int32_t local = 2 * (int32_t)(__popc(bits[0]) + __popc(bits[1]) + __popc(bits[2]) + __popc(bits[3])) -
                    4 * (int32_t)nb;
    if (b0 == 0u && nb > 0u) local -= 2 * (int32_t)(bits[0] & 1u) - 1;
    part[tid] = local;
    __syncthreads();
    for (uint32_t off = 1; off < T; off <<= 1) {  // inclusive Hillis-Steele scan
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t h = part[tid] - local;  // exclusive prefix: h(0, 4 b0 - 1)
#pragma unroll
    for (uint32_t g = 0; g < 4; ++g) {
        if (8u * g >= nb) break;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
            const uint32_t k = 8u * g + i;
            if (k < nb) {
                const uint32_t nib = bits[g] >> (4u * i);
                int4 hv;
                hv.x = (b0 + k == 0u) ? h : h + 2 * (int32_t)(nib & 1u) - 1;
                hv.y = hv.x + 2 * (int32_t)((nib >> 1) & 1u) - 1;
                hv.z = hv.y + 2 * (int32_t)((nib >> 2) & 1u) - 1;
                hv.w = hv.z + 2 * (int32_t)((nib >> 3) & 1u) - 1;
                h = hv.w;
                *reinterpret_cast<int4 *>(h0 + 4u * (b0 + k)) = hv;
            }
        }
    }
}

// Anchors straight from the lattice words (the batch: one workgroup per member).
__device__ __forceinline__ void anchors_body(const uint32_t *__restrict__ words, uint32_t L, uint32_t nbx_log2,
                                             int32_t *__restrict__ h0, int32_t *part)
{
    anchors_scan([&](uint32_t b) { return col0_bits(words, nbx_log2, b); }, L, h0, part);
}

// A single lattice in two launches: the column-0 bits of every band, one
// lane per band across the whole device (one 16-byte read per band, L/4 of
// them 32 L bytes apart: spread over many compute units rather than queued in
// one), one byte per band into col0; then the scan, in one workgroup, over
// those L/4 contiguous bytes.
static __global__ void __launch_bounds__(256) col0_kernel(const uint32_t *__restrict__ words, uint32_t L,
                                                          uint32_t nbx_log2, uint8_t *__restrict__ col0)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < (L >> 2)) col0[b] = (uint8_t)col0_bits(words, nbx_log2, b);
}

static __global__ void __launch_bounds__(1024) anchors_kernel(const uint8_t *__restrict__ col0, uint32_t L,
                                                              int32_t *__restrict__ h0)
{
    __shared__ int32_t part[1024];
    anchors_scan([&](uint32_t b) { return (uint32_t)col0[b]; }, L, h0, part);
}

// Exclusive prefix sum over the 64 lanes of a wave and the wave's total, by
// data-parallel-primitive moves: shifts by 1, 2, 4, 8 within rows of 16
// lanes (lanes shifted in from outside the row read 0), then the last lane of
// row 0 into rows 1 and 3 and the last lane of row 1 into rows 2 and 3.
__device__ __forceinline__ int32_t wave_excl_scan_i32(int32_t v, int32_t &total)
{
    int32_t inc = v;
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x111, 0xF, 0xF, true);  // row_shr:1
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x112, 0xF, 0xF, true);  // row_shr:2
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x114, 0xF, 0xF, true);  // row_shr:4
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x118, 0xF, 0xF, true);  // row_shr:8
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    total = __builtin_amdgcn_readlane(inc, 63);
    return inc - v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int kMomentFields = 6;  // S1_even, S1_odd, S2_even, S2_odd, S_ts, slope overlap

// Offset-byte tables of a byte b of a block row (8 sites, bit j = slope bit
// of site j; P_j = number of 1 bits among bits 0 .. j), two words per entry,
// byte j of the pair = the offset height of site j (see row_offsets):
//   lut[2 b], lut[2 b + 1]               first byte of a row: 2 P_j + 63 - j
//   lut[512 + 2 b], lut[512 + 2 b + 1]   later bytes: 2 P_j + 7 - j, the
//                                        offsets relative to the previous
//                                        byte's last one, plus 8
constexpr uint32_t kLutWords = 1024;

__device__ void build_tables(uint32_t *lut)
{
    for (uint32_t b = threadIdx.x; b < 256; b += blockDim.x) {
        uint32_t acc = 0, first[2] = {0u, 0u}, rest[2] = {0u, 0u};
        for (uint32_t j = 0; j < 8; ++j) {
            acc += (b >> j) & 1u;
            first[j >> 2] |= (2u * acc + 63u - j) << (8 * (j & 3));
            rest[j >> 2] |= (2u * acc + 7u - j) << (8 * (j & 3));
        }
        lut[2 * b] = first[0];
        lut[2 * b + 1] = first[1];
        lut[512 + 2 * b] = rest[0];
        lut[512 + 2 * b + 1] = rest[1];
    }
}

constexpr int kMeasureThreads = 256;

// One row of one 32-site block, bit i = slope bit of site x0 + i (x0 a
// multiple of 32).  Relative heights q_i = sum_{j <= i} (2 b_j - 1) (for the
// lattice's first block site 0 has no step: b_0 is cleared and q_i =
// sum_{1 <= j <= i} (2 b_j - 1)) are formed four at a time as offset bytes
// u_i = q_i + 64 = 2 P_i + 63 - i in [32, 96] (+1 in the first block), P_i
// the number of 1 bits among bits 0 .. i: the row's first byte straight from
// its table entry, each later byte as its table entry (relative offsets + 8)
// plus the previous byte's last offset broadcast to every byte, minus 8 --
// one permute and two three-input adds per byte; no byte sum carries or
// borrows.  Returns q_31, the block's height change; U[k] keeps the bytes of
// nibble k for a cross product.  MOM: byte dot products give the sums of u
// (s1e, s1o) and of u^2 (added to s2e, s2o) over the sites of each parity
// class, each class's bytes of two nibbles gathered into one word by one
// permute.  MOM = false: s1e = the sum of u over all sites (what a snapshot
// row needs), the other outputs untouched.  FIRST: the chunk holding the
// lattice's first block, in lane 0 (the only lane that takes the
// first-block path).
template <int R, bool MOM, bool FIRST>
__device__ __forceinline__ int32_t row_offsets(const uint32_t *lut, uint32_t w, uint32_t (&U)[8], uint32_t &s1e,
                                               uint32_t &s1o, uint32_t &s2e, uint32_t &s2o)
{
    const bool f = FIRST && (threadIdx.x & 63u) == 0u;
    // parity class "even" (x + y even): even i on even rows, odd i on odd rows;
    // bytes (m, m + 2) of nibbles k and k + 1 (permute selectors: 0-3 pick bytes
    // of the second operand, 4-7 of the first)
    constexpr uint32_t sel_e = (R & 1) ? 0x07050301u : 0x06040200u;
    constexpr uint32_t sel_o = (R & 1) ? 0x06040200u : 0x07050301u;
    if (f) w &= ~1u;
    // the u^2 chains continue the caller's sums
    uint32_t prev = 0u, a1 = 0u, b1 = 0u, a2 = s2e, b2 = s2o;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        // byte offset of the table entry
        const uint32_t off = m == 0 ? byte0_x8(w) : ((w >> (8 * m)) & 0xFFu) << 3;
        const uint2 e = *reinterpret_cast<const uint2 *>(reinterpret_cast<const char *>(lut) + (m ? 2048u : 0u) + off);
        uint32_t u0, u1;
        if (m == 0) {
            const uint32_t dl = f ? 0x01010101u : 0u;
            u0 = e.x + dl;
            u1 = e.y + dl;
        } else {
            const uint32_t bp = __builtin_amdgcn_perm(prev, prev, 0x07070707u);  // u_{8m-1} in every byte
            u0 = add3(e.x, bp, 0u - 0x08080808u);
            u1 = add3(e.y, bp, 0u - 0x08080808u);
        }
        prev = u1;
        U[2 * m] = u0;
        U[2 * m + 1] = u1;
        if (MOM) {
            const uint32_t ev = __builtin_amdgcn_perm(u1, u0, sel_e);
            const uint32_t od = __builtin_amdgcn_perm(u1, u0, sel_o);
            a1 = __builtin_amdgcn_udot4(ev, 0x01010101u, a1, false);
            b1 = __builtin_amdgcn_udot4(od, 0x01010101u, b1, false);
            a2 = __builtin_amdgcn_udot4(ev, ev, a2, false);
            b2 = __builtin_amdgcn_udot4(od, od, b2, false);
        } else {
            a1 = __builtin_amdgcn_udot4(u0, 0x01010101u, a1, false);
            a1 = __builtin_amdgcn_udot4(u1, 0x01010101u, a1, false);
        }
    }
    s1e = a1;
    if (MOM) {
        s1o = b1;
        s2e = a2;
        s2o = b2;
    }
    return (int32_t)(prev >> 24) - 64;  // u_31 - 64 = q_31
}

// One wave: the moments of band `band` of one lattice into out[0..5].  Lane l
// handles block l of each chunk of 64 blocks (32 sites of each of the band's
// 4 rows); a wave scan of the blocks' height changes gives each block's
// starting height A.  With q the relative heights of a block row (16 sites
// per parity class), sum h = 16 A + sum q and sum h^2 = 2 A (8 A + sum q) +
// sum q^2 per class; the A-dependent parts are accumulated per row in 64 bits,
// the sums of u and u^2 (A-independent) in 32 bits and turned into sums of q
// and q^2 at the end (q = u - 64).  With a snapshot (CROSS), sum h_t h_s =
// A_t (32 A_s + sum q_s) + A_s sum q_t + sum q_t q_s over the block row, and
// the slope overlap (slope variables that are 1 in both states, for the slope
// autocorrelation C_s) is a population count of the ANDed words.
template <bool CROSS>
__device__ __forceinline__ void rows_band(const uint32_t *lut, const uint32_t *__restrict__ words,
                                          const int32_t *__restrict__ h0, const uint32_t *__restrict__ snap,
                                          const int32_t *__restrict__ h0s, uint32_t band, uint32_t nbx_log2,
                                          int64_t *__restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nbx = 1u << nbx_log2;
    const uint64_t band_base = (static_cast<uint64_t>(band) << nbx_log2) << 3;
    int32_t carry[4] = {0, 0, 0, 0}, carry_s[4] = {0, 0, 0, 0};
    int32_t h0r[4], h0sr[4] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        h0r[r] = h0[4 * band + r];
        if (CROSS) h0sr[r] = h0s[4 * band + r];
    }
    // per class and block row, sum h = 16 A + sum q and sum h^2 = 16 A^2 +
    // 2 A sum q + sum q^2: the A-terms summed over the lane's rows as sum A,
    // sum A^2 and sum A sum u_class (q = u - 64).  |A| <= L <= 2^17 on the
    // periodic surface (gauge h(0,0) = 0) and a lane has at most 4 L/2048
    // block rows of a band, so sum A stays below 2^25
    int32_t sa = 0;
    int64_t aa = 0, au_e = 0, au_o = 0, xa = 0;
    uint32_t u2e = 0, u2o = 0, ue = 0, uo = 0, us_all = 0, uts = 0;
    uint32_t rows = 0;      // block rows this lane took part in
    uint32_t overlap = 0;   // at most 8 L per band
    // one chunk of 64 blocks; FIRST: the band's first chunk, whose lane 0
    // holds the lattice's first block (site 0 without a step)
    // FULL: every lane of the chunk holds a block (bands of at least 64 blocks)
    auto chunk = [&](uint32_t base, auto first_c, auto full_c) {
        constexpr bool FIRST = decltype(first_c)::value;
        constexpr bool FULL = decltype(full_c)::value;
        const uint32_t bx = base + lane;
        const bool active = FULL || bx < nbx;
        uint4 wv = make_uint4(0, 0, 0, 0), sv = make_uint4(0, 0, 0, 0);
        if (active) {
            wv = *reinterpret_cast<const uint4 *>(words + band_base + 8u * bx);  // sx rows 0..3
            if (CROSS) {
                sv = *reinterpret_cast<const uint4 *>(snap + band_base + 8u * bx);
                const uint4 wy = *reinterpret_cast<const uint4 *>(words + band_base + 8u * bx + 4u);  // sy rows
                const uint4 sy = *reinterpret_cast<const uint4 *>(snap + band_base + 8u * bx + 4u);
                overlap += __popc(wv.x & sv.x) + __popc(wv.y & sv.y) + __popc(wv.z & sv.z) + __popc(wv.w & sv.w) +
                           __popc(wy.x & sy.x) + __popc(wy.y & sy.y) + __popc(wy.z & sy.z) + __popc(wy.w & sy.w);
            }
        }
        const uint32_t wk[4] = {wv.x, wv.y, wv.z, wv.w};
        const uint32_t sk[4] = {sv.x, sv.y, sv.z, sv.w};
        auto one_row = [&](auto rc) {
            constexpr int r = decltype(rc)::value;
            uint32_t U[8], Us[8];
            uint32_t se = 0, so = 0, sus = 0, unused = 0;
            // the u^2 sums go straight into the lane's totals when every lane
            // holds a block, else through the row's own (added if active)
            uint32_t t2e = 0, t2o = 0;
            uint32_t &d2e = FULL ? u2e : t2e, &d2o = FULL ? u2o : t2o;
            int32_t R = row_offsets<r, true, FIRST>(lut, wk[r], U, se, so, d2e, d2o);
            int32_t Rs = 0;
            if (CROSS) Rs = row_offsets<r, false, FIRST>(lut, sk[r], Us, sus, unused, unused, unused);
            if (!active) R = Rs = 0;  // lanes past the end of a short band add nothing
            int32_t ex, tot, exs = 0, tot_s = 0;
            if (CROSS) {
                // both scans in one: R + 64 and Rs + 64 (R in [-32, 33]) in the
                // two halves of a word, whose sums over 64 lanes stay below 2^16
                const uint32_t pk = (uint32_t)(R + 64) | ((uint32_t)(Rs + 64) << 16);
                int32_t totp;
                const uint32_t exp = (uint32_t)wave_excl_scan_i32((int32_t)pk, totp);
                const int32_t off = 64 * (int32_t)lane;
                ex = (int32_t)(exp & 0xFFFFu) - off;
                exs = (int32_t)(exp >> 16) - off;
                tot = (int32_t)((uint32_t)totp & 0xFFFFu) - 4096;
                tot_s = (int32_t)((uint32_t)totp >> 16) - 4096;
            } else {
                ex = wave_excl_scan_i32(R, tot);
            }
            const int32_t A = h0r[r] + carry[r] + ex;  // height before the block
            carry[r] += tot;
            int32_t As = 0;
            if (CROSS) {
                As = h0sr[r] + carry_s[r] + exs;
                carry_s[r] += tot_s;
            }
            if (active) {
                sa += A;
                aa += (int64_t)A * A;
                au_e += (int64_t)A * (int32_t)se;
                au_o += (int64_t)A * (int32_t)so;
                if (!FULL) {
                    u2e += t2e;
                    u2o += t2o;
                }
                ue += se;
                uo += so;
                rows += 1;
                if (CROSS) {
                    // sum u_t u_s, chained straight into the lane's total
                    uint32_t x = uts;
#pragma unroll
                    for (int k = 0; k < 8; ++k) x = __builtin_amdgcn_udot4(U[k], Us[k], x, false);
                    uts = x;
                    us_all += sus;
                    xa += (int64_t)A * (32 * As + ((int32_t)sus - 2048)) + (int64_t)As * ((int32_t)(se + so) - 2048);
                }
            }
        };
        one_row(std::integral_constant<int, 0>());
        one_row(std::integral_constant<int, 1>());
        one_row(std::integral_constant<int, 2>());
        one_row(std::integral_constant<int, 3>());
    };
    if (nbx >= 64u) {  // nbx is a power of two: whole chunks only
        chunk(0u, std::true_type(), std::true_type());
        for (uint32_t base = 64; base < nbx; base += 64) chunk(base, std::false_type(), std::true_type());
    } else {
        chunk(0u, std::true_type(), std::false_type());
    }
    // sums of q and q^2 from those of u = q + 64 (16 sites per class per block row)
    const int64_t n16 = 16 * (int64_t)rows;
    int64_t s1e = 16 * (int64_t)sa + (int64_t)ue - 64 * n16;
    int64_t s1o = 16 * (int64_t)sa + (int64_t)uo - 64 * n16;
    int64_t s2e = 16 * aa + 2 * (au_e - 1024 * (int64_t)sa) + ((int64_t)u2e - 128 * (int64_t)ue + 4096 * n16);
    int64_t s2o = 16 * aa + 2 * (au_o - 1024 * (int64_t)sa) + ((int64_t)u2o - 128 * (int64_t)uo + 4096 * n16);
    int64_t sts = 0;
    if (CROSS) sts = xa + ((int64_t)uts - 64 * ((int64_t)ue + uo + us_all) + 4096 * 2 * n16);
    s1e = wave_sum_i64(s1e);
    s1o = wave_sum_i64(s1o);
    s2e = wave_sum_i64(s2e);
    s2o = wave_sum_i64(s2o);
    int64_t ov = 0;
    if (CROSS) {
        sts = wave_sum_i64(sts);
        ov = wave_sum_i64((int64_t)overlap);
    }
    if (lane == 0) {
        out[0] = s1e;
        out[1] = s1o;
        out[2] = s2e;
        out[3] = s2o;
        out[4] = sts;
        out[5] = ov;
    }
}

template <bool CROSS>
__global__ void __launch_bounds__(kMeasureThreads) rows_kernel(const uint32_t *__restrict__ words,
                                                               const int32_t *__restrict__ h0,
                                                               const uint32_t *__restrict__ snap,
                                                               const int32_t *__restrict__ h0s, uint32_t L,
                                                               uint32_t nbx_log2, int64_t *__restrict__ partial)
{
    __shared__ __align__(8) uint32_t lut[kLutWords];
    build_tables(lut);
    __syncthreads();
    const uint32_t band = blockIdx.x * (kMeasureThreads / 64) + (threadIdx.x >> 6);
    if (band >= (L >> 2)) return;
    rows_band<CROSS>(lut, words, h0, snap, h0s, band, nbx_log2,
                     partial + static_cast<uint64_t>(band) * kMomentFields);
}

// 128-bit signed accumulate (two's complement in (lo, hi)).
__device__ __forceinline__ void add_i128(uint64_t &lo, int64_t &hi, uint64_t blo, int64_t bhi)
{
    const uint64_t nlo = lo + blo;
    hi += bhi + (nlo < lo ? 1 : 0);
    lo = nlo;
}

// Final exact reduction of the per-row partials into 128-bit totals, one
// workgroup of up to 1024 lanes: each lane accumulates rows tid, tid + T, ...
// (the six fields of a row are one 48-byte record; four rows in flight), a
// wave sums its lanes by shuffles, and the first lanes add the waves'.
constexpr int kReduceMaxWaves = 16;

__device__ __forceinline__ void reduce_body(const int64_t *__restrict__ partial, uint32_t nrows,
                                            int64_t *__restrict__ out, uint64_t (*lo_s)[kReduceMaxWaves],
                                            int64_t (*hi_s)[kReduceMaxWaves])
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = blockDim.x >> 6;
    uint64_t lo[kMomentFields];
    int64_t hi[kMomentFields];
#pragma unroll
    for (int f = 0; f < kMomentFields; ++f) {
        lo[f] = 0;
        hi[f] = 0;
    }
#pragma unroll 4
    for (uint32_t r = tid; r < nrows; r += blockDim.x) {
        const int64_t *row = partial + static_cast<uint64_t>(r) * kMomentFields;
#pragma unroll
        for (int f = 0; f < kMomentFields; ++f) add_i128(lo[f], hi[f], static_cast<uint64_t>(row[f]), row[f] < 0 ? -1 : 0);
    }
#pragma unroll
    for (int f = 0; f < kMomentFields; ++f) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t olo = __shfl_xor(lo[f], off, 64);
            const int64_t ohi = __shfl_xor(hi[f], off, 64);
            add_i128(lo[f], hi[f], olo, ohi);
        }
        if (lane == 0) {
            lo_s[f][wave] = lo[f];
            hi_s[f][wave] = hi[f];
        }
    }
    __syncthreads();
    if (tid < kMomentFields) {
        uint64_t tlo = 0;
        int64_t thi = 0;
        for (uint32_t w = 0; w < nwaves; ++w) add_i128(tlo, thi, lo_s[tid][w], hi_s[tid][w]);
        out[2 * tid] = static_cast<int64_t>(tlo);
        out[2 * tid + 1] = thi;
    }
}

constexpr int kReduceThreads = 1024;

static __global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const int64_t *__restrict__ partial,
                                                                       uint32_t nrows, int64_t *__restrict__ out)
{
    __shared__ uint64_t lo_s[kMomentFields][kReduceMaxWaves];
    __shared__ int64_t hi_s[kMomentFields][kReduceMaxWaves];
    reduce_body(partial, nrows, out, lo_s, hi_s);
}

}  // namespace okpz
