// DB device step on a row-paired LDS window (the benchmark shapes: square
// domains of 128 or 256 sites, 8 x 8-site thread cells, at least two cells
// per lane).  Same attempts, random draws and delayed-border order as
// sweep_db_columns (Sec. 3 DB, Sec. 3.1 single hit); what changes is how an
// attempt finds and tests its site:
//
//  * Window layout.  Row r of the staged window keeps its sx words at
//    r * W + k and its sy words at r * W + P + k (k = 0 .. NWX-1, block k of
//    the window; row pitch W >= 2P + 1 words), so the four slope words an
//    attempt reads -- sx(x, y), sx(x+1, y), sy(x, y), sy(x, y+1) -- sit at
//    one address plus the immediate offsets 0, 1, P and P + W words (two
//    ds_read2 instructions, one address).  P, W and everything else sized by
//    the domain are compile-time.
//  * A site is one linear index s = ly * 32W + lx (ly, lx: window row and
//    column): the byte address of its sx word is (s >> 3) & ~3, its bit is
//    s mod 32 (the shift instructions read only the low five bits), and the
//    sites to the right and below are s + 1 and s + 32W, which is all the
//    delayed-border dependency checks compare.
//  * Acceptance is decided after the slopes are read: whether the site is a
//    local minimum or maximum is tested on the four slope words at once (two
//    three-input bit operations; the site's bit of the result is then
//    extracted), and only a local minimum (deposition, threshold P) or a
//    local maximum (removal, threshold Q) is compared with its acceptance
//    prefix, and the 32-bit tie-break draw is
//    made only when that prefix equals the threshold's top bits -- for an
//    attempt that can flip.  The variate and its thresholds are those of the
//    generic kernels (U = prefix * 2^32 + r against P or Q), so the outcome
//    of every attempt is the same; ties that cannot matter are just not
//    drawn.
#pragma once

#include "kernels.hpp"

namespace okpz {

// Compile-time geometry of a square D x D domain (LD = log2 D >= 5) with
// C x C-site cells (LC = log2 C): the same window as window_shape() on the
// host (NWX blocks, NB bands).  WIDE: the DT / DTr step's row pitch (below).
template <int LD, int LC, bool WIDE = false>
struct RowPairShape {
    static constexpr uint32_t D = 1u << LD;
    static constexpr uint32_t C = 1u << LC;
    static constexpr uint32_t NWX = D / 32 + 1;
    // the sy words of a row start right after its sx words: an attempt also
    // reads the word after its sx word, which for the last block is the
    // first sy word -- read but never used or written, since a domain site
    // (window column <= D - 1 + 31) is never bit 31 of the last block
    static constexpr uint32_t P = NWX | 1u;
    static constexpr uint32_t NB = D / 4 + 1;
    static constexpr uint32_t NR = 4 * NB;
    // words per window row (sx words, sy words, padding), chosen against LDS
    // bank conflicts (32 banks; the 32 lanes of a half-wave hold one cell
    // row): 2P + 1 below D = 256.  At D = 256, DT / DTr (WIDE): 24 words,
    // which puts the four rows of a quadrant on the bank offsets 0, 24, 16
    // and 8, so that the eight words a cell row's attempts reach in each of
    // them fall on distinct banks (the window then leaves room for six
    // workgroups per compute unit).  DB: 20 words, which spreads the eight
    // rows of a cell over the bank offsets 0, 20, 8, 28, 16, 4, 24, 12, and
    // keeps the window and the published sites of 256 lanes within a
    // seventh of the compute unit's LDS (a 24-word pitch would cost DB the
    // seventh workgroup, and more time than its fewer conflicts save).
    static constexpr uint32_t PITCH = LD == 8 ? (WIDE ? 24u : 20u) : 2 * P + 1;
    static_assert(PITCH >= 2 * P + 1, "a row holds its sx and sy words");
    static constexpr uint32_t ROW = 32 * PITCH;      // bits per window row (linear site index stride)
    static constexpr uint32_t NCX = D / C;           // cells per domain row
    static constexpr uint32_t LOG2NCX = LD - LC;
    static constexpr uint32_t SBITS = 2 * LC;        // site-index bits of a lane draw
    static constexpr uint32_t WORDS = NR * PITCH;    // window words
};

// LDS words of a row-paired workgroup with nt lanes: the window, two
// buffers of published top-cell sites, three round flags.
template <int LD, int LC>
__host__ __device__ constexpr uint32_t rowpair_lds_words(uint32_t nt)
{
    return RowPairShape<LD, LC>::WORDS + 2u * nt + 4u;
}

// Staging of the window (see copy_window) into / out of the row-paired layout.
template <bool LOAD, uint32_t P, uint32_t PITCH>
__device__ __forceinline__ void copy_window_rows(const StepArgs &A, uint32_t *lds, uint32_t bx0, uint32_t by0)
{
    const uint32_t nwaves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    for (uint32_t b = wave; b < A.NB; b += nwaves) {
        const uint64_t band = static_cast<uint64_t>((by0 + b) & A.nby_mask) << A.nbx_log2;
        for (uint32_t t = lane; t < 8u * A.NWX; t += 64) {
            const uint32_t k = t >> 3, wib = t & 7u, row = 4u * b + (wib & 3u);
            const uint64_t g = ((band + ((bx0 + k) & A.nbx_mask)) << 3) + wib;
            const uint32_t li = row * PITCH + (wib >> 2) * P + k;
            if (LOAD)
                lds[li] = A.words[g];
            else
                A.words[g] = lds[li];
        }
    }
}

// One attempt at linear site s (Sec. 2.1 rule; acceptance of Sec. 2.1's
// rates as described above).  pre: the attempt's acceptance prefix (ACCEPT).
// enable: false for attempts that run in a later pass.  rho, cell, tile:
// the counters of the tie-break draw.
// A word of the workgroup's LDS by its LDS byte address.
using lds_word = __attribute__((address_space(3))) uint32_t;

__device__ __forceinline__ lds_word *lds_at(uint32_t byte_addr)
{
    return reinterpret_cast<lds_word *>(static_cast<uintptr_t>(byte_addr));
}

// LDS byte address of a pointer into the workgroup's LDS (0 for the dynamic
// LDS of a kernel without static LDS).
__device__ __forceinline__ uint32_t lds_address(const uint32_t *p)
{
    // a C-style cast is the address-space conversion
    const __attribute__((address_space(3))) uint32_t *q = (const __attribute__((address_space(3))) uint32_t *)p;
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(q));
}

// (a << sh) | b in one instruction (the compiler otherwise folds two such
// terms into a three-input OR after two separate shifts).
__device__ __forceinline__ uint32_t lshl_or(uint32_t a, uint32_t sh, uint32_t b)
{
    uint32_t r;
    asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(sh), "v"(b));
    return r;
}

// a * b + c with a, b 24-bit signed (b uniform), as one instruction
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// f(a, b, c) bit by bit, f given by its truth table TT (bit 4a + 2b + c)
template <uint32_t TT>
__device__ __forceinline__ uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:%4" : "=v"(r) : "v"(a), "v"(b), "v"(c), "i"(TT));
    return r;
}

// 1 << (s mod 32) and 3 << (s mod 32), the flip masks of sx(x) and of
// sx(x), sx(x+1) (shift instructions read the low five bits of s); written
// as instructions so that the test for x = bit 31 stays one compare.
__device__ __forceinline__ void flip_masks(uint32_t s, uint32_t &m1, uint32_t &m3)
{
    asm("v_lshlrev_b32 %0, %1, 1" : "=v"(m1) : "v"(s));
    asm("v_lshlrev_b32 %0, %1, 3" : "=v"(m3) : "v"(s));
}

template <bool ACCEPT, uint32_t P, uint32_t PITCH>
__device__ __forceinline__ void attempt_rows(const StepArgs &A, uint32_t s, uint32_t pre, bool enable, uint32_t rho,
                                             uint32_t cell, uint32_t tile)
{
    lds_word *px = lds_at((s >> 3) & ~3u);
    const uint32_t w0 = px[0], w1 = px[1];
    const uint32_t y0 = px[P], y1 = px[P + PITCH];
    const uint32_t d = __builtin_amdgcn_ubfe(y1, s, 1);
    bool flip;
    if (ACCEPT) {
        // bit s of mm: the slopes (sx(x), sx(x+1), sy(x,y), sy(x,y+1)) are
        // (a, 1-a, a, 1-a), a local minimum (a = 0) or maximum (a = 1); e has
        // sx(x+1) at the bit of x.  Two three-input operations:
        // (e ^ w0) & ~(w0 ^ y0), then that & (y0 ^ y1).
        const uint32_t e = __builtin_amdgcn_alignbit(w1, w0, 1u);
        const uint32_t mm = bitop3<0x60>(bitop3<0x18>(e, w0, y0), y0, y1);
        // a minimum has sy(x,y+1) = 1, a maximum 0: the prefix is compared
        // with P_hi when d = 1, with Q_hi when d = 0, i.e. pre - d (P_hi - Q_hi)
        // with Q_hi (signed: the shifted prefix can be negative); an attempt
        // at neither compares INT_MAX instead
        const int sel = __builtin_amdgcn_sbfe((int)mm, s, 1);  // -1 or 0
        const int rel = mad_i24((int)d, -A.pq_delta, (int)pre);
        const int t = (rel & sel) | (0x7fffffff & ~sel);
        flip = enable && t < (int)A.Q_hi;
        if (enable && t == (int)A.Q_hi) {  // the prefix ties: the low 32 bits of the variate decide
            // the tie counter formed here, where the rare branch runs: as a
            // loop-invariant value the compiler would keep its first Philox
            // products in registers for the whole sweep
            uint32_t c1;
            asm volatile("v_or_b32 %0, 0x80000000, %1" : "=v"(c1) : "v"(cell));
            const uint32_t r = philox4x32_10_lane(A.key0, A.key1, rho, c1, tile, A.c3).x;
            flip = r < (d ? A.P_lo : A.Q_lo);
        }
    } else {
        // pattern index: bit 3 sx(x+1,y), bit 2 sx(x,y), bit 1 sy(x,y), bit 0
        // sy(x,y+1); bit 4 holds a further sx bit (the masks repeat at +16)
        const uint32_t ab = __builtin_amdgcn_alignbit(w1, w0, s);
        const uint32_t key = lshl_or(ab, 2, lshl_or(__builtin_amdgcn_ubfe(y0, s, 1), 1, d));
        flip = enable && __builtin_amdgcn_ubfe(A.flip_table, key, 1) != 0u;
    }
    if (flip) {
        uint32_t m1, m3;
        flip_masks(s, m1, m3);
        __hip_atomic_fetch_xor(&px[0], m3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);      // sx(x), sx(x+1)
        __hip_atomic_fetch_xor(&px[P], m1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);      // sy(x, y)
        __hip_atomic_fetch_xor(&px[P + PITCH], m1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  // sy(x, y+1)
        if (m3 == 0x80000000u)  // x is bit 31: sx(x+1) is bit 0 of the next word
            __hip_atomic_fetch_xor(&px[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// (du + cu) mod D, the column of a draw in the shifted cell grid; at D = 256
// one byte-select add (the sum's low byte, the other bytes cleared).
template <int LD>
__device__ __forceinline__ uint32_t wrap_column(uint32_t du, uint32_t cu)
{
    if constexpr (LD == 8) {
        uint32_t r;
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:BYTE_0 dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:DWORD"
            : "=v"(r) : "v"(du), "v"(cu));
        return r;
    } else {
        return (du + cu) & ((1u << LD) - 1u);
    }
}

// Linear site of a DB lane draw: site (du, dv) = (field mod C, field / C mod
// C) of the cell whose corner, with the round's cell-grid shift, is
// (cu, cv) -- both wrap around the domain (Sec. 3.1 DB: the shifted cell grid
// is periodic on the domain); origin = the linear index of domain site
// (0, 0), counted from LDS address 0.
// wrapv = false: the caller knows the row cannot pass the domain's last row
// (only cells of the last cell row can wrap vertically).
template <int LD, int LC>
__device__ __forceinline__ uint32_t site_rows(uint32_t field, uint32_t cu, uint32_t cv, uint32_t origin,
                                              bool wrapv)
{
    using S = RowPairShape<LD, LC>;
    const uint32_t du = field & (S::C - 1u);
    const uint32_t dv = (field >> LC) & (S::C - 1u);
    const uint32_t u = wrap_column<LD>(du, cu);
    const uint32_t v = wrapv ? (dv + cv) & (S::D - 1u) : dv + cv;
    return __umul24(v, S::ROW) + u + origin;
}

// The same site for a cell that cannot reach past the domain's last row,
// with the round's row base rb = cv ROW + origin (cv: the corner row of the
// lane's top cell with the round's shift) and the cell's row offset voff
// below that corner: s = (dv + voff) ROW + u + rb.
template <int LD, int LC>
__device__ __forceinline__ uint32_t site_rows_nowrap(uint32_t field, uint32_t cu, uint32_t rb, uint32_t voff)
{
    using S = RowPairShape<LD, LC>;
    const uint32_t du = field & (S::C - 1u);
    const uint32_t dv = (field >> LC) & (S::C - 1u);
    return mad24(dv, S::ROW, wrap_column<LD>(du, cu)) + rb + voff * S::ROW;
}

// DB device step with each lane holding a column of CPT vertically stacked
// cells (lane t: cells (t mod NCX, CPT (t / NCX) + j), j = 0 .. CPT-1, j = 0
// on top), as in sweep_db_columns: the top cell is drawn one round ahead
// and its site published for the column above; the cell below is read from
// the same lane (the bottom cell: the published top cell of the column
// below), the cell to the right from the neighbouring lane by a cross-lane
// permute; deferred attempts run in their own wave after the first pass
// (edges, then corners) unless they are remote (bottom row of a bottom cell
// whose column below is in another wave), which run after the barrier.  The
// lane-draw fields are 2^FL bits, the rounds of one Philox block unrolled.
template <bool ACCEPT, int CPT, int LD, int LC>
__device__ __forceinline__ void sweep_db_rows(const StepArgs &A, uint32_t *smem, uint32_t tile)
{
    using S = RowPairShape<LD, LC>;
    constexpr int FL = ACCEPT ? 4 : 3;  // 16-bit fields with acceptance prefixes, 8-bit without
    constexpr uint32_t F = 1u << FL;
    constexpr int RPB = 128 >> FL;      // rounds per Philox block
    constexpr uint32_t P = S::P;
    constexpr uint32_t CM = S::C - 1u;
    static_assert(S::SBITS + (ACCEPT ? 8 : 0) <= F, "field too narrow");
    static_assert(CPT >= 2 && S::NCX <= 64, "a wave must hold whole rows of lanes");
    const uint32_t tid = threadIdx.x, NT = blockDim.x;
    uint32_t *lds = smem;                     // window (row-paired)
    uint32_t *cpos = smem + S::WORDS;         // 2 x NT published top-cell sites
    uint32_t *flags = cpos + 2u * NT;         // 3 round flags

    const uint32_t tx = tile & ((1u << A.log2ntx) - 1u), ty = tile >> A.log2ntx;
    const uint32_t X0 = (A.ox + 2u * S::D * tx + A.set_a * S::D) & A.L_mask;
    const uint32_t Y0 = (A.oy + 2u * S::D * ty + A.set_b * S::D) & A.L_mask;
    // linear index of domain site (0, 0), counted from LDS address 0: the
    // window's own LDS address (a multiple of 4 bytes, so whole words) is
    // 8 bits per byte further on
    const uint32_t origin = (Y0 & 3u) * S::ROW + (X0 & 31u) + 8u * lds_address(lds);

    copy_window_rows<true, P, S::PITCH>(A, lds, X0 >> 5, Y0 >> 2);

    const uint32_t cx = tid & (S::NCX - 1u), grp = tid >> S::LOG2NCX;
    const uint32_t below_lane = (tid + S::NCX) & (NT - 1u);  // lane holding the column below
    const bool border = (below_lane >> 6) != (tid >> 6);     // ... in another wave
    const int rsrc = (int)((cx == S::NCX - 1u ? tid + 1u - S::NCX : tid + 1u) & 63u) << 2;  // column to the right
    const uint32_t base_u = cx << LC;
    const uint32_t base_v0 = (grp * CPT) << LC;               // top cell's corner row
    const uint32_t cell0 = (grp * CPT) * S::NCX + cx;         // top cell's id; cell j = cell0 + j NCX

    // field k of a Philox block, lowest bits first
    auto field_of = [](const uint32_t(&w)[4], int k) -> uint32_t {
        constexpr int FPW = 32 / F;
        return (w[k / FPW] >> (F * (k % FPW))) & ((1u << F) - 1u);
    };
    // the round's cell-grid shift from its block field
    auto shx_of = [](uint32_t f16) { return (f16 >> 2) & CM; };
    auto shy_of = [](uint32_t f16) { return (f16 >> 8) & CM; };
    // rim of an attempt from its field: on its cell's bottom row; on its corner
    // (bottom row and right column: all site-index bits set)
    auto bottom_of = [](uint32_t f) { return (f & (CM << LC)) == (CM << LC); };
    auto corner_of = [](uint32_t f) { return (f & ((1u << S::SBITS) - 1u)) == (1u << S::SBITS) - 1u; };

    BlockDraw bd = {0u, 0u, 0u, 0u};
    uint32_t f16 = next_block_field(A, bd, 0u, tile);
    uint32_t w0[4];  // the top cell's current Philox block
    {
        const u32x4 r = philox4x32_10_lane(A.key0, A.key1, 0u, cell0, tile, A.c3);
        w0[0] = r.x; w0[1] = r.y; w0[2] = r.z; w0[3] = r.w;
    }
    uint32_t ftop = field_of(w0, 0);  // the top cell's field of the coming round
    // the round's row base: the top cell's shifted corner row times the row
    // stride, plus the origin (the lane's part once, the round's shift added
    // as a uniform product)
    const uint32_t rb0 = __umul24(base_v0, S::ROW) + origin;
    uint32_t rb = rb0 + shy_of(f16) * S::ROW;
    uint32_t stop = site_rows_nowrap<LD, LC>(ftop, base_u + shx_of(f16), rb, 0u);
    cpos[tid] = stop;
    if (tid < 3) flags[tid] = 0u;
    __syncthreads();

    const uint32_t nblk = A.rounds / RPB;
    for (uint32_t blk = 0; blk < nblk; ++blk) {
        uint32_t w[CPT][4];
#pragma unroll
        for (int j = 1; j < CPT; ++j) {
            const u32x4 r = philox4x32_10_lane(A.key0, A.key1, blk, cell0 + j * S::NCX, tile, A.c3);
            w[j][0] = r.x; w[j][1] = r.y; w[j][2] = r.z; w[j][3] = r.w;
        }
#pragma unroll
        for (int k = 0; k < RPB; ++k) {
            const uint32_t rho = blk * RPB + k;
            const bool has_next = rho + 1u < A.rounds;
            // this round's fields and sites; the top cell's was drawn last round
            const uint32_t cu = base_u + shx_of(f16), cv = base_v0 + shy_of(f16);
            uint32_t f[CPT], s[CPT];
            f[0] = ftop;
            s[0] = stop;
#pragma unroll
            for (int j = 1; j < CPT; ++j) {
                f[j] = field_of(w[j], k);
                // a lane's lower cells are never in the last cell row but the bottom one
                s[j] = j == CPT - 1 ? site_rows<LD, LC>(f[j], cu, cv + (j << LC), origin, true)
                                    : site_rows_nowrap<LD, LC>(f[j], cu, rb, j << LC);
            }
            // the top cell's attempt of the next round, published for the column above
            uint32_t f16n = 0u, rbn = 0u;
            if (has_next) {
                f16n = next_block_field(A, bd, rho + 1u, tile);
                if (k == RPB - 1) {
                    const u32x4 r = philox4x32_10_lane(A.key0, A.key1, blk + 1u, cell0, tile, A.c3);
                    w0[0] = r.x; w0[1] = r.y; w0[2] = r.z; w0[3] = r.w;
                }
                ftop = field_of(w0, (k + 1) % RPB);
                rbn = rb0 + shy_of(f16n) * S::ROW;
                stop = site_rows_nowrap<LD, LC>(ftop, base_u + shx_of(f16n), rbn, 0u);
                cpos[((rho + 1u) & 1u) * NT + tid] = stop;
            }
            // Delayed-border order dependencies (as in db_columns_round): the
            // attempt of the cell to the right sits on the site right of mine,
            // or the one of the cell below on the site below mine -- which
            // defers mine only if it is in another lane or itself deferred
            // (the first pass runs a lane's cells bottom to top).  Either
            // places mine on its cell's right column / bottom row.
            const uint32_t pbot = cpos[(rho & 1u) * NT + below_lane];
            bool def[CPT];
#pragma unroll
            for (int j = CPT - 1; j >= 0; --j) {
                const uint32_t pr = (uint32_t)__builtin_amdgcn_ds_bpermute(rsrc, (int)s[j]);
                const uint32_t pd = j + 1 < CPT ? s[j + 1 < CPT ? j + 1 : j] : pbot;
                const bool below = pd == s[j] + S::ROW && (j == CPT - 1 || def[j + 1 < CPT ? j + 1 : j]);
                def[j] = pr == s[j] + 1u || below;
            }
            // The first pass: every attempt that no other waits for, bottom to top.
#pragma unroll
            for (int j = CPT - 1; j >= 0; --j)
                attempt_rows<ACCEPT, P, S::PITCH>(A, s[j], f[j] >> S::SBITS, !def[j], rho, cell0 + j * S::NCX, tile);
            // Deferred attempts of this wave (about one lane in a hundred
            // holds one, so about half the waves skip the section): edges,
            // then corners; remote ones -- a bottom-row attempt of a bottom
            // cell whose column below is in another wave -- after the barrier.
            bool anydef = false;
#pragma unroll
            for (int j = 0; j < CPT; ++j) anydef = anydef || def[j];
            bool remote = false;
            if (anydef) {
                remote = border && def[CPT - 1] && bottom_of(f[CPT - 1]);
                wave_order();
                bool cor[CPT];
#pragma unroll
                for (int j = 0; j < CPT; ++j) {  // deferred edges
                    cor[j] = false;
                    if (def[j] && !(j == CPT - 1 && remote)) {
                        cor[j] = corner_of(f[j]);
                        if (!cor[j])
                            attempt_rows<ACCEPT, P, S::PITCH>(A, s[j], f[j] >> S::SBITS, true, rho, cell0 + j * S::NCX, tile);
                    }
                }
                wave_order();
#pragma unroll
                for (int j = 0; j < CPT; ++j)  // deferred corners
                    if (cor[j])
                        attempt_rows<ACCEPT, P, S::PITCH>(A, s[j], f[j] >> S::SBITS, true, rho, cell0 + j * S::NCX, tile);
            }
            const uint64_t wave_any = __ballot(remote);  // every lane takes part in the ballot
            if ((tid & 63u) == 0u && wave_any) atomicOr(&flags[rho % 3u], 1u);
            if (tid == 0) flags[(rho + 1u) % 3u] = 0u;
            __syncthreads();
            if (flags[rho % 3u]) {  // remote edges, then remote corners of the same waves
                const bool rc = remote && corner_of(f[CPT - 1]);
                if (remote && !rc)
                    attempt_rows<ACCEPT, P, S::PITCH>(A, s[CPT - 1], f[CPT - 1] >> S::SBITS, true, rho,
                                            cell0 + (CPT - 1) * S::NCX, tile);
                wave_order();
                if (rc)
                    attempt_rows<ACCEPT, P, S::PITCH>(A, s[CPT - 1], f[CPT - 1] >> S::SBITS, true, rho,
                                            cell0 + (CPT - 1) * S::NCX, tile);
                __syncthreads();
            }
            f16 = f16n;
            rb = rbn;
        }
    }
    copy_window_rows<false, P, S::PITCH>(A, lds, X0 >> 5, Y0 >> 2);
}

// The device-step kernel on the row-paired window, held to seven waves per
// SIMD (its LDS allows seven 256-lane workgroups per compute unit).
template <bool ACCEPT, int CPT, int LD, int LC>
__global__ void __launch_bounds__(kMaxStepThreads) __attribute__((amdgpu_waves_per_eu(7)))
step_db_rows_kernel(StepArgs A)
{
    extern __shared__ uint32_t smem[];
    sweep_db_rows<ACCEPT, CPT, LD, LC>(A, smem, blockIdx.x);
}

}  // namespace okpz
