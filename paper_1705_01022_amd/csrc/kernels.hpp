// Device kernels of the octahedron-model simulator (gfx950).
//
// Packed lattice: uint32 word (y/4)*(L/4) + x/4 holds a 4x4 block of sites,
// bit 4*(y%4)+x%4 = sx (slope to the left neighbour is +1), bit
// 16+4*(y%4)+x%4 = sy (slope to the neighbour at y-1 is +1) - the paper's
// 2-bit-per-site, 16-sites-per-word coding (Sec. 3.1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace okpz {

constexpr uint32_t kFlatWord = 0x5A5A5A5Au;  // h = (x+y) mod 2: slopes +1 on odd sites

enum : int { kDT = 0, kDB = 1, kDTR = 2 };

// ---------------------------------------------------------------- init
__global__ void fill_words_kernel(uint32_t *__restrict__ words, uint64_t n, uint32_t value)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        words[i] = value;
}

// ---------------------------------------------------------------- Philox test
__global__ void philox_kernel(uint32_t k0, uint32_t k1, const uint32_t *__restrict__ ctr,
                              uint32_t *__restrict__ out, uint64_t n)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32x4 r = philox4x32_10(k0, k1, ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
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
    uint32_t lw_mask, lw_log2;  // words per row - 1, log2(words per row)
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
    uint32_t Wx, Wy, pitch;     // LDS window of the domain + halo, in words
    uint32_t dep_always, rem_always;  // p == 1 / q == 1 when no acceptance draw is needed
    uint32_t P_hi, P_lo, Q_hi, Q_lo;  // acceptance thresholds on the (A+32)-bit variate
};

// LDS staging of the domain window: word rows wy0 .. wy0+Wy-1 and word
// columns wx0 .. wx0+Wx-1 (periodic).  Each wave copies whole rows, so
// global accesses are contiguous runs of Wx words.
template <bool LOAD>
__device__ __forceinline__ void copy_window(const StepArgs &A, uint32_t *lds, uint32_t wx0, uint32_t wy0)
{
    const uint32_t nwaves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    for (uint32_t r = wave; r < A.Wy; r += nwaves) {
        uint32_t *row = A.words + (static_cast<uint64_t>((wy0 + r) & A.lw_mask) << A.lw_log2);
        for (uint32_t c = lane; c < A.Wx; c += 64) {
            const uint32_t gx = (wx0 + c) & A.lw_mask;
            if (LOAD)
                lds[r * A.pitch + c] = row[gx];
            else
                row[gx] = lds[r * A.pitch + c];
        }
    }
}

// One update attempt at LDS site (lx, ly) (Sec. 2.1 rule): read sx, sy of
// the site, sx of (lx+1, ly) and sy of (lx, ly+1); a local minimum
// (0,1,0,1) may deposit, a local maximum (1,0,1,0) may be removed; both
// flip the same four bits.  Flips are LDS atomic XORs because attempts of
// neighbouring cells may share a word (never a bit).
template <bool ACCEPT>
__device__ __forceinline__ void do_attempt(const StepArgs &A, uint32_t *lds, uint32_t lx, uint32_t ly,
                                           uint32_t upre, uint32_t rho, uint32_t cell, uint32_t tile)
{
    const uint32_t wi = (ly >> 2) * A.pitch + (lx >> 2);
    const uint32_t bx = lx & 3u, by = ly & 3u;
    const uint32_t sxb = 4u * by + bx;
    const uint32_t w = lds[wi];
    const uint32_t wr = (bx == 3u) ? lds[wi + 1] : w;
    const uint32_t wd = (by == 3u) ? lds[wi + A.pitch] : w;
    const uint32_t a = (w >> sxb) & 1u;
    const uint32_t c = (w >> (16u + sxb)) & 1u;
    const uint32_t b = (wr >> (4u * by + ((bx + 1u) & 3u))) & 1u;
    const uint32_t d = (wd >> (16u + 4u * ((by + 1u) & 3u) + bx)) & 1u;
    const uint32_t pat = a | (b << 1) | (c << 2) | (d << 3);
    const bool is_min = pat == 0xAu;  // a=0 b=1 c=0 d=1
    const bool is_max = pat == 0x5u;  // a=1 b=0 c=1 d=0
    bool flip;
    if (ACCEPT) {
        // U = (upre << 32) | r compared with P (deposition) or Q (removal);
        // r is drawn only when the prefix ties with the threshold's prefix.
        const uint32_t thr_hi = is_min ? A.P_hi : A.Q_hi;
        const uint32_t thr_lo = is_min ? A.P_lo : A.Q_lo;
        flip = (is_min || is_max) && upre < thr_hi;
        if ((is_min || is_max) && upre == thr_hi) {
            const u32x4 r = philox4x32_10(A.key0, A.key1, rho, cell | 0x80000000u, tile, A.c3);
            flip = r.x < thr_lo;
        }
    } else {
        flip = (is_min && A.dep_always) || (is_max && A.rem_always);
    }
    if (flip) {
        uint32_t m0 = (1u << sxb) | (1u << (16u + sxb));
        if (bx != 3u)
            m0 |= 1u << (sxb + 1u);
        else
            atomicXor(&lds[wi + 1], 1u << (4u * by));
        if (by != 3u)
            m0 |= 1u << (16u + sxb + 4u);
        else
            atomicXor(&lds[wi + A.pitch], 1u << (16u + bx));
        atomicXor(&lds[wi], m0);
    }
}

// One device step.  Workgroup = one tile; its active domain (sub-tile set
// (set_a, set_b)) is staged with its +x column and +y row in LDS, swept by
// Cx*Cy single-hit rounds (each cell gets exactly one attempt per round),
// and written back.  Same-set domains never share a word when the domain
// is at least 4 sites wide, so whole-word write-back is race-free.
//
// Lane draws: cell c takes F-bit fields of the Philox block
// (round / (128/F), c, tile, 4*MCS+step), lowest bits first; the low
// s_bits pick the site (in the chosen quadrant for DT/DTr, anywhere in the
// cell for DB) and the rest is the acceptance prefix.  Block draws: 16-bit
// fields of (round/8, 0xFFFFFFFF, tile, 4*MCS+step): bits 0-1 quadrant,
// 2-7 and 8-13 the cell-grid shift.
template <int SCHEME, bool ACCEPT, int CPT>
__global__ void __launch_bounds__(256) step_kernel(StepArgs A)
{
    extern __shared__ uint32_t lds[];
    const uint32_t tile = blockIdx.x;
    const uint32_t tx = tile & ((1u << A.log2ntx) - 1u), ty = tile >> A.log2ntx;
    const uint32_t X0 = (A.ox + 2u * A.Dx * tx + A.set_a * A.Dx) & A.L_mask;
    const uint32_t Y0 = (A.oy + 2u * A.Dy * ty + A.set_b * A.Dy) & A.L_mask;
    const uint32_t offx = X0 & 3u, offy = Y0 & 3u;

    copy_window<true>(A, lds, X0 >> 2, Y0 >> 2);

    const uint32_t NT = blockDim.x;
    const uint32_t Cx = 1u << A.log2Cx, Cy = 1u << A.log2Cy;
    const uint32_t F = 1u << A.F_log2;
    const uint32_t per_word_mask = (32u >> A.F_log2) - 1u;    // fields per word - 1
    const uint32_t per_call_mask = (128u >> A.F_log2) - 1u;   // fields per call - 1
    const uint32_t fmask = F == 32u ? 0xFFFFFFFFu : ((1u << F) - 1u);
    const uint32_t smask = (1u << A.s_bits) - 1u;
    const uint32_t hw_log2 = A.log2Cx - 1u;                   // DT quadrant width, log2

    uint32_t cell[CPT], base_u[CPT], base_v[CPT];
    uint32_t rw[CPT][4];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        cell[j] = threadIdx.x + j * NT;
        base_u[j] = (cell[j] & ((1u << A.log2ncx) - 1u)) << A.log2Cx;
        base_v[j] = (cell[j] >> A.log2ncx) << A.log2Cy;
    }
    uint32_t bw0 = 0, bw1 = 0, bw2 = 0, bw3 = 0;
    __syncthreads();

    for (uint32_t rho = 0; rho < A.rounds; ++rho) {
        if ((rho & 7u) == 0u) {
            const u32x4 r = philox4x32_10(A.key0, A.key1, rho >> 3, 0xFFFFFFFFu, tile, A.c3);
            bw0 = r.x; bw1 = r.y; bw2 = r.z; bw3 = r.w;
        }
        const uint32_t f16 = bw0 & 0xFFFFu;
        if (rho & 1u) {
            bw0 = bw1; bw1 = bw2; bw2 = bw3;
        } else {
            bw0 >>= 16;
        }
        const uint32_t sigma = f16 & 3u;
        const uint32_t bx = SCHEME == kDT ? 0u : ((f16 >> 2) & (Cx - 1u));
        const uint32_t by = SCHEME == kDT ? 0u : ((f16 >> 8) & (Cy - 1u));

        uint32_t lx[CPT], ly[CPT], upre[CPT], phase[CPT];
        const bool refill = (rho & per_call_mask) == 0u;
        const bool rotate = ((rho + 1u) & per_word_mask) == 0u;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (refill) {
                const u32x4 r = philox4x32_10(A.key0, A.key1, rho >> (7u - A.F_log2), cell[j], tile, A.c3);
                rw[j][0] = r.x; rw[j][1] = r.y; rw[j][2] = r.z; rw[j][3] = r.w;
            }
            const uint32_t field = rw[j][0] & fmask;
            if (rotate) {
                rw[j][0] = rw[j][1]; rw[j][1] = rw[j][2]; rw[j][2] = rw[j][3];
            } else {
                rw[j][0] >>= (F & 31u);  // F < 32 here: rotation handles F = 32
            }
            const uint32_t idx = field & smask;
            uint32_t du, dv;
            if (SCHEME == kDB) {
                du = idx & (Cx - 1u);
                dv = idx >> A.log2Cx;
            } else {
                du = ((sigma & 1u) << hw_log2) + (idx & ((1u << hw_log2) - 1u));
                dv = ((sigma >> 1) << (A.log2Cy - 1u)) + (idx >> hw_log2);
            }
            const uint32_t u = (bx + base_u[j] + du) & (A.Dx - 1u);
            const uint32_t v = (by + base_v[j] + dv) & (A.Dy - 1u);
            lx[j] = u + offx;
            ly[j] = v + offy;
            upre[j] = ACCEPT ? (field >> A.s_bits) : 0u;
            phase[j] = SCHEME == kDB ? (uint32_t)(du == Cx - 1u) + (uint32_t)(dv == Cy - 1u) : 0u;
        }
        constexpr int NPH = SCHEME == kDB ? 3 : 1;
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                if (cell[j] < A.ncell && phase[j] == (uint32_t)ph)
                    do_attempt<ACCEPT>(A, lds, lx[j], ly[j], upre[j], rho, cell[j], tile);
            }
            __syncthreads();
        }
    }
    copy_window<false>(A, lds, X0 >> 2, Y0 >> 2);
}

// ---------------------------------------------------------------- measurement
// Heights (gauge h(0,0) = 0): h(0,y) = sum_{y'=1..y} (2 sy[0,y'] - 1);
// h(x,y) = h(0,y) + sum_{x'=1..x} (2 sx[x',y] - 1).

// Column-0 anchors h(0,y), one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) anchors_kernel(const uint32_t *__restrict__ words, uint32_t L,
                                                       uint32_t lw_log2, int32_t *__restrict__ h0)
{
    __shared__ int32_t part[1024];
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    const uint32_t chunk = (L + T - 1) / T;
    const uint32_t y0 = tid * chunk;
    int32_t local = 0;
    for (uint32_t y = y0; y < y0 + chunk && y < L; ++y) {
        if (y == 0) continue;
        const uint32_t w = words[static_cast<uint64_t>(y >> 2) << lw_log2];
        local += 2 * (int32_t)((w >> (16u + 4u * (y & 3u))) & 1u) - 1;
    }
    part[tid] = local;
    __syncthreads();
    for (uint32_t off = 1; off < T; off <<= 1) {  // inclusive Hillis-Steele scan
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t h = part[tid] - local;  // exclusive prefix
    for (uint32_t y = y0; y < y0 + chunk && y < L; ++y) {
        if (y > 0) {
            const uint32_t w = words[static_cast<uint64_t>(y >> 2) << lw_log2];
            h += 2 * (int32_t)((w >> (16u + 4u * (y & 3u))) & 1u) - 1;
        }
        h0[y] = h;
    }
}

// Wave-level inclusive scan of 64-bit values (wave64).
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v)
{
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}

// Exclusive block scan of packed 64-bit values (4 x 16-bit lanes, no
// carries between fields by construction); returns the exclusive prefix and
// the block total.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *wave_tot, uint64_t &total)
{
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t inc = wave_incl_scan(v);
    if (lane == 63u) wave_tot[wave] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (uint32_t i = 0; i < nw; ++i) {
        const uint64_t t = wave_tot[i];
        if (i < wave) before += t;
        all += t;
    }
    __syncthreads();
    total = all;
    return before + inc - v;
}

constexpr int kMeasureThreads = 256;
constexpr int kMomentFields = 5;  // S1_even, S1_odd, S2_even, S2_odd, S_ts

// Per word-row partial moments.  One workgroup per word row (4 site rows);
// the words of the row are streamed in chunks of 256 with a block scan of
// the per-word height increments of the 4 rows (packed in 16-bit fields,
// biased by +4 so fields stay non-negative).  With a snapshot, the same is
// done for the snapshot words and sum h_t h_s is accumulated.
template <bool CROSS>
__global__ void __launch_bounds__(kMeasureThreads) rows_kernel(const uint32_t *__restrict__ words,
                                                               const int32_t *__restrict__ h0,
                                                               const uint32_t *__restrict__ snap,
                                                               const int32_t *__restrict__ h0s, uint32_t L,
                                                               uint32_t lw_log2, int64_t *__restrict__ partial)
{
    __shared__ uint64_t wave_tot[kMeasureThreads / 64];
    __shared__ int64_t red[kMomentFields][kMeasureThreads];
    const uint32_t y4 = blockIdx.x, tid = threadIdx.x;
    const uint32_t lw = 1u << lw_log2;
    const uint64_t row_base = static_cast<uint64_t>(y4) << lw_log2;
    int32_t carry[4], carry_s[4], anchor[4], anchor_s[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        carry[r] = 0;
        carry_s[r] = 0;
        anchor[r] = h0[4 * y4 + r];
        anchor_s[r] = CROSS ? h0s[4 * y4 + r] : 0;
    }
    int64_t s1e = 0, s1o = 0, s2e = 0, s2o = 0, sts = 0;
    for (uint32_t base = 0; base < lw; base += kMeasureThreads) {
        const uint32_t wx = base + tid;
        const bool active = wx < lw;
        const uint32_t w = active ? words[row_base + wx] : 0u;
        const uint32_t ws = (CROSS && active) ? snap[row_base + wx] : 0u;
        // per-row increments over the word; site x = 0 contributes no step
        uint64_t packed = 0, packed_s = 0;
        int32_t inc[4], inc_s[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t nib = (w >> (4 * r)) & 0xFu, nib_s = (ws >> (4 * r)) & 0xFu;
            int32_t steps = 4, steps_s = 4;
            if (wx == 0) {
                nib &= 0xEu;
                nib_s &= 0xEu;
                steps = 3;
                steps_s = 3;
            }
            inc[r] = 2 * __popc(nib) - steps;
            inc_s[r] = 2 * __popc(nib_s) - steps_s;
            if (active) {  // inactive threads sit after every active one and add nothing
                packed |= static_cast<uint64_t>(inc[r] + 4) << (16 * r);
                packed_s |= static_cast<uint64_t>(inc_s[r] + 4) << (16 * r);
            }
        }
        uint64_t tot, tot_s = 0;
        const uint64_t ex = block_excl_scan(packed, wave_tot, tot);
        uint64_t ex_s = 0;
        if (CROSS) ex_s = block_excl_scan(packed_s, wave_tot, tot_s);
        const int32_t nact = (int32_t)min((uint32_t)kMeasureThreads, lw - base);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int32_t pin = carry[r] + (int32_t)((ex >> (16 * r)) & 0xFFFFu) - 4 * (int32_t)tid;
            const int32_t pin_s = CROSS ? carry_s[r] + (int32_t)((ex_s >> (16 * r)) & 0xFFFFu) - 4 * (int32_t)tid : 0;
            carry[r] += (int32_t)((tot >> (16 * r)) & 0xFFFFu) - 4 * nact;
            if (CROSS) carry_s[r] += (int32_t)((tot_s >> (16 * r)) & 0xFFFFu) - 4 * nact;
            if (!active) continue;
            const uint32_t y = 4 * y4 + r;
            int32_t h = anchor[r] + pin, hs = anchor_s[r] + pin_s;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t x = 4 * wx + i;
                if (x != 0) {
                    h += 2 * (int32_t)((w >> (4 * r + i)) & 1u) - 1;
                    if (CROSS) hs += 2 * (int32_t)((ws >> (4 * r + i)) & 1u) - 1;
                }
                const int64_t hv = h;
                if (((x + y) & 1u) == 0u) {
                    s1e += hv;
                    s2e += hv * hv;
                } else {
                    s1o += hv;
                    s2o += hv * hv;
                }
                if (CROSS) sts += hv * (int64_t)hs;
            }
        }
    }
    red[0][tid] = s1e;
    red[1][tid] = s1o;
    red[2][tid] = s2e;
    red[3][tid] = s2o;
    red[4][tid] = sts;
    __syncthreads();
    for (uint32_t off = kMeasureThreads / 2; off > 0; off >>= 1) {
        if (tid < off)
#pragma unroll
            for (int f = 0; f < kMomentFields; ++f) red[f][tid] += red[f][tid + off];
        __syncthreads();
    }
    if (tid < kMomentFields) partial[static_cast<uint64_t>(y4) * kMomentFields + tid] = red[tid][0];
}

// 128-bit signed accumulate (two's complement in (lo, hi)).
__device__ __forceinline__ void add_i128(uint64_t &lo, int64_t &hi, uint64_t blo, int64_t bhi)
{
    const uint64_t nlo = lo + blo;
    hi += bhi + (nlo < lo ? 1 : 0);
    lo = nlo;
}

// Final exact reduction of the per-row partials into 128-bit totals.
__global__ void __launch_bounds__(256) reduce_kernel(const int64_t *__restrict__ partial, uint32_t nrows,
                                                     int64_t *__restrict__ out)
{
    __shared__ uint64_t lo_s[kMomentFields][256];
    __shared__ int64_t hi_s[kMomentFields][256];
    const uint32_t tid = threadIdx.x;
    for (int f = 0; f < kMomentFields; ++f) {
        uint64_t lo = 0;
        int64_t hi = 0;
        for (uint32_t r = tid; r < nrows; r += blockDim.x) {
            const int64_t v = partial[static_cast<uint64_t>(r) * kMomentFields + f];
            add_i128(lo, hi, static_cast<uint64_t>(v), v < 0 ? -1 : 0);
        }
        lo_s[f][tid] = lo;
        hi_s[f][tid] = hi;
    }
    __syncthreads();
    for (uint32_t off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int f = 0; f < kMomentFields; ++f) {
                uint64_t lo = lo_s[f][tid];
                int64_t hi = hi_s[f][tid];
                add_i128(lo, hi, lo_s[f][tid + off], hi_s[f][tid + off]);
                lo_s[f][tid] = lo;
                hi_s[f][tid] = hi;
            }
        __syncthreads();
    }
    if (tid < kMomentFields) {
        out[2 * tid] = static_cast<int64_t>(lo_s[tid][0]);
        out[2 * tid + 1] = hi_s[tid][0];
    }
}

}  // namespace okpz
