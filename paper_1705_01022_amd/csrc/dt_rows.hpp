// DT and DTr device steps on the row-paired LDS window of the DB kernel
// (square domains of 128 or 256 sites, 8 x 8-site cells).  Same attempts and
// random draws as sweep_tile's DT / DTr path (Sec. 3 DT and DTr at block
// level, Sec. 3.1 single hit): in round rho every cell attempts one site of
// the quadrant its block draw names (DTr: of its cell in the shifted cell
// grid), so the attempts of one round touch pairwise disjoint slopes and
// need no ordering among themselves; a barrier separates the rounds.  What
// changes is how an attempt is found and tested -- one LDS address for its
// four slope words, linear site indices, acceptance after the slope pattern
// (attempt_rows) -- with every domain-sized quantity compile-time.
#pragma once

#include "db_rows.hpp"

namespace okpz {

// LDS words of the row-paired DT / DTr step: the window alone (wide rows).
template <int LD, int LC>
__host__ __device__ constexpr uint32_t rowpair_dt_lds_words()
{
    return RowPairShape<LD, LC, true>::WORDS;
}

// Lane t holds the cells (t mod NCX, CPT (t / NCX) + j), j = 0 .. CPT-1,
// stacked vertically, so the lanes of one instruction sit side by side in
// one or two cell rows.  Lane-draw fields are 2^FL bits (16 with acceptance
// prefixes, 4 without), the rounds of one Philox block unrolled.
template <int SCHEME, bool ACCEPT, int CPT, int LD, int LC>
__device__ __forceinline__ void sweep_dt_rows(const StepArgs &A, uint32_t *smem, uint32_t tile)
{
    using S = RowPairShape<LD, LC, true>;
    constexpr int FL = ACCEPT ? 4 : 2;
    constexpr uint32_t F = 1u << FL;
    constexpr int RPB = 128 >> FL;             // rounds per Philox block
    constexpr uint32_t QL = LC - 1;            // log2 of the quadrant side
    constexpr uint32_t QM = (1u << QL) - 1u;
    constexpr uint32_t SBITS = 2 * QL;         // site-index bits of a lane draw
    constexpr uint32_t P = S::P;
    static_assert(SBITS + (ACCEPT ? 8 : 0) <= F && (ACCEPT || SBITS == F), "field width");
    static_assert(SCHEME == kDT || SCHEME == kDTR, "DT or DTr");
    const uint32_t tid = threadIdx.x;
    uint32_t *lds = smem;

    const uint32_t tx = tile & ((1u << A.log2ntx) - 1u), ty = tile >> A.log2ntx;
    const uint32_t X0 = (A.ox + 2u * S::D * tx + A.set_a * S::D) & A.L_mask;
    const uint32_t Y0 = (A.oy + 2u * S::D * ty + A.set_b * S::D) & A.L_mask;
    // linear index of domain site (0, 0), counted from LDS address 0
    const uint32_t origin = (Y0 & 3u) * S::ROW + (X0 & 31u) + 8u * lds_address(lds);

    copy_window_rows<true, P, S::PITCH>(A, lds, X0 >> 5, Y0 >> 2);

    // lanes past the domain's cells (a batch sizes its workgroups for its
    // largest domains) only stage the window and keep the barriers; they
    // shadow the first cell row's lanes, so their reads stay in the window
    const bool act = tid < S::NCX * S::NCX / CPT;
    const uint32_t cx = tid & (S::NCX - 1u), grp = act ? tid >> S::LOG2NCX : 0u;
    const uint32_t base_u = cx << LC;
    const uint32_t base_v0 = (grp * CPT) << LC;   // top cell's corner row
    const uint32_t cell0 = (grp * CPT) * S::NCX + cx;

    auto field_of = [](const uint32_t(&w)[4], int k) -> uint32_t {
        constexpr int FPW = 32 / F;
        return (w[k / FPW] >> (F * (k % FPW))) & ((1u << F) - 1u);
    };

    BlockDraw bd = {0u, 0u, 0u, 0u};
    __syncthreads();
    const uint32_t nblk = A.rounds / RPB;
    for (uint32_t blk = 0; blk < nblk; ++blk) {
        uint32_t w[CPT][4];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const u32x4 r = philox4x32_10_lane(A.key0, A.key1, blk, cell0 + j * S::NCX, tile, A.c3);
            w[j][0] = r.x; w[j][1] = r.y; w[j][2] = r.z; w[j][3] = r.w;
        }
#pragma unroll
        for (int k = 0; k < RPB; ++k) {
            const uint32_t rho = blk * RPB + k;
            const uint32_t f16 = next_block_field(A, bd, rho, tile);
            // the round's quadrant (and, DTr, the shift of the cell grid)
            uint32_t cu = base_u + ((f16 & 1u) << QL), cv = base_v0 + (((f16 >> 1) & 1u) << QL);
            if (SCHEME == kDTR) {
                cu += (f16 >> 2) & (S::C - 1u);
                cv += (f16 >> 8) & (S::C - 1u);
            }
#pragma unroll
            for (int j = CPT - 1; j >= 0; --j) {
                const uint32_t f = field_of(w[j], k);
                uint32_t u = cu + (f & QM);
                uint32_t v = cv + (j << LC) + ((f >> QL) & QM);
                if (SCHEME == kDTR) {
                    // the shifted grid wraps around the domain; only a lane's
                    // bottom cell can be in the last cell row
                    u &= S::D - 1u;
                    if (j == CPT - 1) v &= S::D - 1u;
                }
                const uint32_t s = __umul24(v, S::ROW) + u + origin;
                attempt_rows<ACCEPT, P, S::PITCH>(A, s, f >> SBITS, act, rho, cell0 + j * S::NCX, tile);
            }
            __syncthreads();
        }
    }
    copy_window_rows<false, P, S::PITCH>(A, lds, X0 >> 5, Y0 >> 2);
}

// The DT / DTr device-step kernel on the row-paired window.
template <int SCHEME, bool ACCEPT, int CPT, int LD, int LC>
__global__ void __launch_bounds__(kMaxStepThreads) __attribute__((amdgpu_waves_per_eu(7)))
step_dt_rows_kernel(StepArgs A)
{
    extern __shared__ uint32_t smem[];
    sweep_dt_rows<SCHEME, ACCEPT, CPT, LD, LC>(A, smem, blockIdx.x);
}

}  // namespace okpz
