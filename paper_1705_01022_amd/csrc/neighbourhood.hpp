// Dependency neighbourhood of a batch work item (host and device).
//
// Work item (g, t) of a lattice -- generation g = 4 * MCS + step, tile t of
// the MCS's tiling (Sec. 3 DTr: 2Dx x 2Dy tiles from the MCS's random origin)
// -- may start once generation g - 1 has finished on every tile whose memory
// words it can share.  Every item of a tile stays inside the tile's extended
// region: its 2Dx x 2Dy sites plus the +1 column and row that rim attempts
// touch, widened to whole 32-site words (up to 31 sites on either side) and
// 4-row bands (up to 3 rows).  So within one tiling, tiles further apart than
// 1 + 31/Dx columns or 1 + 3/Dy rows never share a word.  At the first step
// of an MCS the tiling has moved to a new origin: the tiles of the previous
// tiling to wait for lie around the old tile that holds the new tile's
// corner, reaching one tile further on the far side.
#pragma once

#include <stdint.h>

namespace okpz {

struct WaitSet {
    uint32_t cx0, ncol;  // tile columns cx0 .. cx0 + ncol - 1 (mod tiles per row)
    uint32_t cy0, nrow;  // tile rows cy0 .. cy0 + nrow - 1 (mod tile rows)
};

// Tiles of generation g - 1 that item (g, t) waits for (besides tile t
// itself).  L_mask = L - 1; log2ntx = log2(tiles per row); ntiles = tiles per
// step.  new_tiling: g is the first step of an MCS whose origin is (ox, oy),
// the previous MCS's origin (oxp, oyp); otherwise the origins are unused.
__host__ __device__ inline WaitSet wait_set(uint32_t Dx, uint32_t Dy, uint32_t L_mask, uint32_t log2ntx,
                                            uint32_t ntiles, uint32_t t, bool new_tiling, uint32_t ox,
                                            uint32_t oy, uint32_t oxp, uint32_t oyp)
{
    const uint32_t ntx = 1u << log2ntx, nty = ntiles >> log2ntx;
    uint32_t tx = t & (ntx - 1u), ty = t >> log2ntx;
    const uint32_t ex = 31u / Dx, ey = 3u / Dy;  // extra tiles the word / band widening reaches
    uint32_t hix = 1u + ex, hiy = 1u + ey;
    if (new_tiling) {
        // the previous tiling's tile holding this tile's corner
        const uint32_t sx = (uint32_t)__builtin_ctz(2u * Dx), sy = (uint32_t)__builtin_ctz(2u * Dy);
        tx = (((ox + (tx << sx)) - oxp) & L_mask) >> sx;
        ty = (((oy + (ty << sy)) - oyp) & L_mask) >> sy;
        hix += 1u;
        hiy += 1u;
    }
    // columns tx - 1 - ex .. tx + hix (all of them when that wraps), rows likewise
    WaitSet w;
    w.cx0 = (tx + ntx - ((1u + ex) & (ntx - 1u))) & (ntx - 1u);
    w.ncol = 2u + ex + hix;
    w.cy0 = (ty + nty - ((1u + ey) & (nty - 1u))) & (nty - 1u);
    w.nrow = 2u + ey + hiy;
    if (w.ncol >= ntx) {
        w.cx0 = 0u;
        w.ncol = ntx;
    }
    if (w.nrow >= nty) {
        w.cy0 = 0u;
        w.nrow = nty;
    }
    return w;
}

}  // namespace okpz
