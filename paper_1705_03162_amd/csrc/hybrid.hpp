// Hybrid variant (Sec. 5.1, swept rule variants): in the phases whose tiles are
// shifted by w/2, the tile that straddles the domain boundary of a non-periodic
// problem is computed by the host CPU while the GPU computes every other tile of
// the same phase.  The host evaluates the same per-point rules (schemes.hpp,
// compiled for the host with the same operation order and correctly rounded
// fma, division and square root), so results stay bit-identical.
#pragma once

#include "tile.hpp"

namespace sw {

// One straddling tile of one shifted phase, in host memory.
struct HybridTile {
    TileArgs a;        // the phase's geometry and constants; a.state and a.edges are unused
    int scheme;        // SW_HEAT, SW_KS or SW_EULER
    double *slot_a;    // host copy of the tile's slot a (nv * 2 * E doubles), read, and
    double *slot_b;    //   rewritten in place for a Diamond; likewise slot b
    double *top;       // Down: the top level of tile points [0, w), [nv][w] doubles
};

// Compute the tile: a Diamond rewrites both slot copies, a Down fills `top` at
// its top level's computed points.  Runs on any host thread; makes no HIP call.
void hybrid_tile_host(HybridTile &t);

}  // namespace sw
