// Host computation of the wall-straddling tile of a shifted phase (Hybrid variant).
//
// The tile holds the domain's last w/2 points in its left half and the first w/2
// points in its right half; the wall between them lies at the tile centre.  Each
// level updates the computed set [w/2 - r m, w/2 + r m) point by point with the
// scheme's own rule, in the order and with the boundary treatment of the GPU's
// wall tile: across the wall a point sees the Dirichlet ghost values, or for
// insulated heat ends the mirror of the point one inside the end (Appendix B,
// Eq. heatcond); at the widest level of a Diamond the stencil reaches the
// neighbouring triangles' tips just outside the tile.
#include "hybrid.hpp"

#include <vector>

namespace sw {

namespace {

template <class Sch>
void run_tile(HybridTile &t)
{
    constexpr int NV = Sch::NV, R = Sch::R;
    const TileArgs &a = t.a;
    const int w = a.w, half = w / 2, E = a.E, span = w + 2 * R;
    // rows[q][v] over tile positions [-R, w + R)
    std::vector<double> rows((size_t)2 * NV * span, 0.0);
    auto at = [&](int q, int v, int x) -> double & { return rows[(size_t)(q * NV + v) * span + x + R]; };
    for (int v = 0; v < NV; ++v) {
        for (int q = 0; q < 2; ++q)
            for (int x = 0; x < w; ++x)
                at(q, v, x) = x < half ? t.slot_a[(2 * v + q) * E + x + R] : t.slot_b[(2 * v + q) * E + x - half];
        for (int i = 0; i < R; ++i) {   // previous triangles' tips, read at the widest level
            at(1, v, i - R) = t.slot_a[(2 * v + 1) * E + i];
            at(1, v, w + i) = t.slot_b[(2 * v + 1) * E + half + i];
        }
    }
    const bool refl = a.bc == BC_REFLECTIVE;
    const int nlev = tile_levels(a);
    for (int s = 1; s <= nlev; ++s) {
        const int m = half_width(a, s);
        const int qs = (s - 1) & 1, qd = s & 1;
        const bool predictor = (s & 1) != 0;   // odd relative levels are RK2 predictors
        for (int x = half - R * m; x < half + R * m; ++x) {
            double ext[NV][1 + 2 * R];
            for (int v = 0; v < NV; ++v)
                for (int d = 0; d <= 2 * R; ++d) ext[v][d] = at(qs, v, x - R + d);
            if (refl) {   // heat: r = 1
                if (x == half) ext[0][0] = ext[0][2];        // domain point 0: T_{-1} = T_1
                if (x == half - 1) ext[0][2] = ext[0][0];    // domain point n-1: T_n = T_{n-2}
            } else {
                for (int v = 0; v < NV; ++v)
                    for (int d = 0; d <= 2 * R; ++d) {
                        const int pos = x - R + d;
                        if (x >= half && pos < half) ext[v][d] = a.c.ghost_l[v];
                        if (x < half && pos >= half) ext[v][d] = a.c.ghost_r[v];
                    }
            }
            double dst[NV][1];
            for (int v = 0; v < NV; ++v) dst[v][0] = at(qd, v, x);   // u^m for a final stage
            const bool in[1] = {true};
            Sch::template level<1, false>(dst, ext, predictor, a.c, in);
            for (int v = 0; v < NV; ++v) at(qd, v, x) = dst[v][0];
        }
    }
    if (a.kind != PH_DOWN) {   // new L slot into a, new R slot into b (the GPU's store_edge_point)
        for (int v = 0; v < NV; ++v)
            for (int q = 0; q < 2; ++q)
                for (int x = 0; x < w; ++x) {
                    if (x < half + R) t.slot_a[(2 * v + q) * E + x] = at(q, v, x);
                    if (x >= half - R) t.slot_b[(2 * v + q) * E + x - (half - R)] = at(q, v, x);
                }
    }
    int lo, hi;
    const int top = store_top_level<Sch>(a, lo, hi);
    if (top >= 0)
        for (int v = 0; v < NV; ++v)
            for (int x = lo; x < hi; ++x) t.top[(size_t)v * w + x] = at(top & 1, v, x);
}

}  // namespace

void hybrid_tile_host(HybridTile &t)
{
    if (t.scheme == 0) run_tile<Heat>(t);
    else if (t.scheme == 1) run_tile<KS>(t);
    else run_tile<Euler>(t);
}

}  // namespace sw
