// Host-side structure of the EP posterior precision
//   Q = Q0 + sum_n tau_n g_n g_n^T
// on a 3-D grid: the star sightline supports, a nested-dissection ordering
// that respects both the prior stencil and the sightline cliques, and the
// multifrontal (supernodal) layout of the Cholesky factor.
#pragma once
#include <cstdint>
#include <vector>

namespace ep {

struct GridGeom {
    int n = 0;              // nodes per axis
    double L = 0;           // cube side (pc)
    double h = 0;           // spacing L/(n-1)
    double obs[3] = {0, 0, 0};
    double step = 2.0;      // LOS trapezoid step bound (pc)
    int64_t N() const { return (int64_t)n * n * n; }
};

// Sightline supports: CSR over stars of sorted original node ids.
struct Supports {
    std::vector<int64_t> ptr;     // n_stars + 1
    std::vector<int32_t> nodes;   // sorted per star
    std::vector<int32_t> nsamp;   // trapezoid intervals T_n per star
};

void build_supports(const GridGeom& g, int64_t n_stars, const double* xyz, Supports& out);

// Offsets (di, dj, dk) of the prior precision's stencil: pairs of nodes that
// share a Vecchia conditioning row.  Built from the half-ball H of offsets
// q - p of a node's conditioning set: the stencil is {a - b : a, b in H+0}.
struct Stencil {
    int R = 0;                           // max |offset| per axis of H
    std::vector<int> half;               // H as packed (di, dj, dk) triples, q - p < 0 lexicographically
    std::vector<int> full;               // all offsets of Q0 (including 0), packed triples
    // offsets of the factor's pattern: full plus the block {-2..2}^3, so that
    // the 8 corners of every cell, and the 16 corners of any two cells that
    // touch, are pairwise on the pattern (the map predictions read Sigma there)
    std::vector<int> pattern;
};
void build_stencil(const GridGeom& g, double rho, Stencil& st);

// Multifrontal layout.
struct Front {
    int64_t first = 0;     // first new index of V_s
    int32_t nv = 0;        // |V_s|
    int32_t nvpad = 0;     // |V_s| rounded up to the tile
    int32_t nr = 0;        // |R_s|
    int32_t m = 0;         // padded front order: nvpad + roundup(nr)
    int32_t parent = -1;
    int32_t level = 0;     // height in the front tree (leaves 0)
    int64_t off = 0;       // element offset of the m x m column-major block
    int64_t rptr = 0;      // offset into the R lists (rows, relmap)
};

struct Symbolic {
    int tile = 64;
    std::vector<int32_t> perm;      // new -> original
    std::vector<int32_t> iperm;     // original -> new
    std::vector<Front> fronts;
    std::vector<int32_t> snode;     // new index -> front
    std::vector<int64_t> rrows;     // concatenated R_s (new indices)
    std::vector<int32_t> relmap;    // concatenated local rows of R_s in the parent front (-1 root)
    std::vector<int32_t> star_front;  // front holding each star's clique
    std::vector<int32_t> star_loc;    // local row of each support node in its star's front
    int nlevels = 0;
    int64_t total_elems = 0;        // sum m^2
    double factor_flops = 0;        // dense-front partial Cholesky flops
    double selinv_flops = 0;
    double trail_flops = 0;         // trailing updates after each pivot panel
    int64_t max_m = 0;
};

struct OrderingOpts {
    int leaf_size = 512;
    double sep_halfwidth = 0;   // half-width of a separator slab (pc)
    int tile = 64;
    int panel_tiles = 8;        // pivot tiles per factor panel (flop accounting)
};

// Nested dissection + symbolic multifrontal analysis.  Returns 0 or a
// negative error code.
int analyse(const GridGeom& g, const Stencil& st, const Supports& sup, const OrderingOpts& opt,
            Symbolic& sym);

}  // namespace ep
