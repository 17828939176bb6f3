// Prior of the log pseudo-density on the grid: tapered Matern(1/3)
// covariance and its Vecchia (inverse-Cholesky) sparse precision.
#pragma once
#include <cstdint>
#include <vector>

#include "symbolic.h"

namespace ep {

struct PriorParams {
    double mean = -7.0;     // m0
    double var = 1.0;       // sigma_f^2
    double ell = 100.0;     // Matern length scale = outer scale
    double support = 150.0; // taper radius
    double rho = 150.0;     // conditioning radius
};

// Modified Bessel K_nu(x) for non-integer nu from the ascending series of
// I_{+-nu}: K_nu = pi / (2 sin(nu pi)) (I_{-nu} - I_nu).  Accurate for the
// moderate x (< ~8) the tapered kernel needs.
double besselk_series(double nu, double x);
double cov_tapered(const PriorParams& p, double r);

// Vecchia factor: B strictly lower in lexicographic node order (CSR rows,
// ascending columns) and the conditional variances D.
struct Vecchia {
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<double> d;
};

// Returns 0, or -1 if a conditioning system is not positive definite.
int build_vecchia(const GridGeom& g, const PriorParams& p, const Stencil& st, Vecchia& out);

// Q0 = (I-B)^T D^{-1} (I-B) as one value per (node, non-positive stencil
// offset): q0[p * nhalf + o] couples node p with p + offset_o (offset_o
// lexicographically <= 0, offset 0 first).  Offsets in 'lower' (packed
// triples).
struct Q0Table {
    std::vector<int> lower;       // packed (di, dj, dk), first is (0,0,0)
    std::vector<double> val;      // N * nlower
    int nlower = 0;
};
void build_q0(const GridGeom& g, const Stencil& st, const Vecchia& v, Q0Table& out);

// b0 = Q0 (m0 * 1)
void q0_times_const(const GridGeom& g, const Vecchia& v, double m0, std::vector<double>& out);

// Exact prior draw f = m0 + (I-B)^{-1} D^{1/2} xi.
void prior_draw(const GridGeom& g, const Vecchia& v, double m0, const double* xi, double* f);

}  // namespace ep
