// Host-side set-up of libemm (FP64): padded grid, finite-difference and
// interpolation weights, time step, CPML profile, wavelet and DTFT phases.
#pragma once

#include <complex>
#include <vector>

namespace emm {

// Padded node coordinates: nbe extra nodes per side spaced like the adjacent
// end interval (the paper gives only the layer counts, Section 3.4).
std::vector<double> pad_axis(const double *x, int n, int nbe);

// Midpoints x_{i+1/2} = (x_i + x_{i+1})/2 for i = 0..n-2.
std::vector<double> half_nodes(const std::vector<double> &xp);

// Inverse of the transposed Vandermonde matrix V^T(t_0..t_m) (Section 3.1,
// eq. amatrix), column by column from the Bjorck-Pereyra solve of
// V^T a = e_j.  Returns W row-major (m+1)x(m+1): row 0 = interpolation
// weights at the expansion point, row 1 = first-derivative weights.
std::vector<double> vandermonde_inverse(const std::vector<double> &t);

// D- (at integer node i over half nodes i-r..i+r-1) and D+ (at half node
// i+1/2 over integer nodes i-r+1..i+r) tables [n][2r]; zero outside [r, n-1-r].
void fd_tables(const std::vector<double> &xp, int r, std::vector<double> &cm,
               std::vector<double> &cp);

// CPML coefficients (Section 3.4) at integer and half nodes of one axis.
struct CpmlAxis {
    std::vector<double> a_int, b_int, a_half, b_half;
};
CpmlAxis cpml_axis(const std::vector<double> &xp, int nb, double dt, double v_lo,
                   double v_hi, double alpha_max, double npow, double R);

// Lagrange stencil of 2r points bracketing p on `coords`: coords[m] <= p <
// coords[m+1], support m-r+1..m+r.  Returns the base index (may be out of
// range: the caller validates) and fills w[2r].
int point_stencil(const std::vector<double> &coords, double p, int r, double *w);

// Wavelet samples at half steps s_n = s((n+1/2) dt) with
// s(t) = -((t - 4 tau)/tau) exp(-((t - 4 tau)/tau)^2), tau = 1/(pi fp).
std::vector<double> wavelet(int nt, double dt, double fp);

// omega' = (1 + i) sqrt(omega omega0) (Section 2.2, eq. correspondence)
std::complex<double> omega_prime(double f, double omega0);

}  // namespace emm
