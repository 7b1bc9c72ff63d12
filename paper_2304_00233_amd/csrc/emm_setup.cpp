// Host-side set-up of libemm in FP64 (rounded to FP32 only when uploaded).
#include "emm_setup.h"

#include <algorithm>
#include <cmath>

namespace emm {

std::vector<double> pad_axis(const double *x, int n, int nbe) {
    std::vector<double> xp(n + 2 * nbe);
    const double hlo = x[1] - x[0], hhi = x[n - 1] - x[n - 2];
    for (int i = 0; i < n; ++i) xp[nbe + i] = x[i];
    for (int m = 1; m <= nbe; ++m) {
        xp[nbe - m] = x[0] - m * hlo;
        xp[nbe + n - 1 + m] = x[n - 1] + m * hhi;
    }
    return xp;
}

std::vector<double> half_nodes(const std::vector<double> &xp) {
    std::vector<double> h(xp.size() - 1);
    for (size_t i = 0; i + 1 < xp.size(); ++i) h[i] = 0.5 * (xp[i] + xp[i + 1]);
    return h;
}

// Bjorck-Pereyra (Golub & Van Loan, Algorithm 4.6.1) for V^T a = f, applied
// to every unit vector f = e_j at once: the right-hand sides are the columns
// of the identity, so the two sweeps (Newton divided differences, then the
// change from the Newton to the monomial basis) act on a whole matrix.
std::vector<double> vandermonde_inverse(const std::vector<double> &t) {
    const int m = static_cast<int>(t.size());
    std::vector<double> A(m * m, 0.0);          // A[i][j]: coefficient i of column j
    for (int j = 0; j < m; ++j) A[j * m + j] = 1.0;
    // divided differences: level lev replaces rows lev..m-1
    for (int lev = 1; lev < m; ++lev)
        for (int row = m - 1; row >= lev; --row) {
            const double inv = 1.0 / (t[row] - t[row - lev]);
            for (int j = 0; j < m; ++j)
                A[row * m + j] = (A[row * m + j] - A[(row - 1) * m + j]) * inv;
        }
    // Newton form -> monomial coefficients, expanding (t - t_node) factors
    for (int node = m - 2; node >= 0; --node)
        for (int row = node; row < m - 1; ++row)
            for (int j = 0; j < m; ++j) A[row * m + j] -= t[node] * A[(row + 1) * m + j];
    return A;
}

void fd_tables(const std::vector<double> &xp, int r, std::vector<double> &cm,
               std::vector<double> &cp) {
    const int n = static_cast<int>(xp.size());
    const int L = 2 * r;
    const std::vector<double> xh = half_nodes(xp);
    cm.assign(static_cast<size_t>(n) * L, 0.0);
    cp.assign(static_cast<size_t>(n) * L, 0.0);
    std::vector<double> t(L);
    for (int i = r; i <= n - 1 - r; ++i) {
        for (int m = 0; m < L; ++m) t[m] = xh[i - r + m] - xp[i];
        std::vector<double> W = vandermonde_inverse(t);
        for (int m = 0; m < L; ++m) cm[i * L + m] = W[1 * L + m];
        for (int m = 0; m < L; ++m) t[m] = xp[i - r + 1 + m] - xh[i];
        W = vandermonde_inverse(t);
        for (int m = 0; m < L; ++m) cp[i * L + m] = W[1 * L + m];
    }
}

CpmlAxis cpml_axis(const std::vector<double> &xp, int nb, double dt, double v_lo,
                   double v_hi, double alpha_max, double npow, double R) {
    const int n = static_cast<int>(xp.size());
    CpmlAxis c;
    c.a_int.assign(n, 0.0);
    c.b_int.assign(n, 0.0);
    c.a_half.assign(n, 0.0);
    c.b_half.assign(n, 0.0);
    if (nb <= 0) return c;
    const double Llo = xp[nb] - xp[0], Lhi = xp[n - 1] - xp[n - 1 - nb];
    for (int half = 0; half < 2; ++half) {
        std::vector<double> &a = half ? c.a_half : c.a_int;
        std::vector<double> &b = half ? c.b_half : c.b_int;
        for (int i = 0; i < n; ++i) {
            if (half && i == n - 1) continue;             // no half node past the end
            const double pos = half ? 0.5 * (xp[i] + xp[i + 1]) : xp[i];
            double depth, L, v;                           // normalised depth into the layer
            if (i < nb) {
                depth = (xp[nb] - pos) / Llo;
                L = Llo;
                v = v_lo;
            } else if (i > n - 1 - nb) {
                depth = (pos - xp[n - 1 - nb]) / Lhi;
                L = Lhi;
                v = v_hi;
            } else {
                continue;
            }
            if (!(depth > 0.0)) continue;
            const double d0 = -(npow + 1.0) * v * std::log(R) / (2.0 * L);
            const double d = d0 * std::pow(depth, npow);
            const double alpha = alpha_max * (1.0 - depth);
            b[i] = std::exp(-(d + alpha) * dt);
            a[i] = d * (b[i] - 1.0) / (d + alpha);
        }
    }
    return c;
}

int point_stencil(const std::vector<double> &coords, double p, int r, double *w) {
    // m = last index with coords[m] <= p
    const int m = static_cast<int>(std::upper_bound(coords.begin(), coords.end(), p) - coords.begin()) - 1;
    const int base = m - r + 1;
    const int L = 2 * r;
    if (base < 0 || base + L > static_cast<int>(coords.size())) return base;
    std::vector<double> t(L);
    for (int q = 0; q < L; ++q) t[q] = coords[base + q] - p;
    const std::vector<double> W = vandermonde_inverse(t);
    for (int q = 0; q < L; ++q) w[q] = W[q];      // row 0: interpolation weights
    return base;
}

std::vector<double> wavelet(int nt, double dt, double fp) {
    const double pi = 3.14159265358979323846;
    const double tau = 1.0 / (pi * fp);
    std::vector<double> s(nt);
    for (int n = 0; n < nt; ++n) {
        const double u = ((n + 0.5) * dt - 4.0 * tau) / tau;
        s[n] = -u * std::exp(-u * u);
    }
    return s;
}

std::complex<double> omega_prime(double f, double omega0) {
    const double pi = 3.14159265358979323846;
    const double g = std::sqrt(2.0 * pi * f * omega0);
    return {g, g};
}

}  // namespace emm
