// HIP kernels of the discrete adjoint of the time loop (reverse of one
// leap-frog step of Section 3.1 with the CPML recursion of Section 3.4).
//
// Adjoint variables: Et = (dt/eps) * Ebar (the E adjoint scaled by the
// per-cell coefficient) and Hb = Hbar.  Reverse of step n, in order:
//   1. reverse of the H update: Et += (dt/eps) dt/mu0 curlT(F(Hb)), with
//      the transposed D+ tables (their stencil has the D- shape);
//   2. receiver sources of the E channels (stamp (n+1) dt);
//   3. reverse of the E update: grad += Ebar (E^{n+1} - E^n) and
//      Hb -= curlT(F(Et)), with the transposed D- tables (D+ shape);
//   4. receiver sources of the H channels (stamp (n+1/2) dt).
// The curl structure is the forward one (component 1 has y and z taps,
// component 2 x and z, component 3 x and y).  F is the reverse of the CPML
// recursion psi = b psi + a d, d~ = d + psi, applied to the inputs of every
// derivative inside its slab: psibar = b Q + v, Q = psibar, v~ = v + a psibar
// (Q carried backwards in time).  Because F of a tap depends on that tap's
// own memory variable, a slab-only kernel applies it first and writes the
// filtered values to slab arrays that the gather reads instead of the raw
// field.
#include "emm_adjoint.h"

namespace emm {

constexpr int AT = 256;

// slab index of position i on an axis of n nodes, or -1 outside the slabs
__device__ __forceinline__ int slab_index(int i, int n, int nb) {
    return i < nb ? i : (i > n - 1 - nb ? i - (n - 2 * nb) : -1);
}

// 1. CPML reverse filter on the slab cells of the update set, for the six
// (input component, tap axis) pairs.  One thread per slab cell of one axis.
// REV_H = true: inputs Hb, half-node tables (reverse of the H update);
// REV_H = false: inputs Et, integer-node tables (reverse of the E update).
template <bool REV_H>
__global__ __launch_bounds__(AT) void adj_filter(const AdjParams p) {
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const int r = p.r, nb = p.nb, nb2 = 2 * p.nb;
    const long long nx = (long long)p.n3 * p.n2 * nb2, ny = (long long)p.n3 * nb2 * p.n1,
                    nz = (long long)nb2 * p.n2 * p.n1;
    const long long per_src = nx + ny + nz;
    if (t >= per_src * p.nsrc) return;
    const int s = (int)(t / per_src);
    long long u = t - (long long)s * per_src;
    int axis, i, j, k, si;
    if (u < nx) {
        axis = 0;
        si = (int)(u % nb2);
        u /= nb2;
        j = (int)(u % p.n2);
        k = (int)(u / p.n2);
        i = si < nb ? si : si + (p.n1 - nb2);
    } else if (u < nx + ny) {
        axis = 1;
        u -= nx;
        i = (int)(u % p.n1);
        u /= p.n1;
        si = (int)(u % nb2);
        k = (int)(u / nb2);
        j = si < nb ? si : si + (p.n2 - nb2);
    } else {
        axis = 2;
        u -= nx + ny;
        i = (int)(u % p.n1);
        u /= p.n1;
        j = (int)(u % p.n2);
        si = (int)(u / p.n2);
        k = si < nb ? si : si + (p.n3 - nb2);
    }
    if (i < r || i > p.n1 - 1 - r || j < r || j > p.n2 - 1 - r || k < r || k > p.n3 - 1 - r) return;
    const long long g = ((long long)k * p.n2 + j) * p.pitch + i + (long long)s * p.fstride;
    const float *in[3] = {p.in1, p.in2, p.in3};
    // slab array index (layouts: x [n3][n2][2nb], y [n3][2nb][pitch], z [2nb][n2][pitch])
    long long id;
    float a, b;
    int c0, c1;  // the two input components with taps along this axis
    const float *A = REV_H ? p.a_half : p.a_int;
    const float *B = REV_H ? p.b_half : p.b_int;
    if (axis == 0) {
        id = ((long long)k * p.n2 + j) * nb2 + si + (long long)s * p.sxs;
        a = A[i];
        b = B[i];
        c0 = 1;
        c1 = 2;
    } else if (axis == 1) {
        id = ((long long)k * nb2 + si) * p.pitch + i + (long long)s * p.sys;
        a = A[p.n1 + j];
        b = B[p.n1 + j];
        c0 = 0;
        c1 = 2;
    } else {
        id = ((long long)si * p.n2 + j) * p.pitch + i + (long long)s * p.szs;
        a = A[p.n1 + p.n2 + k];
        b = B[p.n1 + p.n2 + k];
        c0 = 0;
        c1 = 1;
    }
    float *Q0 = p.Q[2 * axis], *Q1 = p.Q[2 * axis + 1];
    float *T0 = p.T[2 * axis], *T1 = p.T[2 * axis + 1];
    const float v0 = in[c0][g], v1 = in[c1][g];
    const float ps0 = b * Q0[id] + v0, ps1 = b * Q1[id] + v1;
    Q0[id] = ps0;
    Q1[id] = ps1;
    T0[id] = v0 + a * ps0;
    T1[id] = v1 + a * ps1;
}

// value of the CPML-filtered input `comp` (0..2) at a tap position that
// differs from an update-set cell only along `axis`; 0 outside the update set
template <int AXIS>
__device__ __forceinline__ float tap(const AdjParams &p, const float *in, int comp, int s,
                                     int k, int j, int i, long long g) {
    const int r = p.r, nb = p.nb, nb2 = 2 * p.nb;
    const int q = AXIS == 0 ? i : (AXIS == 1 ? j : k);
    const int n = AXIS == 0 ? p.n1 : (AXIS == 1 ? p.n2 : p.n3);
    if (q < r || q > n - 1 - r) return 0.f;
    const int si = slab_index(q, n, nb);
    if (si < 0) return in[g];
    // slab slot of this (comp, axis): x: comps 1,2; y: comps 0,2; z: comps 0,1
    const int slot = AXIS == 0 ? (comp == 1 ? 0 : 1) : (AXIS == 1 ? (comp == 0 ? 0 : 1) : (comp == 0 ? 0 : 1));
    const float *T = p.T[2 * AXIS + slot];
    long long id;
    if (AXIS == 0) id = ((long long)k * p.n2 + j) * nb2 + si + (long long)s * p.sxs;
    else if (AXIS == 1) id = ((long long)k * nb2 + si) * p.pitch + i + (long long)s * p.sys;
    else id = ((long long)si * p.n2 + j) * p.pitch + i + (long long)s * p.szs;
    return T[id];
}

// 2./3. transposed curl gathers.  One thread per (i, j) column of one
// source, looping over z.  REV_H = true: Et += (dt/eps) dtmu curlT(F(Hb))
// with transposed D+ tables (offsets -R..R-1); REV_H = false: gradient,
// then Hb -= scale curlT(F(Et)) (scale 1) with transposed D- tables
// (offsets -R+1..R).
template <int R, bool REV_H>
__global__ __launch_bounds__(AT) void adj_gather(const AdjParams p) {
    constexpr int L = 2 * R;
    constexpr int LO = REV_H ? R : R - 1;      // taps at q - LO .. q - LO + L - 1
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const long long ncol = (long long)p.n2 * p.pitch;
    if (t >= ncol * p.nsrc) return;
    const int s = (int)(t / ncol);
    const long long c = t - (long long)s * ncol;
    const int j = (int)(c / p.pitch), i = (int)(c - (long long)j * p.pitch);
    if (i < R || i > p.n1 - 1 - R || j < R || j > p.n2 - 1 - R) return;
    const long long fo = (long long)s * p.fstride;
    const float *in[3] = {p.in1 + fo, p.in2 + fo, p.in3 + fo};
    float *out1 = p.out1 + fo, *out2 = p.out2 + fo, *out3 = p.out3 + fo;
    const float *tx_ = p.tx + i * L, *ty_ = p.ty + j * L;
    const long long plane = (long long)p.n2 * p.pitch;
    for (int k = R; k <= p.n3 - 1 - R; ++k) {
        const long long g = k * plane + (long long)j * p.pitch + i;
        const float *tz_ = p.tz + k * L;
        // the six transposed derivatives of the filtered inputs
        float dx1 = 0.f, dx2 = 0.f, dy0 = 0.f, dy2 = 0.f, dz0 = 0.f, dz1 = 0.f;
#pragma unroll
        for (int m = 0; m < L; ++m) {
            const int o = m - LO;
            dx1 += tx_[m] * tap<0>(p, in[1], 1, s, k, j, i + o, g + o);
            dx2 += tx_[m] * tap<0>(p, in[2], 2, s, k, j, i + o, g + o);
            dy0 += ty_[m] * tap<1>(p, in[0], 0, s, k, j + o, i, g + (long long)o * p.pitch);
            dy2 += ty_[m] * tap<1>(p, in[2], 2, s, k, j + o, i, g + (long long)o * p.pitch);
            dz0 += tz_[m] * tap<2>(p, in[0], 0, s, k + o, j, i, g + o * plane);
            dz1 += tz_[m] * tap<2>(p, in[1], 1, s, k + o, j, i, g + o * plane);
        }
        // forward curl signs: out1 = D2(c3) - D3(c2), out2 = D3(c1) - D1(c3), out3 = D1(c2) - D2(c1)
        const float c1 = dy2 - dz1, c2 = dz0 - dx2, c3 = dx1 - dy0;
        if (REV_H) {
            out1[g] += p.ce1[g] * p.scale * c1;
            out2[g] += p.ce2[g] * p.scale * c2;
            out3[g] += p.ce3[g] * p.scale * c3;
        } else {
            // gradient wrt log(dt/eps): Ebar (E^{n+1} - E^n), Ebar = Et / (dt/eps)
            const float *En1 = p.E_next + fo, *En = p.E_prev + fo;
            const long long fs3 = (long long)p.nsrc * p.fstride;   // component stride of E snapshots
            double *gr = p.grad + (long long)s * 3 * p.gstride;
            gr[g] += (double)(in[0][g] / p.ce1[g]) * (double)(En1[g] - En[g]);
            gr[g + p.gstride] += (double)(in[1][g] / p.ce2[g]) * (double)(En1[g + fs3] - En[g + fs3]);
            gr[g + 2 * p.gstride] += (double)(in[2][g] / p.ce3[g]) * (double)(En1[g + 2 * fs3] - En[g + 2 * fs3]);
            // Hbar update has the signs of the forward H step
            out1[g] -= p.scale * c1;
            out2[g] -= p.scale * c2;
            out3[g] -= p.scale * c3;
        }
    }
}

// 2./4. receiver adjoint sources: one thread per target cell of the
// injection list (cells sorted, contributions in a fixed order, so the sum
// is deterministic).  dchi/du_n of item q = sum_f Re(A[q][f] ph[n][f]).
__global__ __launch_bounds__(AT) void adj_inject(const InjectParams p, int n) {
    const int t = blockIdx.x * AT + threadIdx.x;
    if (t >= p.ncells) return;
    float acc = 0.f;
    for (int e = p.row[t]; e < p.row[t + 1]; ++e) {
        const int q = p.item[e];
        double sb = 0.0;
        for (int f = 0; f < p.nf; ++f) {
            const double2 A = p.A[(long long)q * p.nf + f];
            const double2 z = p.phase[(long long)n * p.nf + f];
            sb += A.x * z.x - A.y * z.y;
        }
        acc += p.w[e] * (float)sb;
    }
    const long long g = p.cell[t];
    const int comp = p.comp[t];
    float *F = comp == 0 ? p.F1 : (comp == 1 ? p.F2 : p.F3);
    const long long mc = p.mcell[t];
    const float scale = p.scale_ce ? (comp == 0 ? p.ce1[mc] : (comp == 1 ? p.ce2[mc] : p.ce3[mc])) : 1.f;
    F[g] += scale * acc;
}

void launch_adj_filter(bool rev_h, const AdjParams &p, hipStream_t st) {
    const long long per_src = (long long)2 * p.nb * ((long long)p.n3 * p.n2 + (long long)p.n3 * p.n1 +
                                                      (long long)p.n2 * p.n1);
    const long long total = per_src * p.nsrc;
    if (total == 0) return;
    const dim3 grid((unsigned)((total + AT - 1) / AT)), block(AT);
    if (rev_h) hipLaunchKernelGGL(adj_filter<true>, grid, block, 0, st, p);
    else hipLaunchKernelGGL(adj_filter<false>, grid, block, 0, st, p);
}

template <bool REV_H>
static void gather(int r, const AdjParams &p, hipStream_t st) {
    const long long total = (long long)p.n2 * p.pitch * p.nsrc;
    const dim3 grid((unsigned)((total + AT - 1) / AT)), block(AT);
    switch (r) {
    case 1: hipLaunchKernelGGL((adj_gather<1, REV_H>), grid, block, 0, st, p); break;
    case 2: hipLaunchKernelGGL((adj_gather<2, REV_H>), grid, block, 0, st, p); break;
    case 3: hipLaunchKernelGGL((adj_gather<3, REV_H>), grid, block, 0, st, p); break;
    default: hipLaunchKernelGGL((adj_gather<4, REV_H>), grid, block, 0, st, p); break;
    }
}

void launch_adj_gather(int r, bool rev_h, const AdjParams &p, hipStream_t st) {
    if (rev_h) gather<true>(r, p, st);
    else gather<false>(r, p, st);
}

void launch_adj_inject(const InjectParams &p, int n, hipStream_t st) {
    if (p.ncells == 0) return;
    const dim3 grid((p.ncells + AT - 1) / AT), block(AT);
    hipLaunchKernelGGL(adj_inject, grid, block, 0, st, p, n);
}

}  // namespace emm
