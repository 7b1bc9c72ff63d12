// HIP kernels of the discrete adjoint of the time loop (reverse of one
// leap-frog step of Section 3.1 with the CPML recursion of Section 3.4).
//
// Adjoint variables: Et = (dt/eps) * Ebar (the E adjoint scaled by the
// per-cell coefficient) and Hb = Hbar.  Reverse of step n, in order:
//   1. reverse of the H update: Et += (dt/eps) dt/mu0 curlT(F(Hb)), with
//      the transposed D+ tables (their stencil has the D- shape);
//   2. receiver sources of the E channels (stamp (n+1) dt);
//   3. reverse of the E update: grad += Ebar (E^{n+1} - E^n) (summed as
//      Et (E^{n+1} - E^n) in FP32 over a few steps, then divided by dt/eps
//      and added to the FP64 gradient) and
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

// 2./3. transposed curl gathers, in the layout of the forward stencil
// kernel: a TX x (256/TX) tile of columns per 256-thread block marching a
// chunk of kz planes, x/y taps staged in LDS per plane (double-buffered,
// one barrier per plane, the next plane's loads issued right after it),
// z taps in a 2r-deep register queue.  Because the CPML reverse filter
// makes the tap value depend on the tap axis inside a slab, the staged
// copies are per (component, axis): the x taps of components 2 and 3 over
// the own rows with the x halo, the y taps of components 1 and 3 over the
// own columns with the y halo; every staged value is the filtered one (the
// slab array T inside the slab of its axis, the field elsewhere, zero off
// the update set on that axis).  CI (reverse of the H update only): dt/eps
// from the compact form, the table in LDS.
// planes of loads in flight per thread: two at 8th order, as in step_kernel
template <int R, bool REV_H, bool CI, int TX, int PF = (R >= 4 ? 2 : 1)>
__global__ __launch_bounds__(kTileX * kTileY) void adj_tile(const AdjParams p) {
    constexpr int NT = kTileX * kTileY, TY = NT / TX;
    static_assert(TX * TY == NT && (TX & (TX - 1)) == 0, "tile of NT threads, power-of-two width");
    constexpr int L = 2 * R;
    constexpr int HL = REV_H ? R : R - 1;     // taps at q - HL .. q - HL + L - 1
    constexpr int W = TX + L - 1;
    constexpr int HR = TY + L - 1;
    constexpr int NX = (TY * W + NT - 1) / NT;        // x-type staging loads per thread
    constexpr int NY = (HR * TX + NT - 1) / NT;       // y-type staging loads per thread
    __shared__ float s3x[2][TY][W], s2x[2][TY][W];    // x taps of components 3 and 2
    __shared__ float s3y[2][HR][TX], s1y[2][HR][TX];  // y taps of components 3 and 1
    __shared__ float sCe[CI ? kCeTable : 1];
    static_assert(kCeTable <= NT, "one table entry per thread");
    // read only after the first barrier of the plane loop
    if (CI && (int)threadIdx.x < p.ncet) sCe[threadIdx.x] = p.cet[threadIdx.x];

    int t = xcd_tile(blockIdx.x, p.nstencil);
    const int s = tile_source(t, p.nsrc, p.nstencil, p.sorder);
    const int bxt = t % p.xt;
    t /= p.xt;
    const int byt = t % p.yt;
    const int bzt = t / p.yt;
    const int tid = threadIdx.x, tx = tid & (TX - 1), ty = tid / TX;
    const int i0 = bxt * TX, j0 = R + byt * TY;
    const int i = i0 + tx, j = j0 + ty;
    const int k0 = R + bzt * p.kz, k1 = min(k0 + p.kz, p.n3 - R);
    const bool valid = i >= R && i <= p.n1 - 1 - R && j <= p.n2 - 1 - R;
    const int jc = min(j, p.n2 - 1);
    const int nb = p.nb, nb2 = 2 * p.nb;
    const int plane = p.n2 * p.pitch;
    const long long fo = (long long)s * p.fstride;
    const float *A1 = p.in1 + fo, *A2 = p.in2 + fo, *A3 = p.in3 + fo;
    // slab arrays of this source: x [n3][n2][2nb], y [n3][2nb][pitch], z [2nb][n2][pitch]
    const float *Tx2 = p.T[0] + s * p.sxs, *Tx3 = p.T[1] + s * p.sxs;
    const float *Ty1 = p.T[2] + s * p.sys, *Ty3 = p.T[3] + s * p.sys;
    const float *Tz1 = p.T[4] + s * p.szs, *Tz2 = p.T[5] + s * p.szs;
    const int xplane = p.n2 * nb2, yplane = nb2 * p.pitch;

    const int ic = valid ? i : R;
    float cx[L], cy[L];
#pragma unroll
    for (int m = 0; m < L; ++m) {
        cx[m] = p.tx[ic * L + m];
        cy[m] = p.ty[jc * L + m];
    }
    auto slab = [&](int q, int n) { return q < nb ? q : (q > n - 1 - nb ? q - (n - nb2) : -1); };
    auto on_set = [&](int q, int n) { return q >= R && q <= n - 1 - R; };

    // x-type element u: own row ly, column i0 - HL + lx.  Per element: field
    // offset in the plane (or -1: zero), x-slab offset in the plane (or -1).
    int xo[NX], xs[NX];
#pragma unroll
    for (int u = 0; u < NX; ++u) {
        const int e = tid + u * NT;
        const int ly = e / W, lx = e - ly * W;
        const int gj = j0 + ly, gi = i0 - HL + lx;
        const bool in = e < TY * W && gj < p.n2 && gi >= 0 && gi < p.n1 && on_set(gi, p.n1);
        const int si = in ? slab(gi, p.n1) : -1;
        xo[u] = in ? gj * p.pitch + gi : -1;
        xs[u] = si >= 0 ? gj * nb2 + si : -1;
    }
    // y-type element u: row j0 - HL + ly, own column
    int yo[NY], ys[NY];
#pragma unroll
    for (int u = 0; u < NY; ++u) {
        const int e = tid + u * NT;
        const int ly = e / TX, lx = e & (TX - 1);
        const int gj = j0 - HL + ly, gi = i0 + lx;
        const bool in = e < HR * TX && gj >= 0 && gj < p.n2 && on_set(gj, p.n2) && gi < p.pitch;
        const int si = in ? slab(gj, p.n2) : -1;
        yo[u] = in ? gj * p.pitch + gi : -1;
        ys[u] = si >= 0 ? si * p.pitch + gi : -1;
    }
    const int own = jc * p.pitch + i;
    const int ownz = jc * p.pitch + i;               // offset inside a z-slab plane
    // z-filtered value of component (1: A1/Tz1, 2: A2/Tz2) at plane kk of the own column
    auto zval = [&](const float *A, const float *Tz, int kk) -> float {
        if (kk < R || kk > p.n3 - 1 - R) return 0.f;
        const int sk = slab(kk, p.n3);
        return sk >= 0 ? Tz[(unsigned)(sk * plane + ownz)] : A[(unsigned)(kk * plane + own)];
    };
    float q1[L], q2[L];
#pragma unroll
    for (int m = 0; m < L - 1; ++m) {
        q1[m] = zval(A1, Tz1, k0 - HL + m);
        q2[m] = zval(A2, Tz2, k0 - HL + m);
    }
    float *O1 = p.out1 + fo, *O2 = p.out2 + fo, *O3 = p.out3 + fo;
    const long long fs3 = (long long)p.nsrc * p.fstride;     // component stride of E snapshots
    const float *En1 = REV_H ? nullptr : p.E_next + fo, *En = REV_H ? nullptr : p.E_prev + fo;
    float *gr = REV_H ? nullptr : p.grad32 + (long long)s * 3 * p.gstride;

    // staged registers of a plane in flight; PF sets, so that the loads of PF
    // planes are in flight while one is computed
    struct Stage {
        float f3x[NX], f2x[NX], f3y[NY], f1y[NY], e1n, e2n;
        float o1, o2, o3, w1, w2, w3;
        float gn1, gn2, gn3;                  // FP32 gradient partial sums (reverse of the E update)
        float xa1, xa2, xa3, xn1, xn2, xn3, xp1, xp2, xp3;
        unsigned wi;
    };
    auto issue = [&](Stage &S, int k) {
        float(&f3x)[NX] = S.f3x;
        float(&f2x)[NX] = S.f2x;
        float(&f3y)[NY] = S.f3y;
        float(&f1y)[NY] = S.f1y;
        float &e1n = S.e1n, &e2n = S.e2n, &o1 = S.o1, &o2 = S.o2, &o3 = S.o3, &w1 = S.w1, &w2 = S.w2, &w3 = S.w3;
        float &gn1 = S.gn1, &gn2 = S.gn2, &gn3 = S.gn3, &xa1 = S.xa1, &xa2 = S.xa2, &xa3 = S.xa3;
        float &xn1 = S.xn1, &xn2 = S.xn2, &xn3 = S.xn3, &xp1 = S.xp1, &xp2 = S.xp2, &xp3 = S.xp3;
        unsigned &wi = S.wi;
        const int pk = k * plane;
#pragma unroll
        for (int u = 0; u < NX; ++u) {
            f3x[u] = xs[u] >= 0 ? Tx3[(unsigned)(k * xplane + xs[u])] : (xo[u] >= 0 ? A3[(unsigned)(pk + xo[u])] : 0.f);
            f2x[u] = xs[u] >= 0 ? Tx2[(unsigned)(k * xplane + xs[u])] : (xo[u] >= 0 ? A2[(unsigned)(pk + xo[u])] : 0.f);
        }
#pragma unroll
        for (int u = 0; u < NY; ++u) {
            f3y[u] = ys[u] >= 0 ? Ty3[(unsigned)(k * yplane + ys[u])] : (yo[u] >= 0 ? A3[(unsigned)(pk + yo[u])] : 0.f);
            f1y[u] = ys[u] >= 0 ? Ty1[(unsigned)(k * yplane + ys[u])] : (yo[u] >= 0 ? A1[(unsigned)(pk + yo[u])] : 0.f);
        }
        e1n = zval(A1, Tz1, k - HL + L - 1);
        e2n = zval(A2, Tz2, k - HL + L - 1);
        if (valid) {
            const unsigned g = (unsigned)(pk + own);
            o1 = O1[g];
            o2 = O2[g];
            o3 = O3[g];
            if (REV_H && CI) {
                wi = p.cei[g];
            } else if (REV_H) {
                w1 = p.ce1[g];
                w2 = p.ce2[g];
                w3 = p.ce3[g];
            } else {
                // raw Et at the own cell, E^{n+1} and E^n (their product is
                // formed when the plane is computed, after the loads landed)
                xa1 = A1[g];
                xa2 = A2[g];
                xa3 = A3[g];
                xn1 = En1[g];
                xn2 = En1[g + fs3];
                xn3 = En1[g + 2 * fs3];
                xp1 = En[g];
                xp2 = En[g + fs3];
                xp3 = En[g + 2 * fs3];
                gn1 = gr[g];
                gn2 = gr[g + p.gstride];
                gn3 = gr[g + 2 * p.gstride];
            }
        }
    };
    auto step = [&](Stage &S, int k) {
        const int b = (k - k0) & 1;
        const float(&f3x)[NX] = S.f3x;
        const float(&f2x)[NX] = S.f2x;
        const float(&f3y)[NY] = S.f3y;
        const float(&f1y)[NY] = S.f1y;
        q1[L - 1] = S.e1n;
        q2[L - 1] = S.e2n;
#pragma unroll
        for (int u = 0; u < NX; ++u)
            if (u < NX - 1 || tid + u * NT < TY * W) {
                (&s3x[b][0][0])[tid + u * NT] = f3x[u];
                (&s2x[b][0][0])[tid + u * NT] = f2x[u];
            }
#pragma unroll
        for (int u = 0; u < NY; ++u)
            if (u < NY - 1 || tid + u * NT < HR * TX) {
                (&s3y[b][0][0])[tid + u * NT] = f3y[u];
                (&s1y[b][0][0])[tid + u * NT] = f1y[u];
            }
        const float u1 = S.o1, u2 = S.o2, u3 = S.o3;
        const float g1 = S.gn1, g2 = S.gn2, g3 = S.gn3;
        float v1 = S.w1, v2 = S.w2, v3 = S.w3;
        if (!REV_H) {
            v1 = S.xa1 * (S.xn1 - S.xp1);
            v2 = S.xa2 * (S.xn2 - S.xp2);
            v3 = S.xa3 * (S.xn3 - S.xp3);
        }
        const unsigned vi = S.wi;
        __syncthreads();
        if (k + PF < k1) issue(S, k + PF);
        if (CI) {
            v1 = sCe[vi & 255u];
            v2 = sCe[(vi >> 8) & 255u];
            v3 = sCe[(vi >> 16) & 255u];
        }
        if (valid) {
            const cfloat *cz = uniform_table(p.tz + k * L);
            float d2a3 = 0.f, d2a1 = 0.f, d1a3 = 0.f, d1a2 = 0.f, d3a2 = 0.f, d3a1 = 0.f;
#pragma unroll
            for (int m = 0; m < L; ++m) {
                d2a3 += cy[m] * s3y[b][ty + m][tx];
                d2a1 += cy[m] * s1y[b][ty + m][tx];
                d1a3 += cx[m] * s3x[b][ty][tx + m];
                d1a2 += cx[m] * s2x[b][ty][tx + m];
                d3a2 += cz[m] * q2[m];
                d3a1 += cz[m] * q1[m];
            }
            const float c1 = d2a3 - d3a2, c2 = d3a1 - d1a3, c3 = d1a2 - d2a1;
            const unsigned g = (unsigned)(k * plane + own);
            if (REV_H) {
                O1[g] = u1 + v1 * p.scale * c1;
                O2[g] = u2 + v2 * p.scale * c2;
                O3[g] = u3 + v3 * p.scale * c3;
            } else {
                gr[g] = g1 + v1;
                gr[g + p.gstride] = g2 + v2;
                gr[g + 2 * p.gstride] = g3 + v3;
                O1[g] = u1 - p.scale * c1;
                O2[g] = u2 - p.scale * c2;
                O3[g] = u3 - p.scale * c3;
            }
        }
#pragma unroll
        for (int m = 0; m < L - 1; ++m) {
            q1[m] = q1[m + 1];
            q2[m] = q2[m + 1];
        }
    };
    Stage SA = {}, SB = {};
    issue(SA, k0);
    int k = k0;
    if (PF == 2) {
        if (k0 + 1 < k1) issue(SB, k0 + 1);
        for (; k + 1 < k1; k += 2) {
            step(SA, k);
            step(SB, k + 1);
        }
        if (k < k1) step(SA, k);
    } else {
        for (; k < k1; ++k) step(SA, k);
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

// grad += grad32 / (dt/eps), grad32 = 0, over every cell of every source
__global__ __launch_bounds__(AT) void adj_flush(const AdjParams p) {
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const long long per_src = 3 * p.gstride;
    if (t >= per_src * p.nsrc) return;
    const long long u = t % per_src;
    const int c = (int)(u / p.gstride);
    const long long g = u - (long long)c * p.gstride;
    const float *ce = c == 0 ? p.ce1 : (c == 1 ? p.ce2 : p.ce3);
    const float v = p.grad32[t];
    if (v != 0.f) {
        p.grad[t] += (double)v / (double)ce[g];
        p.grad32[t] = 0.f;
    }
}

// out[((c nd2 + kk) nd1 + jj) nd0 + ii] = (accumulate ? out : 0) - sum over
// sources s, then the padded cells (k, j, i) of the update set that fold
// onto input cell (ii, jj, kk) (the padding layers onto the edge cells), in
// increasing k, j, i, of grad[s][c][k][j][i]: the sum over sources and the
// fold of the model padding, in a fixed order per output.
__global__ __launch_bounds__(AT) void adj_fold(const double *grad, double *out, int nsrc, long long fstride,
                                               long long plane, int pitch, int n1, int n2, int n3, int r, int nbe,
                                               int nd0, int nd1, int nd2, int accumulate) {
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const long long per = (long long)nd0 * nd1 * nd2;
    if (t >= 3 * per) return;
    const int c = (int)(t / per);
    long long u = t - (long long)c * per;
    const int kk = (int)(u / ((long long)nd0 * nd1));
    u -= (long long)kk * nd0 * nd1;
    const int jj = (int)(u / nd0), ii = (int)(u - (long long)jj * nd0);
    const int i0 = ii == 0 ? r : ii + nbe, i1 = ii == nd0 - 1 ? n1 - 1 - r : ii + nbe;
    const int j0 = jj == 0 ? r : jj + nbe, j1 = jj == nd1 - 1 ? n2 - 1 - r : jj + nbe;
    const int k0 = kk == 0 ? r : kk + nbe, k1 = kk == nd2 - 1 ? n3 - 1 - r : kk + nbe;
    double acc = accumulate ? out[t] : 0.0;
    for (int s = 0; s < nsrc; ++s) {
        const double *g = grad + ((long long)s * 3 + c) * fstride;
        for (int k = k0; k <= k1; ++k)
            for (int j = j0; j <= j1; ++j)
                for (int i = i0; i <= i1; ++i) acc -= g[(long long)k * plane + (long long)j * pitch + i];
    }
    out[t] = acc;
}

void launch_adj_fold(const double *grad, double *out, int nsrc, long long fstride, long long plane, int pitch,
                     int n1, int n2, int n3, int r, int nbe, int nd0, int nd1, int nd2, bool accumulate,
                     hipStream_t st) {
    const long long total = 3LL * nd0 * nd1 * nd2;
    const dim3 grid((unsigned)((total + AT - 1) / AT)), block(AT);
    hipLaunchKernelGGL(adj_fold, grid, block, 0, st, grad, out, nsrc, fstride, plane, pitch, n1, n2, n3, r, nbe, nd0,
                       nd1, nd2, accumulate ? 1 : 0);
}

void launch_adj_flush(const AdjParams &p, hipStream_t st) {
    const long long total = 3 * p.gstride * p.nsrc;
    const dim3 grid((unsigned)((total + AT - 1) / AT)), block(AT);
    hipLaunchKernelGGL(adj_flush, grid, block, 0, st, p);
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

template <bool REV_H, bool CI, int TX>
static void tiled(int r, const AdjParams &p, hipStream_t st) {
    const dim3 grid(p.nstencil), block(kTileX * kTileY);
    switch (r) {
    case 1: hipLaunchKernelGGL((adj_tile<1, REV_H, CI, TX>), grid, block, 0, st, p); break;
    case 2: hipLaunchKernelGGL((adj_tile<2, REV_H, CI, TX>), grid, block, 0, st, p); break;
    case 3: hipLaunchKernelGGL((adj_tile<3, REV_H, CI, TX>), grid, block, 0, st, p); break;
    default: hipLaunchKernelGGL((adj_tile<4, REV_H, CI, TX>), grid, block, 0, st, p); break;
    }
}

void launch_adj_tile(int r, bool rev_h, const AdjParams &p, hipStream_t st) {
    const bool w32 = p.tw == 32;
    if (rev_h && p.cei) {
        if (w32) tiled<true, true, 32>(r, p, st);
        else tiled<true, true, 64>(r, p, st);
    } else if (rev_h) {
        if (w32) tiled<true, false, 32>(r, p, st);
        else tiled<true, false, 64>(r, p, st);
    } else {
        if (w32) tiled<false, false, 32>(r, p, st);
        else tiled<false, false, 64>(r, p, st);
    }
}

void launch_adj_inject(const InjectParams &p, int n, hipStream_t st) {
    if (p.ncells == 0) return;
    const dim3 grid((p.ncells + AT - 1) / AT), block(AT);
    hipLaunchKernelGGL(adj_inject, grid, block, 0, st, p, n);
}

}  // namespace emm
