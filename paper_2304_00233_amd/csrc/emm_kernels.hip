// HIP kernels of the fictitious-wave-domain FDTD hot path, written for
// CDNA4 (gfx950).
//
// One kernel template serves both half steps of the leap-frog scheme
// (Section 3.1):
//   E step:  E += (dt/eps) (curl H - J)   curl with D- (eq. HFD2), J = dipole
//   H step:  H -= (dt/mu0)  curl E        curl with D+ (eq. HFD1)
// fused with the CPML memory-variable recursion psi = b psi + a d,
// d <- d + psi inside the absorbing slabs (Section 3.4), the electric dipole
// injection (E step only) and, in extra waves of the same launch, the
// receiver interpolation plus the on-the-fly DTFT of Section 3.5 for the
// fields the kernel only reads (H channels in the E step, E channels in the
// H step).  No curl arrays are written (the paper's curl and update kernels
// are one pass here).
//
// Arrays that a launch touches once (the updated field, dt/eps) can be
// moved with nontemporal hints (p.stream): on grids whose working set is
// larger than the Infinity Cache this keeps the cache for the re-read halo
// planes; on smaller grids plain accesses let the arrays stay resident
// between steps.  The autotuner times both.
//
// Work decomposition: a 256-thread block covers a 64 (x) by 4 (y) or a 32
// by 8 tile of columns and marches a chunk of z planes.  A wavefront owns
// one 64-wide row along x, or two 32-wide rows (coalesced 256- or 128-byte
// accesses per row segment).  Per plane, the x/y stencil
// operands are staged in LDS with their halos; the two z-differentiated
// components live in a 2r-deep register queue per column, so every plane of
// them is loaded once.  Tiles are mapped to the eight XCDs in contiguous
// ranges so that neighbouring tiles share an L2.
#include "emm_internal.h"

#include <hip/hip_ext.h>

#include <algorithm>

namespace emm {

constexpr int TY = kTileY;
constexpr int NT = kTileX * TY;

int block_threads() { return NT; }

// Planes of loads in flight per thread in step_kernel's plane loop: two at
// 8th order (E/H steps 3-4 % faster on the large grid, 8 sources or one,
// despite 149-155 registers and 3 waves per SIMD), one below (a second set
// costs the 2nd-order kernels a wave per SIMD and 24 % on the marine grid).
template <int R>
constexpr int prefetch_planes() { return R >= 4 ? 2 : 1; }

// CPML memory-variable update psi <- b psi + a d, with one fixed rounding
// (b psi fused onto the rounded a d) in every kernel, so that all tile shapes
// and the fused step give the same bits.
__device__ __forceinline__ float cpml_mem(float b, float psi, float a, float d) {
    return __builtin_fmaf(b, psi, a * d);
}

template <bool ST, typename T>
__device__ __forceinline__ T ld1(const T *p) {
    if constexpr (ST) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool ST>
__device__ __forceinline__ void st1(float *p, float v) {
    if constexpr (ST) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Receiver sample + DTFT: one wavefront per (source, receiver, channel)
// item.  u = sum over the (2r)^3 tensor-product stencil of w * F, reduced in
// FP64; then acc[f] += u * exp(i w'_f t_n) for every frequency (lane l takes
// frequencies l, l + 64, ...).
template <int R>
__device__ void rec_dft(const StepParams &p, int blk, const float *F0,
                        const float *F1, const float *F2, int n, int waves = NT / 64) {
    constexpr int L = 2 * R;
    const int lane = threadIdx.x & 63;
    const int item = blk * waves + (threadIdx.x >> 6);
    if (item >= p.nitems) return;
    const int *inf = p.item_info + 6 * item;
    const int s = inf[0], f = inf[1], bx = inf[2], by = inf[3], bz = inf[4], slot = inf[5];
    const float *w = p.item_w + 3 * L * item;
    const float *F = (f == 0 ? F0 : (f == 1 ? F1 : F2)) + (long long)s * p.fstride;
    double u = 0.0;
    for (int q = lane; q < L * L * L; q += 64) {
        const int a = q % L, b = (q / L) % L, c = q / (L * L);
        const float wt = w[a] * w[L + b] * w[2 * L + c];
        u += (double)wt * (double)F[(unsigned)((bz + c) * (int)p.plane + (by + b) * p.pitch + bx + a)];
    }
    for (int off = 32; off > 0; off >>= 1) u += __shfl_xor(u, off, 64);
    // lane fr updates frequencies fr, fr + 64, ... (any number of them)
    for (int fr = lane; fr < p.nf; fr += 64) {
        const double2 ph = p.phase[(long long)n * p.nf + fr];
        const long long k = (long long)slot * p.nf + fr;
        if (p.dft_mode == 0) {
            double2 a = p.acc[k];
            a.x += u * ph.x;
            a.y += u * ph.y;
            p.acc[k] = a;
        } else {
            // FP32 Kahan-compensated sum: (re, c_re, im, c_im)
            float4 a = p.acck[k];
            const float uf = (float)u;
            const float xr = uf * (float)ph.x, xi = uf * (float)ph.y;
            float y = xr - a.y, t = a.x + y;
            a.y = (t - a.x) - y;
            a.x = t;
            y = xi - a.w;
            t = a.z + y;
            a.w = (t - a.z) - y;
            a.z = t;
            p.acck[k] = a;
        }
    }
}

// ST: nontemporal hints on the updated field and dt/eps.
// HS = false: E step (reads H, updates E, D- tables, integer-node CPML,
//             injects J, records H channels);
// HS = true:  H step (reads E, updates H, D+ tables, half-node CPML,
//             records E channels).
//
// Per plane k the loop (i) moves the staged operands of plane k from
// registers into one of two LDS buffers, (ii) passes one barrier, (iii)
// issues every global load of plane k+1 (staging, queue edge, updated field,
// dt/eps), and (iv) computes plane k from LDS and registers while those
// loads are in flight.  Two LDS buffers make one barrier per plane enough: a
// buffer is rewritten only after every wave has passed the barrier that
// follows its last use.
//
// CI (E step only): dt/eps comes from the compact form, one index word per
// cell (4 bytes instead of 12) into a table of the model's distinct values,
// held in LDS.  TX: tile width (TX x NT/TX columns per block).
template <int R, bool HS, bool ST, bool CI, int TX, int PF = prefetch_planes<R>()>
__global__ __launch_bounds__(NT) void step_kernel(const StepParams p, int n_arg) {
    const int n = (p.step_base ? *p.step_base : 0) + n_arg;
    constexpr int L = 2 * R;
    constexpr int TYS = NT / TX;
    static_assert(TX * TYS == NT && (TX & (TX - 1)) == 0, "tile of NT threads, power-of-two width");
    constexpr int HL = HS ? R - 1 : R;        // halo below the own index
    constexpr int W = TX + L - 1;             // LDS row length incl. halo
    constexpr int HR = TYS + L - 1;           // LDS rows incl. halo
    constexpr int N3 = (HR * W + NT - 1) / NT;              // A3 staging loads per thread
    constexpr int N1 = ((L - 1) * TX + NT - 1) / NT;        // A1 halo loads per thread
    __shared__ float sA3[2][HR][W];           // x and y taps
    __shared__ float sA2[2][TYS][W];          // x taps
    __shared__ float sA1[2][HR][TX];          // y taps
    __shared__ float sCe[CI ? kCeTable : 1];
    static_assert(kCeTable <= NT, "one table entry per thread");

    const float *A1 = HS ? p.E1 : p.H1;
    const float *A2 = HS ? p.E2 : p.H2;
    const float *A3 = HS ? p.E3 : p.H3;

    const int blk = blockIdx.x;
    if (blk < p.nrecblk) {
        rec_dft<R>(p, blk, A1, A2, A3, n);
        return;
    }
    // logical tile: source fastest (the blocks of all sources for one
    // spatial tile run together on one XCD and share the model and table
    // reads through L2) or slowest (each XCD streams whole sources, and
    // neighbouring tiles of one source share their halos through L2), then
    // x, y, z chunk
    int t = xcd_tile(blk - p.nrecblk, p.nstencil);
    const int s = tile_source(t, p.nsrc, p.nstencil, p.sorder);
    const int bxt = t % p.xt;
    t /= p.xt;
    const int byt = t % p.yt;
    const int bzt = t / p.yt;

    // With 64-wide tiles the row index is wave-uniform (one row per
    // wavefront); declaring it so moves the y coefficients and y-slab values
    // to scalar registers, which pays in the E step and in the H step at
    // 8th order.
    constexpr bool kScalarRow = TX == 64 && (!HS || R >= 4);
    const int tid = threadIdx.x, tx = tid & (TX - 1);
    const int ty = kScalarRow ? __builtin_amdgcn_readfirstlane(tid / TX) : tid / TX;
    const int i0 = bxt * TX, j0 = R + byt * TYS;
    const int i = i0 + tx, j = j0 + ty;
    const int k0 = p.kmin + bzt * p.kz;
    const int k1 = min(k0 + p.kz, p.n3 - R);
    const bool valid = i >= R && i <= p.n1 - 1 - R && j <= p.n2 - 1 - R;
    const int jc = min(j, p.n2 - 1);
    const long long fo = (long long)s * p.fstride;   // per-block (uniform) base offset
    A1 += fo;
    A2 += fo;
    A3 += fo;
    const int plane = (int)p.plane;                   // 32-bit offsets below this base
    const float *U1 = (HS ? p.H1 : p.E1) + fo;
    const float *U2 = (HS ? p.H2 : p.E2) + fo;
    const float *U3 = (HS ? p.H3 : p.E3) + fo;
    float *O1 = (HS ? p.H1 : p.Eo1) + fo;     // updated field (E may go out of place)
    float *O2 = (HS ? p.H2 : p.Eo2) + fo;
    float *O3 = (HS ? p.H3 : p.Eo3) + fo;

    const float *tx_ = HS ? p.cpx : p.cmx;
    const float *ty_ = HS ? p.cpy : p.cmy;
    const float *tz_ = HS ? p.cpz : p.cmz;
    const int ic = valid ? i : R;
    float cx[L], cy[L];
#pragma unroll
    for (int m = 0; m < L; ++m) {
        cx[m] = tx_[ic * L + m];
        cy[m] = ty_[jc * L + m];
    }

    // CPML slabs: index < nb or > n - 1 - nb on the derivative's own axis
    const int nb = p.nb, nb2 = 2 * p.nb;
    const bool xs = valid && (i < nb || i > p.n1 - 1 - nb);
    const bool ys = valid && (j < nb || j > p.n2 - 1 - nb);
    float ax = 0.f, bx = 0.f, ay = 0.f, by = 0.f;
    int ix = 0, jy = 0;
    if (xs) {
        ax = (HS ? p.axh : p.axi)[i];
        bx = (HS ? p.bxh : p.bxi)[i];
        ix = i < nb ? i : i - (p.n1 - nb2);
    }
    if (ys) {
        ay = (HS ? p.ayh : p.ayi)[j];
        by = (HS ? p.byh : p.byi)[j];
        jy = j < nb ? j : j - (p.n2 - nb2);
    }
    const float *az_ = HS ? p.azh : p.azi;
    const float *bz_ = HS ? p.bzh : p.bzi;
    float *px0 = p.psx0 + s * p.psxs, *px1 = p.psx1 + s * p.psxs;
    float *py0 = p.psy0 + s * p.psys, *py1 = p.psy1 + s * p.psys;
    float *pz0 = p.psz0 + s * p.pszs, *pz1 = p.psz1 + s * p.pszs;
    const float *ce1 = p.ce1, *ce2 = p.ce2, *ce3 = p.ce3;
    // read only after the first barrier of the plane loop
    if (CI && (int)threadIdx.x < p.ncet) sCe[threadIdx.x] = p.cet[threadIdx.x];

    // dipole source of this block's source (E step only)
    int scomp = -1, sbx = 0, sby = 0, sbz = 0;
    float sn = 0.f;
    const float *sq = nullptr;
    if (!HS) {
        scomp = p.src_info[4 * s];
        sbx = p.src_info[4 * s + 1];
        sby = p.src_info[4 * s + 2];
        sbz = p.src_info[4 * s + 3];
        sn = p.wavelet[n];
        sq = p.src_q + (long long)s * L * L * L;
    }

    // Staging map (identical for every plane): element e of the A3 tile is
    // row e / W, column e % W of the LDS tile, i.e. global (j0 - HL + row,
    // i0 - HL + col); out-of-array elements stage zeros.
    // (LDS index of A3 element u: tid + u * NT; of A1 halo element u: row
    // ly1(u) * TX + tx.)
    int o3[N3];        // plane offset, or -1 (outside the array or the tile)
#pragma unroll
    for (int u = 0; u < N3; ++u) {
        const int e = tid + u * NT;
        const int ly = e / W, lx = e - ly * W;
        const int gj = j0 - HL + ly, gi = i0 - HL + lx;
        o3[u] = (e < HR * W && gj >= 0 && gj < p.n2 && gi >= 0 && gi < p.pitch) ? gj * p.pitch + gi : -1;
    }
    auto ly1 = [&](int u) {
        const int hy = (tid + u * NT) / TX;
        return hy < HL ? hy : TYS + hy;
    };
    int o1[N1];
#pragma unroll
    for (int u = 0; u < N1; ++u) {
        const int e = tid + u * NT;
        const int gj = j0 - HL + ly1(u);
        o1[u] = (e < (L - 1) * TX && gj >= 0 && gj < p.n2) ? gj * p.pitch + i0 + tx : -1;
    }
    int o2 = -1, l2 = -1;
    if (tid < TYS * (L - 1)) {
        const int hy = tid / (L - 1), hx = tid % (L - 1);
        const int lx = hx < HL ? hx : TX + hx;
        const int gi = i0 - HL + lx, gj = min(j0 + hy, p.n2 - 1);
        l2 = hy * W + lx;
        o2 = (gi >= 0 && gi < p.pitch) ? gj * p.pitch + gi : -1;
    }
    const int own = jc * p.pitch + i;          // plane offset of this thread's column

    // z queues of the two z-differentiated components: planes k-HL .. k-HL+L-1
    float q1[L], q2[L];
#pragma unroll
    for (int m = 0; m < L - 1; ++m) {
        q1[m] = A1[(unsigned)((k0 - HL + m) * plane + own)];
        q2[m] = A2[(unsigned)((k0 - HL + m) * plane + own)];
    }

    // staged registers of a plane in flight (fields, dt/eps and the CPML
    // memory variables of its slab cells); PF sets, so that the loads of PF
    // planes are in flight while one is computed
    struct Stage {
        float f3[N3], f1[N1], f2, e1n, e2n;
        float un1, un2, un3, cn1, cn2, cn3;
        float mxn0, mxn1, myn0, myn1, mzn0, mzn1;
        unsigned cin;
    };
    auto issue = [&](Stage &S, int k) {
        float(&f3)[N3] = S.f3;
        float(&f1)[N1] = S.f1;
        float &f2 = S.f2, &e1n = S.e1n, &e2n = S.e2n, &un1 = S.un1, &un2 = S.un2, &un3 = S.un3;
        float &cn1 = S.cn1, &cn2 = S.cn2, &cn3 = S.cn3, &mxn0 = S.mxn0, &mxn1 = S.mxn1;
        float &myn0 = S.myn0, &myn1 = S.myn1, &mzn0 = S.mzn0, &mzn1 = S.mzn1;
        unsigned &cin = S.cin;
        const int pk = k * plane;
#pragma unroll
        for (int u = 0; u < N3; ++u) f3[u] = o3[u] >= 0 ? A3[(unsigned)(pk + o3[u])] : 0.f;
#pragma unroll
        for (int u = 0; u < N1; ++u) f1[u] = o1[u] >= 0 ? A1[(unsigned)(pk + o1[u])] : 0.f;
        if (o2 >= 0) f2 = A2[(unsigned)(pk + o2)];
        const unsigned ge = (unsigned)((k - HL + L - 1) * plane + own);
        e1n = A1[ge];
        e2n = A2[ge];
        if (valid) {
            if (xs) {
                const unsigned id = (unsigned)((k * p.n2 + j) * nb2 + ix);
                mxn0 = px0[id];
                mxn1 = px1[id];
            }
            if (ys) {
                const unsigned id = (unsigned)((k * nb2 + jy) * p.pitch + i);
                myn0 = py0[id];
                myn1 = py1[id];
            }
            if (k < nb || k > p.n3 - 1 - nb) {
                const int kz = k < nb ? k : k - (p.n3 - nb2);
                const unsigned id = (unsigned)((kz * p.n2 + j) * p.pitch + i);
                mzn0 = pz0[id];
                mzn1 = pz1[id];
            }
            const unsigned g = (unsigned)(pk + own);
            un1 = ld1<ST>(&U1[g]);
            un2 = ld1<ST>(&U2[g]);
            un3 = ld1<ST>(&U3[g]);
            if (!HS && CI) {
                cin = ld1<ST>(&p.cei[g]);
            } else if (!HS) {
                cn1 = ld1<ST>(&ce1[g]);
                cn2 = ld1<ST>(&ce2[g]);
                cn3 = ld1<ST>(&ce3[g]);
            }
        }
    };
    auto step = [&](Stage &S, int k) {
        const int b = (k - k0) & 1;
        const float(&f3)[N3] = S.f3;
        const float(&f1)[N1] = S.f1;
        const float f2 = S.f2;
        q1[L - 1] = S.e1n;
        q2[L - 1] = S.e2n;
        float *s3 = &sA3[b][0][0];
#pragma unroll
        for (int u = 0; u < N3; ++u)
            if (u < N3 - 1 || tid + u * NT < HR * W) s3[tid + u * NT] = f3[u];
        float *s1 = &sA1[b][0][0];
#pragma unroll
        for (int u = 0; u < N1; ++u)
            if (u < N1 - 1 || tid + u * NT < (L - 1) * TX) s1[ly1(u) * TX + tx] = f1[u];
        if (l2 >= 0) (&sA2[b][0][0])[l2] = o2 >= 0 ? f2 : 0.f;
        sA2[b][ty][tx + HL] = q2[HL];
        sA1[b][ty + HL][tx] = q1[HL];
        const float u1 = S.un1, u2 = S.un2, u3 = S.un3;
        const float mx0 = S.mxn0, mx1 = S.mxn1, my0 = S.myn0, my1 = S.myn1, mz0 = S.mzn0, mz1 = S.mzn1;
        float ce1 = S.cn1, ce2 = S.cn2, ce3 = S.cn3;
        const unsigned ci = S.cin;
        __syncthreads();
        if (k + PF < k1) issue(S, k + PF);
        if (CI) {
            ce1 = sCe[ci & 255u];
            ce2 = sCe[(ci >> 8) & 255u];
            ce3 = sCe[(ci >> 16) & 255u];
        }

        if (valid) {
            const cfloat *cz = uniform_table(tz_ + k * L);
            float d2a3 = 0.f, d2a1 = 0.f, d1a3 = 0.f, d1a2 = 0.f, d3a2 = 0.f, d3a1 = 0.f;
#pragma unroll
            for (int m = 0; m < L; ++m) {
                d2a3 += cy[m] * sA3[b][ty + m][tx + HL];
                d2a1 += cy[m] * sA1[b][ty + m][tx];
                d1a3 += cx[m] * sA3[b][ty + HL][tx + m];
                d1a2 += cx[m] * sA2[b][ty][tx + m];
                d3a2 += cz[m] * q2[m];
                d3a1 += cz[m] * q1[m];
            }
            if (xs) {
                const unsigned id = (unsigned)((k * p.n2 + j) * nb2 + ix);
                float v = cpml_mem(bx, mx0, ax, d1a3);
                px0[id] = v;
                d1a3 += v;
                v = cpml_mem(bx, mx1, ax, d1a2);
                px1[id] = v;
                d1a2 += v;
            }
            if (ys) {
                const unsigned id = (unsigned)((k * nb2 + jy) * p.pitch + i);
                float v = cpml_mem(by, my0, ay, d2a3);
                py0[id] = v;
                d2a3 += v;
                v = cpml_mem(by, my1, ay, d2a1);
                py1[id] = v;
                d2a1 += v;
            }
            if (k < nb || k > p.n3 - 1 - nb) {
                const int kz = k < nb ? k : k - (p.n3 - nb2);
                const float az = uniform_table(az_)[k], bz = uniform_table(bz_)[k];
                const unsigned id = (unsigned)((kz * p.n2 + j) * p.pitch + i);
                float v = cpml_mem(bz, mz0, az, d3a2);
                pz0[id] = v;
                d3a2 += v;
                v = cpml_mem(bz, mz1, az, d3a1);
                pz1[id] = v;
                d3a1 += v;
            }
            float c1 = d2a3 - d3a2, c2 = d3a1 - d1a3, c3 = d1a2 - d2a1;
            const unsigned g = (unsigned)(k * plane + own);
            if (HS) {
                st1<ST>(&O1[g], u1 - p.ch * c1);
                st1<ST>(&O2[g], u2 - p.ch * c2);
                st1<ST>(&O3[g], u3 - p.ch * c3);
            } else {
                if (k >= sbz && k < sbz + L && j >= sby && j < sby + L && i >= sbx && i < sbx + L) {
                    const float jv = sn * sq[((k - sbz) * L + (j - sby)) * L + (i - sbx)];
                    if (scomp == 0) c1 -= jv;
                    else if (scomp == 1) c2 -= jv;
                    else c3 -= jv;
                }
                st1<ST>(&O1[g], u1 + ce1 * c1);
                st1<ST>(&O2[g], u2 + ce2 * c2);
                st1<ST>(&O3[g], u3 + ce3 * c3);
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

// Register-blocked variant of step_kernel: a 64-wide tile of 4 RY rows,
// wavefront w owning rows w RY .. w RY + RY - 1, so every row index is
// wave-uniform (y coefficients and y-slab CPML values in scalar registers)
// and each thread updates RY cells per plane.  Per cell it stages
// (4 RY + 2r - 1)(64 + 2r - 1) / (256 RY) plane values of the x/y-tap
// component instead of (4 + 2r - 1)(64 + 2r - 1) / 256 (1.6 against 3.0 at
// r = 4, RY = 4), keeps RY z queues of the two z-differentiated components,
// and has RY times as many loads in flight per thread.  Each derivative is
// the same sum in the same order as in step_kernel, so both kernels give the
// same bits.
template <int R, bool HS, bool ST, bool CI, int RY>
__global__ __launch_bounds__(NT) void step_kernel_rb(const StepParams p, int n_arg) {
    const int n = (p.step_base ? *p.step_base : 0) + n_arg;
    constexpr int L = 2 * R;
    constexpr int TX = 64;
    constexpr int TYS = (NT / TX) * RY;       // rows per tile
    constexpr int HL = HS ? R - 1 : R;        // halo below the own index
    constexpr int W = TX + L - 1;             // LDS row length incl. halo
    constexpr int HR = TYS + L - 1;           // LDS rows incl. halo
    constexpr int N3 = (HR * W + NT - 1) / NT;              // A3 staging loads per thread
    constexpr int N1 = ((L - 1) * TX + NT - 1) / NT;        // A1 halo loads per thread
    constexpr int NC = RY + L - 1;            // y-tap column values a thread's rows read
    static_assert(TYS * (L - 1) <= NT, "one A2 halo value per thread at most");
    __shared__ float sA3[2][HR][W];           // x and y taps
    __shared__ float sA2[2][TYS][W];          // x taps
    __shared__ float sA1[2][HR][TX];          // y taps
    __shared__ float sCe[CI ? kCeTable : 1];

    const float *A1 = HS ? p.E1 : p.H1;
    const float *A2 = HS ? p.E2 : p.H2;
    const float *A3 = HS ? p.E3 : p.H3;

    const int blk = blockIdx.x;
    if (blk < p.nrecblk) {
        rec_dft<R>(p, blk, A1, A2, A3, n);
        return;
    }
    int t = xcd_tile(blk - p.nrecblk, p.nstencil);
    const int s = tile_source(t, p.nsrc, p.nstencil, p.sorder);
    const int bxt = t % p.xt;
    t /= p.xt;
    const int byt = t % p.yt;
    const int bzt = t / p.yt;

    const int tid = threadIdx.x, tx = tid & (TX - 1);
    const int w0 = __builtin_amdgcn_readfirstlane((tid / TX) * RY);   // first tile row of this wave
    const int i0 = bxt * TX, j0 = R + byt * TYS;
    const int i = i0 + tx;
    const int k0 = p.kmin + bzt * p.kz;
    const int k1 = min(k0 + p.kz, p.n3 - R);
    const bool ivalid = i >= R && i <= p.n1 - 1 - R;
    const long long fo = (long long)s * p.fstride;
    A1 += fo;
    A2 += fo;
    A3 += fo;
    const int plane = (int)p.plane;
    const float *U1 = (HS ? p.H1 : p.E1) + fo;
    const float *U2 = (HS ? p.H2 : p.E2) + fo;
    const float *U3 = (HS ? p.H3 : p.E3) + fo;
    float *O1 = (HS ? p.H1 : p.Eo1) + fo;
    float *O2 = (HS ? p.H2 : p.Eo2) + fo;
    float *O3 = (HS ? p.H3 : p.Eo3) + fo;

    const float *tx_ = HS ? p.cpx : p.cmx;
    const float *ty_ = HS ? p.cpy : p.cmy;
    const float *tz_ = HS ? p.cpz : p.cmz;
    const int nb = p.nb, nb2 = 2 * p.nb;
    const int ic = ivalid ? i : R;
    float cx[L];
#pragma unroll
    for (int m = 0; m < L; ++m) cx[m] = tx_[ic * L + m];
    const bool xs = ivalid && (i < nb || i > p.n1 - 1 - nb);
    float ax = 0.f, bx = 0.f;
    int ix = 0;
    if (xs) {
        ax = (HS ? p.axh : p.axi)[i];
        bx = (HS ? p.bxh : p.bxi)[i];
        ix = i < nb ? i : i - (p.n1 - nb2);
    }
    // rows of this wavefront (wave-uniform)
    float cy[RY][L], ay[RY], by[RY];
    int own[RY], jy[RY];
    bool rv[RY], ys[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) {
        const int j = j0 + w0 + q;
        const int jc = min(j, p.n2 - 1);
        rv[q] = j <= p.n2 - 1 - R;
        own[q] = jc * p.pitch + i;
#pragma unroll
        for (int m = 0; m < L; ++m) cy[q][m] = ty_[jc * L + m];
        ys[q] = rv[q] && (j < nb || j > p.n2 - 1 - nb);
        ay[q] = by[q] = 0.f;
        jy[q] = 0;
        if (ys[q]) {
            ay[q] = (HS ? p.ayh : p.ayi)[j];
            by[q] = (HS ? p.byh : p.byi)[j];
            jy[q] = j < nb ? j : j - (p.n2 - nb2);
        }
    }
    const float *az_ = HS ? p.azh : p.azi;
    const float *bz_ = HS ? p.bzh : p.bzi;
    float *px0 = p.psx0 + s * p.psxs, *px1 = p.psx1 + s * p.psxs;
    float *py0 = p.psy0 + s * p.psys, *py1 = p.psy1 + s * p.psys;
    float *pz0 = p.psz0 + s * p.pszs, *pz1 = p.psz1 + s * p.pszs;
    const float *ce1 = p.ce1, *ce2 = p.ce2, *ce3 = p.ce3;
    if (CI && (int)threadIdx.x < p.ncet) sCe[threadIdx.x] = p.cet[threadIdx.x];

    int scomp = -1, sbx = 0, sby = 0, sbz = 0;
    float sn = 0.f;
    const float *sq = nullptr;
    if (!HS) {
        scomp = p.src_info[4 * s];
        sbx = p.src_info[4 * s + 1];
        sby = p.src_info[4 * s + 2];
        sbz = p.src_info[4 * s + 3];
        sn = p.wavelet[n];
        sq = p.src_q + (long long)s * L * L * L;
    }

    // staging map, as in step_kernel
    int o3[N3];
#pragma unroll
    for (int u = 0; u < N3; ++u) {
        const int e = tid + u * NT;
        const int ly = e / W, lx = e - ly * W;
        const int gj = j0 - HL + ly, gi = i0 - HL + lx;
        o3[u] = (e < HR * W && gj >= 0 && gj < p.n2 && gi >= 0 && gi < p.pitch) ? gj * p.pitch + gi : -1;
    }
    auto ly1 = [&](int u) {
        const int hy = (tid + u * NT) / TX;
        return hy < HL ? hy : TYS + hy;
    };
    int o1[N1];
#pragma unroll
    for (int u = 0; u < N1; ++u) {
        const int e = tid + u * NT;
        const int gj = j0 - HL + ly1(u);
        o1[u] = (e < (L - 1) * TX && gj >= 0 && gj < p.n2) ? gj * p.pitch + i0 + tx : -1;
    }
    int o2 = -1, l2 = -1;
    if (tid < TYS * (L - 1)) {
        const int hy = tid / (L - 1), hx = tid % (L - 1);
        const int lx = hx < HL ? hx : TX + hx;
        const int gi = i0 - HL + lx, gj = min(j0 + hy, p.n2 - 1);
        l2 = hy * W + lx;
        o2 = (gi >= 0 && gi < p.pitch) ? gj * p.pitch + gi : -1;
    }

    float q1[RY][L], q2[RY][L];
#pragma unroll
    for (int q = 0; q < RY; ++q)
#pragma unroll
        for (int m = 0; m < L - 1; ++m) {
            q1[q][m] = A1[(unsigned)((k0 - HL + m) * plane + own[q])];
            q2[q][m] = A2[(unsigned)((k0 - HL + m) * plane + own[q])];
        }

    float f3[N3], f1[N1], f2 = 0.f, e1n[RY], e2n[RY];
    float un1[RY], un2[RY], un3[RY], cn1[RY], cn2[RY], cn3[RY];
    unsigned cin[RY];
#pragma unroll
    for (int q = 0; q < RY; ++q) {
        un1[q] = un2[q] = un3[q] = cn1[q] = cn2[q] = cn3[q] = 0.f;
        cin[q] = 0u;
    }
    auto issue = [&](int k) {
        const int pk = k * plane;
#pragma unroll
        for (int u = 0; u < N3; ++u) f3[u] = o3[u] >= 0 ? A3[(unsigned)(pk + o3[u])] : 0.f;
#pragma unroll
        for (int u = 0; u < N1; ++u) f1[u] = o1[u] >= 0 ? A1[(unsigned)(pk + o1[u])] : 0.f;
        if (o2 >= 0) f2 = A2[(unsigned)(pk + o2)];
        const int pe = (k - HL + L - 1) * plane;
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            e1n[q] = A1[(unsigned)(pe + own[q])];
            e2n[q] = A2[(unsigned)(pe + own[q])];
            if (ivalid && rv[q]) {
                const unsigned g = (unsigned)(pk + own[q]);
                un1[q] = ld1<ST>(&U1[g]);
                un2[q] = ld1<ST>(&U2[g]);
                un3[q] = ld1<ST>(&U3[g]);
                if (!HS && CI) {
                    cin[q] = ld1<ST>(&p.cei[g]);
                } else if (!HS) {
                    cn1[q] = ld1<ST>(&ce1[g]);
                    cn2[q] = ld1<ST>(&ce2[g]);
                    cn3[q] = ld1<ST>(&ce3[g]);
                }
            }
        }
    };
    issue(k0);

    for (int k = k0; k < k1; ++k) {
        const int b = (k - k0) & 1;
        float *s3 = &sA3[b][0][0];
#pragma unroll
        for (int u = 0; u < N3; ++u)
            if (u < N3 - 1 || tid + u * NT < HR * W) s3[tid + u * NT] = f3[u];
        float *s1 = &sA1[b][0][0];
#pragma unroll
        for (int u = 0; u < N1; ++u)
            if (u < N1 - 1 || tid + u * NT < (L - 1) * TX) s1[ly1(u) * TX + tx] = f1[u];
        if (l2 >= 0) (&sA2[b][0][0])[l2] = o2 >= 0 ? f2 : 0.f;
        float u1[RY], u2[RY], u3[RY], ce1v[RY], ce2v[RY], ce3v[RY];
        unsigned ci[RY];
#pragma unroll
        for (int q = 0; q < RY; ++q) {
            q1[q][L - 1] = e1n[q];
            q2[q][L - 1] = e2n[q];
            sA2[b][w0 + q][tx + HL] = q2[q][HL];
            sA1[b][w0 + q + HL][tx] = q1[q][HL];
            u1[q] = un1[q];
            u2[q] = un2[q];
            u3[q] = un3[q];
            ce1v[q] = cn1[q];
            ce2v[q] = cn2[q];
            ce3v[q] = cn3[q];
            ci[q] = cin[q];
        }
        __syncthreads();
        if (k + 1 < k1) issue(k + 1);
        if (CI) {
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                ce1v[q] = sCe[ci[q] & 255u];
                ce2v[q] = sCe[(ci[q] >> 8) & 255u];
                ce3v[q] = sCe[(ci[q] >> 16) & 255u];
            }
        }
        if (ivalid) {
            const cfloat *cz = uniform_table(tz_ + k * L);
            // the y-tap columns of this thread's rows, read from LDS once
            float c3[NC], c1[NC];
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                c3[u] = sA3[b][w0 + u][tx + HL];
                c1[u] = sA1[b][w0 + u][tx];
            }
            const bool zs = k < nb || k > p.n3 - 1 - nb;
            const int kz = k < nb ? k : k - (p.n3 - nb2);
            const float az = zs ? uniform_table(az_)[k] : 0.f, bz = zs ? uniform_table(bz_)[k] : 0.f;
#pragma unroll
            for (int q = 0; q < RY; ++q) {
                if (!rv[q]) continue;
                const int j = j0 + w0 + q;
                float d2a3 = 0.f, d2a1 = 0.f, d1a3 = 0.f, d1a2 = 0.f, d3a2 = 0.f, d3a1 = 0.f;
#pragma unroll
                for (int m = 0; m < L; ++m) {
                    d2a3 += cy[q][m] * c3[q + m];
                    d2a1 += cy[q][m] * c1[q + m];
                    d1a3 += cx[m] * sA3[b][w0 + q + HL][tx + m];
                    d1a2 += cx[m] * sA2[b][w0 + q][tx + m];
                    d3a2 += cz[m] * q2[q][m];
                    d3a1 += cz[m] * q1[q][m];
                }
                if (xs) {
                    const unsigned id = (unsigned)((k * p.n2 + j) * nb2 + ix);
                    float v = cpml_mem(bx, px0[id], ax, d1a3);
                    px0[id] = v;
                    d1a3 += v;
                    v = cpml_mem(bx, px1[id], ax, d1a2);
                    px1[id] = v;
                    d1a2 += v;
                }
                if (ys[q]) {
                    const unsigned id = (unsigned)((k * nb2 + jy[q]) * p.pitch + i);
                    float v = cpml_mem(by[q], py0[id], ay[q], d2a3);
                    py0[id] = v;
                    d2a3 += v;
                    v = cpml_mem(by[q], py1[id], ay[q], d2a1);
                    py1[id] = v;
                    d2a1 += v;
                }
                if (zs) {
                    const unsigned id = (unsigned)((kz * p.n2 + j) * p.pitch + i);
                    float v = cpml_mem(bz, pz0[id], az, d3a2);
                    pz0[id] = v;
                    d3a2 += v;
                    v = cpml_mem(bz, pz1[id], az, d3a1);
                    pz1[id] = v;
                    d3a1 += v;
                }
                float r1 = d2a3 - d3a2, r2 = d3a1 - d1a3, r3 = d1a2 - d2a1;
                const unsigned g = (unsigned)(k * plane + own[q]);
                if (HS) {
                    st1<ST>(&O1[g], u1[q] - p.ch * r1);
                    st1<ST>(&O2[g], u2[q] - p.ch * r2);
                    st1<ST>(&O3[g], u3[q] - p.ch * r3);
                } else {
                    if (k >= sbz && k < sbz + L && j >= sby && j < sby + L && i >= sbx && i < sbx + L) {
                        const float jv = sn * sq[((k - sbz) * L + (j - sby)) * L + (i - sbx)];
                        if (scomp == 0) r1 -= jv;
                        else if (scomp == 1) r2 -= jv;
                        else r3 -= jv;
                    }
                    st1<ST>(&O1[g], u1[q] + ce1v[q] * r1);
                    st1<ST>(&O2[g], u2[q] + ce2v[q] * r2);
                    st1<ST>(&O3[g], u3[q] + ce3v[q] * r3);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RY; ++q)
#pragma unroll
            for (int m = 0; m < L - 1; ++m) {
                q1[q][m] = q1[q][m + 1];
                q2[q][m] = q2[q][m + 1];
            }
    }
}

// Fused leap-frog step: one launch per time step reads E^n, H^{n+1/2} and
// dt/eps once and writes E^{n+1}, H^{n+3/2} to the other buffers of a
// ping-pong pair (60 B per cell and step instead of 84 for the two half-step
// kernels).  A block of kLeapRows wavefronts owns an output tile of
// (65 - 2r) x (kLeapRows + 1 - 2r) columns and a z chunk; it computes
// E^{n+1} on the 64 x kLeapRows "E region" (the output tile plus the r - 1
// / r cells of x/y halo the D+ stencil of the H update reaches), plane by
// plane from z = k0 - r + 1 to k1 + r - 1, keeping the last r + 1 planes in
// LDS and the last 2r values of E1, E2 of its own column in registers; the
// H update of plane k - r follows each E plane k.  Every value is the same
// expression as in the half-step kernels; halo cells' E is computed by
// several blocks and written only by the owner.  The E-step CPML memories
// are double-buffered as well (read pe.ps*, write x.q*), because halo cells
// read the neighbour's memories; the H-step memories stay in place.  The
// DTFT waves record H^{n+1/2} (stamp (n+1/2) dt) and E^n (stamp n dt, n > 0;
// E^{nt} is recorded by a last launch with no stencil blocks).
template <int R, bool ST>
__global__ __launch_bounds__(kTileX * kLeapRows) void leap_kernel(const StepParams pe, const StepParams ph,
                                                                 const LeapParams x, int n_arg) {
    const int n = (pe.step_base ? *pe.step_base : 0) + n_arg;
    constexpr int TYE = kLeapRows, NTL = kTileX * TYE;
    constexpr int L = 2 * R;
    constexpr int W = kTileX + L - 1;         // staged H row length (E-step halo R below, R-1 above)
    constexpr int HR = TYE + L - 1;           // staged H rows
    constexpr int TXO = kTileX - (L - 1), TYO = TYE - (L - 1);
    constexpr int N3 = (HR * W + NTL - 1) / NTL;
    constexpr int N1 = ((L - 1) * kTileX + NTL - 1) / NTL;
    __shared__ float sA3[2][HR][W];           // H3: x and y taps of the E update
    __shared__ float sA2[2][TYE][W];          // H2: x taps
    __shared__ float sA1[2][HR][kTileX];      // H1: y taps
    __shared__ float rE1[R + 1][TYE][kTileX]; // E^{n+1} of the last r + 1 planes (H taps)
    __shared__ float rE2[R + 1][TYE][kTileX];
    __shared__ float rE3[R + 1][TYE][kTileX];

    const int blk = blockIdx.x;
    if (blk < x.nrech) {
        rec_dft<R>(pe, blk, pe.H1, pe.H2, pe.H3, n, TYE);
        return;
    }
    if (blk < x.nrech + x.nrece) {
        if (n > 0) rec_dft<R>(ph, blk - x.nrech, pe.E1, pe.E2, pe.E3, n - 1, TYE);
        return;
    }
    int t = xcd_tile(blk - x.nrech - x.nrece, x.nstencil);
    const int s = t % pe.nsrc;
    t /= pe.nsrc;
    const int bxt = t % x.xt;
    t /= x.xt;
    const int byt = t % x.yt;
    const int bzt = t / x.yt;

    const int n1 = pe.n1, n2 = pe.n2, n3 = pe.n3, pitch = pe.pitch, plane = (int)pe.plane;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int i0 = R + bxt * TXO - (R - 1), j0 = R + byt * TYO - (R - 1);   // E region origin
    const int i = i0 + tx, j = j0 + ty;
    const int k0 = R + bzt * x.kz, k1 = min(k0 + x.kz, n3 - R);
    const bool ein = i >= R && i <= n1 - 1 - R && j >= R && j <= n2 - 1 - R;   // E cell in the update set
    const bool own = ein && tx >= R - 1 && tx < R - 1 + TXO && ty >= R - 1 && ty < R - 1 + TYO;
    const int ic = min(max(i, 0), pitch - 1), jc = min(max(j, 0), n2 - 1);
    const int ownc = jc * pitch + ic;          // clamped plane offset of this thread's column
    const long long fo = (long long)s * pe.fstride;
    const float *H1 = pe.H1 + fo, *H2 = pe.H2 + fo, *H3 = pe.H3 + fo;
    const float *E1 = pe.E1 + fo, *E2 = pe.E2 + fo, *E3 = pe.E3 + fo;
    float *Eo1 = x.Eo1 + fo, *Eo2 = x.Eo2 + fo, *Eo3 = x.Eo3 + fo;
    float *Ho1 = x.Ho1 + fo, *Ho2 = x.Ho2 + fo, *Ho3 = x.Ho3 + fo;

    // tables: D- (E update) and D+ (H update) rows of this column / row
    const int it = ein ? i : R, jt = ein ? j : R;
    float cxm[L], cym[L], cxp[L], cyp[L];
#pragma unroll
    for (int m = 0; m < L; ++m) {
        cxm[m] = pe.cmx[it * L + m];
        cym[m] = pe.cmy[jt * L + m];
        cxp[m] = ph.cpx[it * L + m];
        cyp[m] = ph.cpy[jt * L + m];
    }
    const int nb = pe.nb, nb2 = 2 * nb;
    const bool xs = ein && (i < nb || i > n1 - 1 - nb);
    const bool ys = ein && (j < nb || j > n2 - 1 - nb);
    const int ix = i < nb ? i : i - (n1 - nb2), jy = j < nb ? j : j - (n2 - nb2);
    float axi = 0.f, bxi = 0.f, ayi = 0.f, byi = 0.f, axh = 0.f, bxh = 0.f, ayh = 0.f, byh = 0.f;
    if (xs) {
        axi = pe.axi[i];
        bxi = pe.bxi[i];
        axh = ph.axh[i];
        bxh = ph.bxh[i];
    }
    if (ys) {
        ayi = pe.ayi[j];
        byi = pe.byi[j];
        ayh = ph.ayh[j];
        byh = ph.byh[j];
    }
    // E-step memories: read pe.ps*, write x.q* (owner only); H-step memories in place
    const float *ex0 = pe.psx0 + s * pe.psxs, *ex1 = pe.psx1 + s * pe.psxs;
    const float *ey0 = pe.psy0 + s * pe.psys, *ey1 = pe.psy1 + s * pe.psys;
    const float *ez0 = pe.psz0 + s * pe.pszs, *ez1 = pe.psz1 + s * pe.pszs;
    float *qx0 = x.qx0 + s * pe.psxs, *qx1 = x.qx1 + s * pe.psxs;
    float *qy0 = x.qy0 + s * pe.psys, *qy1 = x.qy1 + s * pe.psys;
    float *qz0 = x.qz0 + s * pe.pszs, *qz1 = x.qz1 + s * pe.pszs;
    float *hx0 = ph.psx0 + s * ph.psxs, *hx1 = ph.psx1 + s * ph.psxs;
    float *hy0 = ph.psy0 + s * ph.psys, *hy1 = ph.psy1 + s * ph.psys;
    float *hz0 = ph.psz0 + s * ph.pszs, *hz1 = ph.psz1 + s * ph.pszs;

    const int scomp = pe.src_info[4 * s], sbx = pe.src_info[4 * s + 1], sby = pe.src_info[4 * s + 2],
              sbz = pe.src_info[4 * s + 3];
    const float sn = pe.wavelet[n];
    const float *sq = pe.src_q + (long long)s * L * L * L;

    // staging map of the H planes (as the E step of the half-step kernel)
    int o3[N3];
#pragma unroll
    for (int u = 0; u < N3; ++u) {
        const int e = tid + u * NTL;
        const int ly = e / W, lx = e - ly * W;
        const int gj = j0 - R + ly, gi = i0 - R + lx;
        o3[u] = (e < HR * W && gj >= 0 && gj < n2 && gi >= 0 && gi < pitch) ? gj * pitch + gi : -1;
    }
    auto ly1 = [&](int u) {
        const int hy = (tid + u * NTL) >> 6;
        return hy < R ? hy : TYE + hy;
    };
    int o1[N1];
#pragma unroll
    for (int u = 0; u < N1; ++u) {
        const int e = tid + u * NTL;
        const int gj = j0 - R + ly1(u);
        o1[u] = (e < (L - 1) * kTileX && gj >= 0 && gj < n2 && i >= 0 && i < pitch) ? gj * pitch + i : -1;
    }
    int o2 = -1, l2 = -1;
    if (tid < TYE * (L - 1)) {
        const int hy = tid / (L - 1), hx = tid % (L - 1);
        const int lx = hx < R ? hx : kTileX + hx;
        const int gi = i0 - R + lx, gj = j0 + hy;
        l2 = hy * W + lx;
        o2 = (gi >= 0 && gi < pitch && gj >= 0 && gj < n2) ? gj * pitch + gi : -1;
    }
    const bool colin = i >= 0 && i < pitch && j >= 0 && j < n2;   // own column inside the array

    const int ka = k0 - R + 1, kb = k1 + R - 1;   // E planes computed
    // z queues of H1, H2 (E update, planes k-R .. k+R-1) and of E1, E2 (H update)
    float q1[L], q2[L], g1[L], g2[L];
    auto hz = [&](const float *A, int kk) -> float {
        return (colin && kk >= 0 && kk < n3) ? A[(unsigned)(kk * plane + ownc)] : 0.f;
    };
#pragma unroll
    for (int m = 0; m < L; ++m) {
        g1[m] = 0.f;
        g2[m] = 0.f;
    }
#pragma unroll
    for (int m = 0; m < L - 1; ++m) {
        q1[m] = hz(H1, ka - R + m);
        q2[m] = hz(H2, ka - R + m);
    }
    float f3[N3], f1[N1], f2 = 0.f, e1n = 0.f, e2n = 0.f;
    float un1 = 0.f, un2 = 0.f, un3 = 0.f, cn1 = 0.f, cn2 = 0.f, cn3 = 0.f;
    auto issue = [&](int k) {
        const int pk = k * plane;
#pragma unroll
        for (int u = 0; u < N3; ++u) f3[u] = o3[u] >= 0 ? H3[(unsigned)(pk + o3[u])] : 0.f;
#pragma unroll
        for (int u = 0; u < N1; ++u) f1[u] = o1[u] >= 0 ? H1[(unsigned)(pk + o1[u])] : 0.f;
        if (o2 >= 0) f2 = H2[(unsigned)(pk + o2)];
        e1n = hz(H1, k + R - 1);
        e2n = hz(H2, k + R - 1);
        if (ein && k >= R && k <= n3 - 1 - R) {
            const unsigned g = (unsigned)(pk + ownc);
            un1 = ld1<ST>(&E1[g]);
            un2 = ld1<ST>(&E2[g]);
            un3 = ld1<ST>(&E3[g]);
            cn1 = ld1<ST>(&pe.ce1[g]);
            cn2 = ld1<ST>(&pe.ce2[g]);
            cn3 = ld1<ST>(&pe.ce3[g]);
        }
    };
    issue(ka);
    for (int k = ka; k <= kb; ++k) {
        const int b = (k - ka) & 1;
        q1[L - 1] = e1n;
        q2[L - 1] = e2n;
        float *s3 = &sA3[b][0][0];
#pragma unroll
        for (int u = 0; u < N3; ++u)
            if (u < N3 - 1 || tid + u * NTL < HR * W) s3[tid + u * NTL] = f3[u];
        float *s1 = &sA1[b][0][0];
#pragma unroll
        for (int u = 0; u < N1; ++u)
            if (u < N1 - 1 || tid + u * NTL < (L - 1) * kTileX) s1[ly1(u) * kTileX + tx] = f1[u];
        if (l2 >= 0) (&sA2[b][0][0])[l2] = o2 >= 0 ? f2 : 0.f;
        sA2[b][ty][tx + R] = q2[R];
        sA1[b][ty + R][tx] = q1[R];
        const float u1 = un1, u2 = un2, u3 = un3, ce1 = cn1, ce2 = cn2, ce3 = cn3;
        __syncthreads();
        if (k + 1 <= kb) issue(k + 1);

        // ---- E^{n+1} at plane k of the E region
        float e1 = 0.f, e2 = 0.f, e3 = 0.f;
        if (ein && k >= R && k <= n3 - 1 - R) {
            const float *cz = pe.cmz + k * L;
            float d2a3 = 0.f, d2a1 = 0.f, d1a3 = 0.f, d1a2 = 0.f, d3a2 = 0.f, d3a1 = 0.f;
#pragma unroll
            for (int m = 0; m < L; ++m) {
                d2a3 += cym[m] * sA3[b][ty + m][tx + R];
                d2a1 += cym[m] * sA1[b][ty + m][tx];
                d1a3 += cxm[m] * sA3[b][ty + R][tx + m];
                d1a2 += cxm[m] * sA2[b][ty][tx + m];
                d3a2 += cz[m] * q2[m];
                d3a1 += cz[m] * q1[m];
            }
            const bool wr = own && k >= k0 && k < k1;
            if (xs) {
                const unsigned id = (unsigned)((k * n2 + j) * nb2 + ix);
                float v = cpml_mem(bxi, ex0[id], axi, d1a3);
                if (wr) qx0[id] = v;
                d1a3 += v;
                v = cpml_mem(bxi, ex1[id], axi, d1a2);
                if (wr) qx1[id] = v;
                d1a2 += v;
            }
            if (ys) {
                const unsigned id = (unsigned)((k * nb2 + jy) * pitch + i);
                float v = cpml_mem(byi, ey0[id], ayi, d2a3);
                if (wr) qy0[id] = v;
                d2a3 += v;
                v = cpml_mem(byi, ey1[id], ayi, d2a1);
                if (wr) qy1[id] = v;
                d2a1 += v;
            }
            if (k < nb || k > n3 - 1 - nb) {
                const int kz = k < nb ? k : k - (n3 - nb2);
                const float az = pe.azi[k], bz = pe.bzi[k];
                const unsigned id = (unsigned)((kz * n2 + j) * pitch + i);
                float v = cpml_mem(bz, ez0[id], az, d3a2);
                if (wr) qz0[id] = v;
                d3a2 += v;
                v = cpml_mem(bz, ez1[id], az, d3a1);
                if (wr) qz1[id] = v;
                d3a1 += v;
            }
            float c1 = d2a3 - d3a2, c2 = d3a1 - d1a3, c3 = d1a2 - d2a1;
            if (k >= sbz && k < sbz + L && j >= sby && j < sby + L && i >= sbx && i < sbx + L) {
                const float jv = sn * sq[((k - sbz) * L + (j - sby)) * L + (i - sbx)];
                if (scomp == 0) c1 -= jv;
                else if (scomp == 1) c2 -= jv;
                else c3 -= jv;
            }
            e1 = u1 + ce1 * c1;
            e2 = u2 + ce2 * c2;
            e3 = u3 + ce3 * c3;
            if (wr) {
                const unsigned g = (unsigned)(k * plane + ownc);
                st1<ST>(&Eo1[g], e1);
                st1<ST>(&Eo2[g], e2);
                st1<ST>(&Eo3[g], e3);
            }
        }
        const int rs = (k - ka) % (R + 1);
        rE1[rs][ty][tx] = e1;
        rE2[rs][ty][tx] = e2;
        rE3[rs][ty][tx] = e3;
#pragma unroll
        for (int m = 0; m < L - 1; ++m) {
            g1[m] = g1[m + 1];
            g2[m] = g2[m + 1];
        }
        g1[L - 1] = e1;
        g2[L - 1] = e2;
        __syncthreads();

        // ---- H^{n+3/2} at plane kh = k - R (E planes kh-R+1 .. kh+R are in g1/g2)
        const int kh = k - R;
        if (own && kh >= k0 && kh < k1) {
            const int hs = (kh - ka) % (R + 1);
            const float *cz = ph.cpz + kh * L;
            float d2a3 = 0.f, d2a1 = 0.f, d1a3 = 0.f, d1a2 = 0.f, d3a2 = 0.f, d3a1 = 0.f;
#pragma unroll
            for (int m = 0; m < L; ++m) {
                d2a3 += cyp[m] * rE3[hs][ty - R + 1 + m][tx];
                d2a1 += cyp[m] * rE1[hs][ty - R + 1 + m][tx];
                d1a3 += cxp[m] * rE3[hs][ty][tx - R + 1 + m];
                d1a2 += cxp[m] * rE2[hs][ty][tx - R + 1 + m];
                d3a2 += cz[m] * g2[m];
                d3a1 += cz[m] * g1[m];
            }
            if (xs) {
                const unsigned id = (unsigned)((kh * n2 + j) * nb2 + ix);
                float v = cpml_mem(bxh, hx0[id], axh, d1a3);
                hx0[id] = v;
                d1a3 += v;
                v = cpml_mem(bxh, hx1[id], axh, d1a2);
                hx1[id] = v;
                d1a2 += v;
            }
            if (ys) {
                const unsigned id = (unsigned)((kh * nb2 + jy) * pitch + i);
                float v = cpml_mem(byh, hy0[id], ayh, d2a3);
                hy0[id] = v;
                d2a3 += v;
                v = cpml_mem(byh, hy1[id], ayh, d2a1);
                hy1[id] = v;
                d2a1 += v;
            }
            if (kh < nb || kh > n3 - 1 - nb) {
                const int kz = kh < nb ? kh : kh - (n3 - nb2);
                const float az = ph.azh[kh], bz = ph.bzh[kh];
                const unsigned id = (unsigned)((kz * n2 + j) * pitch + i);
                float v = cpml_mem(bz, hz0[id], az, d3a2);
                hz0[id] = v;
                d3a2 += v;
                v = cpml_mem(bz, hz1[id], az, d3a1);
                hz1[id] = v;
                d3a1 += v;
            }
            const float c1 = d2a3 - d3a2, c2 = d3a1 - d1a3, c3 = d1a2 - d2a1;
            const unsigned g = (unsigned)(kh * plane + ownc);
            st1<ST>(&Ho1[g], ld1<ST>(&H1[g]) - ph.ch * c1);
            st1<ST>(&Ho2[g], ld1<ST>(&H2[g]) - ph.ch * c2);
            st1<ST>(&Ho3[g], ld1<ST>(&H3[g]) - ph.ch * c3);
        }
#pragma unroll
        for (int m = 0; m < L - 1; ++m) {
            q1[m] = q1[m + 1];
            q2[m] = q2[m + 1];
        }
    }
}

int leap_threads() { return kTileX * kLeapRows; }

template <int R, bool ST>
static void leap_r(const StepParams &pe, const StepParams &ph, const LeapParams &x, int n, hipStream_t s,
                   hipEvent_t t0, hipEvent_t t1) {
    const dim3 grid(x.nrech + x.nrece + x.nstencil), block(kTileX * kLeapRows);
    if (t0 || t1) hipExtLaunchKernelGGL((leap_kernel<R, ST>), grid, block, 0, s, t0, t1, 0, pe, ph, x, n);
    else hipLaunchKernelGGL((leap_kernel<R, ST>), grid, block, 0, s, pe, ph, x, n);
}

void launch_leap(int r, const StepParams &pe, const StepParams &ph, const LeapParams &x, int n,
                 hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    switch (r * 2 + (pe.stream ? 1 : 0)) {
    case 2: leap_r<1, false>(pe, ph, x, n, s, t0, t1); break;
    case 3: leap_r<1, true>(pe, ph, x, n, s, t0, t1); break;
    case 4: leap_r<2, false>(pe, ph, x, n, s, t0, t1); break;
    case 5: leap_r<2, true>(pe, ph, x, n, s, t0, t1); break;
    case 6: leap_r<3, false>(pe, ph, x, n, s, t0, t1); break;
    case 7: leap_r<3, true>(pe, ph, x, n, s, t0, t1); break;
    case 8: leap_r<4, false>(pe, ph, x, n, s, t0, t1); break;
    default: leap_r<4, true>(pe, ph, x, n, s, t0, t1); break;
    }
}

template <int R, bool HS, bool ST, bool CI>
static void launch_r(const StepParams &p, int n, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    const dim3 grid(p.nrecblk + p.nstencil), block(NT);
    if (p.ry == 2 || p.ry == 4) {
        if (p.ry == 2) {
            if (t0 || t1) hipExtLaunchKernelGGL((step_kernel_rb<R, HS, ST, CI, 2>), grid, block, 0, s, t0, t1, 0, p, n);
            else hipLaunchKernelGGL((step_kernel_rb<R, HS, ST, CI, 2>), grid, block, 0, s, p, n);
        } else {
            if (t0 || t1) hipExtLaunchKernelGGL((step_kernel_rb<R, HS, ST, CI, 4>), grid, block, 0, s, t0, t1, 0, p, n);
            else hipLaunchKernelGGL((step_kernel_rb<R, HS, ST, CI, 4>), grid, block, 0, s, p, n);
        }
    } else if (p.tx == 32) {
        if (t0 || t1) hipExtLaunchKernelGGL((step_kernel<R, HS, ST, CI, 32>), grid, block, 0, s, t0, t1, 0, p, n);
        else hipLaunchKernelGGL((step_kernel<R, HS, ST, CI, 32>), grid, block, 0, s, p, n);
    } else {
        if (t0 || t1) hipExtLaunchKernelGGL((step_kernel<R, HS, ST, CI, 64>), grid, block, 0, s, t0, t1, 0, p, n);
        else hipLaunchKernelGGL((step_kernel<R, HS, ST, CI, 64>), grid, block, 0, s, p, n);
    }
}

template <bool HS, bool ST, bool CI>
static void launch(int r, const StepParams &p, int n, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    switch (r) {
    case 1: launch_r<1, HS, ST, CI>(p, n, s, t0, t1); break;
    case 2: launch_r<2, HS, ST, CI>(p, n, s, t0, t1); break;
    case 3: launch_r<3, HS, ST, CI>(p, n, s, t0, t1); break;
    default: launch_r<4, HS, ST, CI>(p, n, s, t0, t1); break;
    }
}

void launch_e_step(int r, const StepParams &p, int n, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (p.cei) {
        if (p.stream) launch<false, true, true>(r, p, n, s, t0, t1);
        else launch<false, false, true>(r, p, n, s, t0, t1);
    } else {
        if (p.stream) launch<false, true, false>(r, p, n, s, t0, t1);
        else launch<false, false, false>(r, p, n, s, t0, t1);
    }
}

// zero n 4-byte words: 16-byte stores for the aligned bulk, then the tail
__global__ __launch_bounds__(256) void zero_kernel(unsigned *p, size_t n) {
    const size_t n4 = n / 4;
    uint4 *q = reinterpret_cast<uint4 *>(p);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        q[i] = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = 4 * n4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    if (n == 0) return;
    const size_t want = (n / 4 + 255) / 256;
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>(want, 4096));
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, (unsigned *)p, n);
}

// graph replays: advance the device step counter by k after each replay
__global__ void advance_kernel(int *step, int k) {
    if (blockIdx.x == 0 && threadIdx.x == 0) step[0] += k;
}

void launch_advance(int *step, int k, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step, k);
}
void launch_h_step(int r, const StepParams &p, int n, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    if (p.stream) launch<true, true, false>(r, p, n, s, t0, t1);
    else launch<true, false, false>(r, p, n, s, t0, t1);
}

}  // namespace emm
