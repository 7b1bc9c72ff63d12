// Internal types shared by the host runtime and the HIP kernels of libemm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace emm {

constexpr int kTileX = 64;     // one wavefront row along x (wave64)
constexpr int kMaxR = 4;       // 8th order in space at most
constexpr int kTileY = 4;      // rows (wavefronts) per thread block
// The forward step kernels run 256-thread tiles of 64 x 4 or 32 x 8
// columns (StepParams::tx): 32-wide tiles leave fewer idle lanes in the
// last tile of a row and stage less y halo per cell; 64-wide ones keep the
// row index wave-uniform.
constexpr int kStepThreads = kTileX * kTileY;
constexpr int kCeTable = 256;  // distinct dt/eps values of a model in the compact form

// Everything one half-step kernel needs; passed by value.
struct StepParams {
    // padded grid and device layout: [n3][n2][pitch], x fastest
    int n1, n2, n3, pitch;
    long long plane;            // pitch * n2
    long long fstride;          // one source's field array: plane * n3
    int nb;
    // launch decomposition
    int tx;                     // tile width: 64 (x 4 rows) or 32 (x 8 rows)
    int ry;                     // rows per wavefront: 1, or 2 / 4 (register-blocked 64-wide
                                // tiles of 8 / 16 rows, step_kernel_rb)
    int xt, yt, zc, kz;         // x tiles, y tiles, z chunks, planes per chunk
    int kmin;                   // first updated z plane (r, or the surface node under air)
    int nsrc;
    int nstencil;               // xt * yt * zc * nsrc
    int sorder;                 // tile order: 0 = source fastest (the blocks of all sources for
                                // one spatial tile together), 1 = source slowest (each source's
                                // tiles contiguous: neighbouring tiles share halos in L2)
    int nrecblk;                // receiver blocks placed first (multiple of 8)
    int stream;                 // 1: nontemporal loads/stores of the arrays touched once per launch
    // fields (source 0; source s at + s * fstride)
    float *E1, *E2, *E3, *H1, *H2, *H3;
    float *Eo1, *Eo2, *Eo3;          // where the E step writes E (== E1..3: in place)
    const float *ce1, *ce2, *ce3;   // dt/eps at Ex/Ey/Ez positions
    // Optional compact dt/eps for the E step (nullptr: read ce1..3): per cell
    // one word whose bytes 0, 1, 2 index the Ex, Ey, Ez values in cet, the
    // table of the ncet (<= kCeTable) distinct dt/eps values of the model
    // (exact: the same FP32 values)
    const unsigned *cei;
    const float *cet;
    int ncet;
    float ch;                        // dt/mu0
    // FD tables [n_d][2R]: cm = D- at integer nodes, cp = D+ at half nodes
    const float *cmx, *cmy, *cmz, *cpx, *cpy, *cpz;
    // CPML coefficients per axis: integer nodes (E step) and half nodes (H step)
    const float *axi, *bxi, *ayi, *byi, *azi, *bzi;
    const float *axh, *bxh, *ayh, *byh, *azh, *bzh;
    // CPML memory variables of this half step, two per axis, per source:
    //   x: [n3][n2][2nb], y: [n3][2nb][pitch], z: [2nb][n2][pitch]
    float *psx0, *psx1, *psy0, *psy1, *psz0, *psz1;
    long long psxs, psys, pszs;      // per-source strides
    // sources (E step only): per source {comp, bx, by, bz}, (2R)^3 q values
    const int *src_info;
    const float *src_q;
    const float *wavelet;            // s_n
    // receiver DFT items handled by this kernel
    int nitems;
    const int *item_info;            // per item {src, field 0..2, bx, by, bz, slot}
    const float *item_w;             // per item wx[2R], wy[2R], wz[2R]
    const double2 *phase;            // [nt][nf] exp(i w' t) of this kernel's stamp
    int nf;
    double2 *acc;                    // [slots][nf]           (dft_mode 0)
    float4 *acck;                    // [slots][nf] re,cre,im,cim (dft_mode 1)
    int dft_mode;
    // step index = *step_base + n when step_base is set (graph replays), else n
    const int *step_base;
};

// The fused leap-frog step (one launch per time step): E^{n+1} into new
// arrays, then H^{n+3/2} into new arrays, with E recomputed on the x/y halo
// that the H stencil needs.  pe / ph carry the E- and H-step parameters
// (inputs E^n, H^{n+1/2}; tables; CPML; source; DTFT items of the H and E
// channels); this struct carries the outputs and the fused tiling.
constexpr int kLeapRows = 8;   // wavefront rows per block (E region)

struct LeapParams {
    float *Eo1, *Eo2, *Eo3, *Ho1, *Ho2, *Ho3;   // E^{n+1}, H^{n+3/2} (source 0)
    float *qx0, *qx1, *qy0, *qy1, *qz0, *qz1;   // E-step CPML memories written (pe.ps* are read)
    int xt, yt, zc, kz, nstencil;               // tiles of (65 - 2r) x (kLeapRows + 1 - 2r) outputs
    int nrech, nrece;                           // DTFT blocks: H channels of H^{n+1/2}, E channels of E^n
};

void launch_leap(int r, const StepParams &pe, const StepParams &ph, const LeapParams &x, int n,
                 hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
int leap_threads();

// Wave-uniform read-only tables (the z rows of the FD tables, the z-CPML
// coefficients) are read in the constant address space inside the plane
// loops: scalar loads, counted apart from the vector loads of the next
// plane's prefetch, so using them does not wait for that prefetch to land.
typedef __attribute__((address_space(4))) const float cfloat;
__device__ __forceinline__ const cfloat *uniform_table(const float *p) { return (const cfloat *)p; }

// Source and spatial tile of logical tile t (0 <= t < nstencil, nstencil =
// tiles * nsrc) in the order `sorder` (see StepParams::sorder); t becomes
// the spatial tile.
__device__ __forceinline__ int tile_source(int &t, int nsrc, int nstencil, int sorder) {
    if (sorder) {
        const int per = nstencil / nsrc;
        const int s = t / per;
        t -= s * per;
        return s;
    }
    const int s = t % nsrc;
    t /= nsrc;
    return s;
}

// Hardware dispatches workgroup w to XCD w % 8; give every XCD one
// contiguous range of logical tiles.
__device__ __forceinline__ int xcd_tile(int w, int total) {
    const int q = total >> 3, rem = total & 7;
    const int x = w & 7, local = w >> 3;
    return x * q + min(x, rem) + local;
}

// t0/t1 (optional): events stamped with the kernel's own start and end
// (hipExtLaunchKernel), i.e. the duration a kernel trace reports
void launch_e_step(int r, const StepParams &p, int n, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
void launch_advance(int *step, int k, hipStream_t s);
void launch_h_step(int r, const StepParams &p, int n, hipStream_t s, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
int block_threads();
// zero `bytes` (a multiple of 4) at p, 4-byte aligned, with a fill kernel
void launch_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace emm
