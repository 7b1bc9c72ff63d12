// Parameters of the adjoint kernels of libemm (see emm_adjoint.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "emm_internal.h"

namespace emm {

struct AdjParams {
    int n1, n2, n3, pitch, r, nb, nsrc;
    int kz;                       // z planes per thread block of the gathers
    int tw;                       // tile width of the gathers: 64 (x 4 rows) or 32 (x 8 rows)
    int xt, yt, zc, nstencil;     // tiles along x, y, z chunks; xt * yt * zc * nsrc
    int sorder;                   // tile order of the sources (StepParams::sorder)
    long long fstride;            // one source's field array (plane * n3)
    // inputs (filtered by the CPML reverse) and outputs of the gather,
    // source 0 (source s at + s * fstride)
    const float *in1, *in2, *in3;
    float *out1, *out2, *out3;
    const float *ce1, *ce2, *ce3; // dt/eps
    // optional compact dt/eps for the reverse of the H update (as StepParams)
    const unsigned *cei;
    const float *cet;
    int ncet;
    float scale;                  // Et += ce * scale * curl (REV_H), Hb -= scale * curl (else)
    // transposed FD tables [n_d][2r] of this reverse half step
    const float *tx, *ty, *tz;
    // CPML tables of the forward half step being reversed, axes concatenated [n1 | n2 | n3]
    const float *a_int, *b_int, *a_half, *b_half;
    // memory-variable adjoints and filtered taps: [0,1] x slab (comps 2,3),
    // [2,3] y slab (comps 1,3), [4,5] z slab (comps 1,2), per source
    float *Q[6];
    float *T[6];
    long long sxs, sys, szs;      // per-source strides of the x, y, z slab arrays
    // gradient (reverse of the E update only): E^{n+1}, E^n snapshots laid
    // out like the fields ([comp][src][...]); per-source partial sums
    // grad32[src][comp][...] of Et (E^{n+1} - E^n) over a few steps, flushed
    // into grad[src][comp][...] (double) divided by dt/eps
    const float *E_next, *E_prev;
    float *grad32;
    double *grad;
    long long gstride;            // component stride of one source's grad (fstride)
};

struct InjectParams {
    int ncells, nf;
    const int *row;               // CSR rows [ncells + 1]
    const int *item;              // receiver item of each entry
    const float *w;               // interpolation weight of each entry
    const long long *cell;        // target index in the field array (source offset included)
    const long long *mcell;       // model index (for dt/eps)
    const int *comp;              // target component 0..2
    const double2 *A;             // [items][nf] adjoint-source coefficients
    const double2 *phase;         // [nt][nf]
    float *F1, *F2, *F3;          // target fields
    const float *ce1, *ce2, *ce3; // dt/eps per component: targets are Et (scaled), or
    int scale_ce;                 // 0: targets are Hb (unscaled)
};

void launch_adj_filter(bool rev_h, const AdjParams &p, hipStream_t st);
void launch_adj_inject(const InjectParams &p, int n, hipStream_t st);
void launch_adj_flush(const AdjParams &p, hipStream_t st);
// the gradient per source and padded cell [s][c][cells] summed over sources
// and folded onto the input cells (negated: d/dlog sigma = -d/dlog(dt/eps)),
// into out[c][nd2][nd1][nd0], added to it when accumulate
void launch_adj_fold(const double *grad, double *out, int nsrc, long long fstride, long long plane, int pitch,
                     int n1, int n2, int n3, int r, int nbe, int nd0, int nd1, int nd2, bool accumulate,
                     hipStream_t st);
void launch_adj_tile(int r, bool rev_h, const AdjParams &p, hipStream_t st);

}  // namespace emm
