// Air above the sea surface (Section 3.3).  No cell above the surface node
// ks is updated; after each half step the ghost planes that the stencils
// of the cells near the surface reach are filled from the surface plane:
//   E1, E2 at the r - 1 integer nodes above ks: each horizontal Fourier mode
//     of the surface value decays as exp(-|k| h) (Laplace's equation in the
//     air, z positive down);
//   H1, H2 at the r half nodes above ks, from H3 at ks: H is a potential
//     field in the source-free, non-conducting air, so Hx^ = i kx/|k| Hz^,
//     Hy^ = i ky/|k| Hz^, times exp(-|k| h), with the half-cell shift of H1
//     (x) and H2 (y) relative to H3 as a phase (the k = 0 mode is 0).
// Transforms: batched 2-D real-to-complex and complex-to-real FFTs (hipFFT)
// over the whole padded x-y plane, which must have uniform spacing.  With
// one ghost plane per component, the inverse transform writes it for all
// sources and both components directly (their arrays are one field stride
// apart); with more, one inverse execution covers every ghost plane of the
// fill into a scratch buffer and one kernel scatters them.
#include "emm_air.h"

#include <cmath>

namespace emm {

namespace {

constexpr int AT = 256;

// W[m][b][bin] = S[b][bin] * dec[m][bin]
__global__ __launch_bounds__(AT) void air_mul_e(const float2 *S, float2 *W, const float *dec, int nbin,
                                                 int nbatch, int nm) {
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const long long per_m = (long long)nbatch * nbin;
    if (t >= per_m * nm) return;
    const int m = (int)(t / per_m);
    const long long u = t - m * per_m;
    const int bin = (int)(u % nbin);
    const float d = dec[(long long)m * nbin + bin];
    const float2 v = S[u];
    W[t] = make_float2(v.x * d, v.y * d);
}

// W[m][c][s][bin] = S[s][bin] * (c == 0 ? rx : ry)[m][bin]
__global__ __launch_bounds__(AT) void air_mul_h(const float2 *S, float2 *W, const float2 *rx,
                                                 const float2 *ry, int nbin, int nsrc, int nm) {
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const long long per_c = (long long)nsrc * nbin, per_m = 2 * per_c;
    if (t >= per_m * nm) return;
    const int m = (int)(t / per_m);
    const long long u = t - m * per_m;
    const int c = (int)(u / per_c);
    const long long sb = u - c * per_c;
    const int bin = (int)(sb % nbin);
    const float2 f = (c == 0 ? rx : ry)[(long long)m * nbin + bin];
    const float2 v = S[sb];
    W[t] = make_float2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
}

// ghost plane o of the scratch (o = (m - 1) * 2 nsrc + a, a = component *
// nsrc + source) into plane ks - m of field array a; n1 of the pitch columns
__global__ __launch_bounds__(AT) void air_scatter(const float *G, float *F, long long fstride, long long plane,
                                                   int ks, int two_ns, int n1, int n2, int pitch, int nplanes) {
    const long long t = (long long)blockIdx.x * AT + threadIdx.x;
    const long long per = (long long)n2 * n1;
    if (t >= per * nplanes) return;
    const int o = (int)(t / per);
    const long long u = t - (long long)o * per;
    const int y = (int)(u / n1), x = (int)(u - (long long)y * n1);
    const int a = o % two_ns, m = o / two_ns + 1;
    F[a * fstride + (ks - m) * plane + (long long)y * pitch + x] = G[((long long)o * n2 + y) * pitch + x];
}

unsigned blocks(long long n) { return (unsigned)((n + AT - 1) / AT); }

const char *fft_name(hipfftResult r) {
    switch (r) {
    case HIPFFT_SUCCESS: return "success";
    case HIPFFT_INVALID_PLAN: return "invalid plan";
    case HIPFFT_ALLOC_FAILED: return "allocation failed";
    case HIPFFT_INVALID_VALUE: return "invalid value";
    case HIPFFT_EXEC_FAILED: return "execution failed";
    case HIPFFT_SETUP_FAILED: return "setup failed";
    case HIPFFT_INVALID_SIZE: return "invalid size";
    default: return "hipFFT error";
    }
}

}  // namespace

AirBoundary::~AirBoundary() {
    if (have_fwdE_) (void)hipfftDestroy(fwdE_);
    if (have_fwdH_) (void)hipfftDestroy(fwdH_);
    if (have_invE_) (void)hipfftDestroy(invE_);
    if (have_invH_) (void)hipfftDestroy(invH_);
    if (have_invEall_) (void)hipfftDestroy(invEall_);
    if (have_invHall_) (void)hipfftDestroy(invHall_);
    for (void *p : {(void *)spec_, (void *)work_, (void *)decE_, (void *)rx_, (void *)ry_, (void *)ghost_})
        if (p) (void)hipFree(p);
}

bool AirBoundary::init(const AirSpec &spec, std::string &err) {
    s_ = spec;
    const int n1 = s_.n1, n2 = s_.n2, n1h = n1 / 2 + 1, r = s_.r, ns = s_.nsrc;
    nbin_ = n2 * n1h;
    auto plan = [&](hipfftHandle &h, bool &have, hipfftType type, int batch) -> bool {
        int n[2] = {n2, n1};
        int real_emb[2] = {n2, s_.pitch};
        int cplx_emb[2] = {n2, n1h};
        const bool r2c = type == HIPFFT_R2C;
        hipfftResult e = hipfftPlanMany(&h, 2, n, r2c ? real_emb : cplx_emb, 1,
                                        r2c ? (int)s_.fstride : nbin_, r2c ? cplx_emb : real_emb, 1,
                                        r2c ? nbin_ : (int)s_.fstride, type, batch);
        if (e != HIPFFT_SUCCESS) {
            err = std::string("hipfftPlanMany: ") + fft_name(e);
            return false;
        }
        have = true;
        return true;
    };
    if (!plan(fwdE_, have_fwdE_, HIPFFT_R2C, 2 * ns) || !plan(fwdH_, have_fwdH_, HIPFFT_R2C, ns) ||
        !plan(invE_, have_invE_, HIPFFT_C2R, 2 * ns) || !plan(invH_, have_invH_, HIPFFT_C2R, 2 * ns))
        return false;
    // all ghost planes of a fill at once, into the scratch planes
    auto plan_all = [&](hipfftHandle &h, bool &have, int batch) -> bool {
        int n[2] = {n2, n1};
        int real_emb[2] = {n2, s_.pitch};
        int cplx_emb[2] = {n2, n1h};
        hipfftResult e = hipfftPlanMany(&h, 2, n, cplx_emb, 1, nbin_, real_emb, 1, n2 * s_.pitch, HIPFFT_C2R, batch);
        if (e != HIPFFT_SUCCESS) {
            err = std::string("hipfftPlanMany: ") + fft_name(e);
            return false;
        }
        have = true;
        return true;
    };
    if (r - 1 > 1 && !plan_all(invEall_, have_invEall_, (r - 1) * 2 * ns)) return false;
    if (r > 1 && !plan_all(invHall_, have_invHall_, r * 2 * ns)) return false;
    // spectral factors in FP64, stored in FP32 with the 1/(n1 n2) of the inverse
    const double norm = 1.0 / ((double)n1 * n2);
    const double pi = 3.14159265358979323846;
    std::vector<float> dec((size_t)std::max(1, r - 1) * nbin_, 0.f);
    std::vector<float2> fx((size_t)r * nbin_), fy((size_t)r * nbin_);
    for (int b = 0; b < n2; ++b) {
        const int qy = b <= (n2 - 1) / 2 ? b : b - n2;
        const double ky = 2.0 * pi * qy / (n2 * s_.dy);
        for (int a = 0; a < n1h; ++a) {
            const double kx = 2.0 * pi * a / (n1 * s_.dx);
            const double kap = std::sqrt(kx * kx + ky * ky);
            const size_t bin = (size_t)b * n1h + a;
            for (int m = 1; m < r; ++m) dec[(size_t)(m - 1) * nbin_ + bin] = (float)(std::exp(-kap * s_.hE[m - 1]) * norm);
            for (int m = 1; m <= r; ++m) {
                const double d = std::exp(-kap * s_.hH[m - 1]) * norm;
                double xr = 0.0, xi = 0.0, yr = 0.0, yi = 0.0;
                if (kap > 0.0) {
                    // (i kx/|k|) exp(-i kx dx/2) and (i ky/|k|) exp(-i ky dy/2)
                    const double cx = std::cos(0.5 * kx * s_.dx), sx = std::sin(0.5 * kx * s_.dx);
                    const double cy = std::cos(0.5 * ky * s_.dy), sy = std::sin(0.5 * ky * s_.dy);
                    xr = kx / kap * sx;
                    xi = kx / kap * cx;
                    yr = ky / kap * sy;
                    yi = ky / kap * cy;
                }
                fx[(size_t)(m - 1) * nbin_ + bin] = make_float2((float)(xr * d), (float)(xi * d));
                fy[(size_t)(m - 1) * nbin_ + bin] = make_float2((float)(yr * d), (float)(yi * d));
            }
        }
    }
    const size_t spec_n = (size_t)2 * ns * nbin_;
    const size_t work_n = (size_t)std::max(1, r) * 2 * ns * nbin_;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&spec_, spec_n * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&work_, work_n * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&decE_, dec.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&rx_, fx.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&ry_, fy.size() * sizeof(float2));
    if (e == hipSuccess && r > 1)
        e = hipMalloc(&ghost_, (size_t)r * 2 * ns * n2 * s_.pitch * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(decE_, dec.data(), dec.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(rx_, fx.data(), fx.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ry_, fy.data(), fy.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        err = std::string("air boundary buffers: ") + hipGetErrorString(e);
        return false;
    }
    return true;
}

bool AirBoundary::fill_E(float *E1, hipStream_t st, std::string &err) {
    const int r = s_.r, ns = s_.nsrc;
    if (r < 2) return true;
    hipfftResult f = hipfftSetStream(fwdE_, st);
    if (f == HIPFFT_SUCCESS) f = hipfftSetStream(invE_, st);
    if (f == HIPFFT_SUCCESS) f = hipfftExecR2C(fwdE_, E1 + (long long)s_.ks * s_.plane, (hipfftComplex *)spec_);
    if (f != HIPFFT_SUCCESS) {
        err = std::string("air boundary E transform: ") + fft_name(f);
        return false;
    }
    const long long total = (long long)(r - 1) * 2 * ns * nbin_;
    hipLaunchKernelGGL(air_mul_e, dim3(blocks(total)), dim3(AT), 0, st, spec_, work_, decE_, nbin_, 2 * ns, r - 1);
    if (have_invEall_) {
        f = hipfftSetStream(invEall_, st);
        if (f == HIPFFT_SUCCESS) f = hipfftExecC2R(invEall_, (hipfftComplex *)work_, ghost_);
        const long long cells = (long long)(r - 1) * 2 * ns * s_.n2 * s_.n1;
        if (f == HIPFFT_SUCCESS)
            hipLaunchKernelGGL(air_scatter, dim3(blocks(cells)), dim3(AT), 0, st, ghost_, E1, s_.fstride, s_.plane,
                               s_.ks, 2 * ns, s_.n1, s_.n2, s_.pitch, (r - 1) * 2 * ns);
    } else {
        for (int m = 1; m < r && f == HIPFFT_SUCCESS; ++m)
            f = hipfftExecC2R(invE_, (hipfftComplex *)(work_ + (size_t)(m - 1) * 2 * ns * nbin_),
                              E1 + (long long)(s_.ks - m) * s_.plane);
    }
    if (f != HIPFFT_SUCCESS) {
        err = std::string("air boundary E inverse: ") + fft_name(f);
        return false;
    }
    return true;
}

bool AirBoundary::fill_H(float *H1, const float *H3, hipStream_t st, std::string &err) {
    const int r = s_.r, ns = s_.nsrc;
    hipfftResult f = hipfftSetStream(fwdH_, st);
    if (f == HIPFFT_SUCCESS) f = hipfftSetStream(invH_, st);
    if (f == HIPFFT_SUCCESS)
        f = hipfftExecR2C(fwdH_, const_cast<float *>(H3) + (long long)s_.ks * s_.plane, (hipfftComplex *)spec_);
    if (f != HIPFFT_SUCCESS) {
        err = std::string("air boundary H transform: ") + fft_name(f);
        return false;
    }
    const long long total = (long long)r * 2 * ns * nbin_;
    hipLaunchKernelGGL(air_mul_h, dim3(blocks(total)), dim3(AT), 0, st, spec_, work_, rx_, ry_, nbin_, ns, r);
    if (have_invHall_) {
        f = hipfftSetStream(invHall_, st);
        if (f == HIPFFT_SUCCESS) f = hipfftExecC2R(invHall_, (hipfftComplex *)work_, ghost_);
        const long long cells = (long long)r * 2 * ns * s_.n2 * s_.n1;
        if (f == HIPFFT_SUCCESS)
            hipLaunchKernelGGL(air_scatter, dim3(blocks(cells)), dim3(AT), 0, st, ghost_, H1, s_.fstride, s_.plane,
                               s_.ks, 2 * ns, s_.n1, s_.n2, s_.pitch, r * 2 * ns);
    } else {
        for (int m = 1; m <= r && f == HIPFFT_SUCCESS; ++m)
            f = hipfftExecC2R(invH_, (hipfftComplex *)(work_ + (size_t)(m - 1) * 2 * ns * nbin_),
                              H1 + (long long)(s_.ks - m) * s_.plane);
    }
    if (f != HIPFFT_SUCCESS) {
        err = std::string("air boundary H inverse: ") + fft_name(f);
        return false;
    }
    return true;
}

}  // namespace emm
