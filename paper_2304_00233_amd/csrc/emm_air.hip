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
// Transforms over the whole padded x-y plane, which must have uniform
// spacing, in one of two forms:
//  * direct (planes of at most kDftMax points per axis): three kernels per
//    fill in FP64, one block per (row, batch) for the forward transform
//    along x, one per (column kx, batch, output plane) for the forward and
//    inverse transforms along y around the spectral factor, one per (row,
//    output plane) for the inverse transform along x into the ghost plane;
//  * hipFFT (FP32): batched 2-D real-to-complex and complex-to-real FFTs.
//    With one ghost plane per component, the inverse transform writes it for
//    all sources and both components directly (their arrays are one field
//    stride apart); with more, one inverse execution covers every ghost
//    plane of the fill into a scratch buffer and one kernel scatters them.
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

// ---- direct transforms in FP64 (the vector units run FP64 FMAs at the FP32
// rate, so the fills cost the same in either precision, and FP64 keeps the
// ghost values accurate where the surface field spans many orders of
// magnitude across the plane: a transform's rounding is relative to the
// plane's largest value, not to the local one).  One level of Cooley-Tukey
// (n = f m, f the largest divisor of n not above sqrt(n)) evaluated by
// plain sums, (m + f) / n of a direct DFT's work, for planes of at most
// kDftMax points per axis.  tw[e] = exp(2 pi i e / n); sign -1 forward,
// +1 inverse.
//   D[j m + k'] = sum_{l < m} in[l f + j] w^(f l k')   (f transforms of length m)
//   out[k]      = sum_{j < f} w^(j k) D[j m + k mod m]
// Every sum runs in a fixed order in one thread: results do not depend on
// the launch, and replays repeat them bit for bit.

__device__ __forceinline__ double2 twid(const double2 *tw, int e, double sg) {
    const double2 w = tw[e];
    return make_double2(w.x, sg * w.y);
}

__device__ __forceinline__ double2 cmac(double2 acc, double2 v, double2 w) {
    acc.x = fma(v.x, w.x, acc.x);
    acc.x = fma(-v.y, w.y, acc.x);
    acc.y = fma(v.x, w.y, acc.y);
    acc.y = fma(v.y, w.x, acc.y);
    return acc;
}

// stage a over a complex input in LDS
__device__ void dft_stage_a(const double2 *in, double2 *D, int n, int f, int m, const double2 *tw, double sg) {
    for (int idx = threadIdx.x; idx < n; idx += AT) {
        const int j = idx / m, kp = idx - j * m;
        const int step = (f * kp) % n;
        double2 acc = make_double2(0.0, 0.0);
        int e = 0;
        for (int l = 0; l < m; ++l) {
            acc = cmac(acc, in[l * f + j], twid(tw, e, sg));
            e += step;
            if (e >= n) e -= n;
        }
        D[idx] = acc;
    }
}

// stage b for one output k
__device__ __forceinline__ double2 dft_stage_b(const double2 *D, int n, int f, int m, const double2 *tw, double sg,
                                               int k) {
    const int km = k % m;
    double2 acc = make_double2(0.0, 0.0);
    int e = 0;
    for (int j = 0; j < f; ++j) {
        acc = cmac(acc, D[j * m + km], twid(tw, e, sg));
        e += k;
        if (e >= n) e -= n;
    }
    return acc;
}

// stage a over a real input in LDS
__device__ void dft_stage_a_real(const float *in, double2 *D, int n, int f, int m, const double2 *tw, double sg) {
    for (int idx = threadIdx.x; idx < n; idx += AT) {
        const int j = idx / m, kp = idx - j * m;
        const int step = (f * kp) % n;
        double2 acc = make_double2(0.0, 0.0);
        int e = 0;
        for (int l = 0; l < m; ++l) {
            const double v = (double)in[l * f + j];
            const double2 w = twid(tw, e, sg);
            acc.x = fma(v, w.x, acc.x);
            acc.y = fma(v, w.y, acc.y);
            e += step;
            if (e >= n) e -= n;
        }
        D[idx] = acc;
    }
}

// Forward transform along x of row y of batch b's surface plane:
// X[b][y][a], a < n1/2 + 1.  Dynamic LDS: D, tw (n1 double2 each), the row
// (n1 floats).
__global__ __launch_bounds__(AT) void air_rows_fwd(const float *F, long long fstride, long long plane_off, int pitch,
                                                    int n1, int f1, int n2, const double2 *tw1, double2 *X) {
    extern __shared__ double2 lds[];
    double2 *D = lds, *tw = D + n1;
    float *row = reinterpret_cast<float *>(tw + n1);
    const int y = blockIdx.x, b = blockIdx.y, n1h = n1 / 2 + 1, m1 = n1 / f1;
    const float *src = F + b * fstride + plane_off + (long long)y * pitch;
    for (int x = threadIdx.x; x < n1; x += AT) {
        row[x] = src[x];
        tw[x] = tw1[x];
    }
    __syncthreads();
    dft_stage_a_real(row, D, n1, f1, m1, tw, -1.0);
    __syncthreads();
    double2 *out = X + ((long long)b * n2 + y) * n1h;
    for (int k = threadIdx.x; k < n1h; k += AT) out[k] = dft_stage_b(D, n1, f1, m1, tw, -1.0, k);
}

// Block (a, b, j): column a (kx) of batch b, output j of that batch: the
// forward transform of the column along y, times the spectral factor of
// output j, the inverse transform along y into W[o][y][a].
//   E (HF = false): batch b = component * nsrc + source, outputs j = m - 1
//     for the ghost nodes m = 1 .. nm, o = j 2 nsrc + b, factor dec[j][bin]
//     (real);
//   H (HF = true): batch b = source, outputs j = 2 (m - 1) + c for H1
//     (c = 0) and H2 (c = 1), o = (m - 1) 2 nsrc + c nsrc + b, factors
//     rx / ry[m - 1][bin] (complex).
// Dynamic LDS: col, D, t2 (n2 double2 each).
template <bool HF>
__global__ __launch_bounds__(AT) void air_cols(const double2 *X, double2 *W, const double *dec, const double2 *rx,
                                                const double2 *ry, const double2 *tw2, int n1h, int n2, int f2,
                                                int nsrc) {
    extern __shared__ double2 lds[];
    double2 *col = lds, *D = col + n2, *t2 = D + n2;
    const int a = blockIdx.x, b = blockIdx.y, j = blockIdx.z, tid = threadIdx.x, m2 = n2 / f2;
    const long long nbin = (long long)n2 * n1h;
    const double2 *in = X + (long long)b * nbin + a;
    for (int q = tid; q < n2; q += AT) {
        col[q] = in[(long long)q * n1h];
        t2[q] = tw2[q];
    }
    __syncthreads();
    dft_stage_a(col, D, n2, f2, m2, t2, -1.0);
    __syncthreads();
    const int mm = HF ? j / 2 : j, c = HF ? j % 2 : 0;
    for (int q = tid; q < n2; q += AT) {
        const double2 v = dft_stage_b(D, n2, f2, m2, t2, -1.0, q);
        const long long bin = (long long)mm * nbin + (long long)q * n1h + a;
        if (HF) {
            const double2 g = (c == 0 ? rx : ry)[bin];
            col[q] = make_double2(v.x * g.x - v.y * g.y, v.x * g.y + v.y * g.x);
        } else {
            const double d = dec[bin];
            col[q] = make_double2(v.x * d, v.y * d);
        }
    }
    __syncthreads();
    dft_stage_a(col, D, n2, f2, m2, t2, 1.0);
    __syncthreads();
    const int o = mm * 2 * nsrc + (HF ? c * nsrc + b : b);
    double2 *out = W + (long long)o * nbin + a;
    for (int y = tid; y < n2; y += AT) out[(long long)y * n1h] = dft_stage_b(D, n2, f2, m2, t2, 1.0, y);
}

// Inverse transform along x of row y of output plane o (the half spectrum
// W[o][y][a], a < n1/2 + 1, extended by Hermitian symmetry, the imaginary
// parts of a = 0 and a = n1/2 dropped as a complex-to-real transform does)
// into plane ks - m of field array o mod 2 nsrc, m = o / (2 nsrc) + 1.
// Dynamic LDS: S, D, tw (n1 double2 each).
__global__ __launch_bounds__(AT) void air_rows_inv(const double2 *W, float *F, long long fstride, long long plane,
                                                    int ks, int two_ns, int pitch, int n1, int f1, int n2,
                                                    const double2 *tw1) {
    extern __shared__ double2 lds[];
    double2 *S = lds, *D = S + n1, *tw = D + n1;
    const int y = blockIdx.x, o = blockIdx.y, n1h = n1 / 2 + 1, m1 = n1 / f1;
    const double2 *in = W + ((long long)o * n2 + y) * n1h;
    for (int x = threadIdx.x; x < n1; x += AT) {
        double2 v;
        if (x < n1h) {
            v = in[x];
            if (x == 0 || 2 * x == n1) v.y = 0.0;
        } else {
            const double2 u = in[n1 - x];
            v = make_double2(u.x, -u.y);
        }
        S[x] = v;
        tw[x] = tw1[x];
    }
    __syncthreads();
    dft_stage_a(S, D, n1, f1, m1, tw, 1.0);
    __syncthreads();
    const int a = o % two_ns, m = o / two_ns + 1;
    float *out = F + a * fstride + (long long)(ks - m) * plane + (long long)y * pitch;
    for (int x = threadIdx.x; x < n1; x += AT) out[x] = (float)dft_stage_b(D, n1, f1, m1, tw, 1.0, x).x;
}

int largest_divisor_to_sqrt(int n) {
    int f = 1;
    for (int d = 1; (long long)d * d <= n; ++d)
        if (n % d == 0) f = d;
    return f;
}

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
    for (void *p : {(void *)spec_, (void *)work_, (void *)decE_, (void *)rx_, (void *)ry_, (void *)ghost_,
                    (void *)tw1_, (void *)tw2_, (void *)dec64_, (void *)rx64_, (void *)ry64_, (void *)sp64_,
                    (void *)wk64_})
        if (p) (void)hipFree(p);
}

bool AirBoundary::init(const AirSpec &spec, std::string &err) {
    s_ = spec;
    const int n1 = s_.n1, n2 = s_.n2, n1h = n1 / 2 + 1, r = s_.r, ns = s_.nsrc;
    nbin_ = n2 * n1h;
    f1_ = largest_divisor_to_sqrt(n1);
    f2_ = largest_divisor_to_sqrt(n2);
    const bool fits = n1 <= kDftMax && n2 <= kDftMax;
    // by size: the FP64 direct kernels whenever both axes fit, hipFFT above
    direct_ = s_.method == 2 || (s_.method == 0 && fits);
    if (direct_ && !fits) {
        err = "the direct air-boundary transforms take at most " + std::to_string(kDftMax) +
              " points per horizontal axis";
        return false;
    }
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
    if (!direct_ &&
        (!plan(fwdE_, have_fwdE_, HIPFFT_R2C, 2 * ns) || !plan(fwdH_, have_fwdH_, HIPFFT_R2C, ns) ||
         !plan(invE_, have_invE_, HIPFFT_C2R, 2 * ns) || !plan(invH_, have_invH_, HIPFFT_C2R, 2 * ns)))
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
    if (!direct_ && r - 1 > 1 && !plan_all(invEall_, have_invEall_, (r - 1) * 2 * ns)) return false;
    if (!direct_ && r > 1 && !plan_all(invHall_, have_invHall_, r * 2 * ns)) return false;
    // spectral factors in FP64 with the 1/(n1 n2) of the inverse (in FP32 for hipFFT)
    const double norm = 1.0 / ((double)n1 * n2);
    const double pi = 3.14159265358979323846;
    std::vector<double> dec((size_t)std::max(1, r - 1) * nbin_, 0.0);
    std::vector<double2> fx((size_t)r * nbin_), fy((size_t)r * nbin_);
    for (int b = 0; b < n2; ++b) {
        const int qy = b <= (n2 - 1) / 2 ? b : b - n2;
        const double ky = 2.0 * pi * qy / (n2 * s_.dy);
        for (int a = 0; a < n1h; ++a) {
            const double kx = 2.0 * pi * a / (n1 * s_.dx);
            const double kap = std::sqrt(kx * kx + ky * ky);
            const size_t bin = (size_t)b * n1h + a;
            for (int m = 1; m < r; ++m) dec[(size_t)(m - 1) * nbin_ + bin] = std::exp(-kap * s_.hE[m - 1]) * norm;
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
                fx[(size_t)(m - 1) * nbin_ + bin] = make_double2(xr * d, xi * d);
                fy[(size_t)(m - 1) * nbin_ + bin] = make_double2(yr * d, yi * d);
            }
        }
    }
    hipError_t e = hipSuccess;
    auto upload = [&](void **dst, const void *src, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(dst, bytes);
        if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    if (direct_) {
        std::vector<double2> t1(n1), t2(n2);
        for (int q = 0; q < n1; ++q) t1[q] = make_double2(std::cos(2.0 * pi * q / n1), std::sin(2.0 * pi * q / n1));
        for (int q = 0; q < n2; ++q) t2[q] = make_double2(std::cos(2.0 * pi * q / n2), std::sin(2.0 * pi * q / n2));
        upload((void **)&tw1_, t1.data(), t1.size() * sizeof(double2));
        upload((void **)&tw2_, t2.data(), t2.size() * sizeof(double2));
        upload((void **)&dec64_, dec.data(), dec.size() * sizeof(double));
        upload((void **)&rx64_, fx.data(), fx.size() * sizeof(double2));
        upload((void **)&ry64_, fy.data(), fy.size() * sizeof(double2));
        if (e == hipSuccess) e = hipMalloc(&sp64_, (size_t)2 * ns * nbin_ * sizeof(double2));
        if (e == hipSuccess) e = hipMalloc(&wk64_, (size_t)std::max(1, r) * 2 * ns * nbin_ * sizeof(double2));
    } else {
        std::vector<float> dec32(dec.begin(), dec.end());
        std::vector<float2> fx32(fx.size()), fy32(fy.size());
        for (size_t i = 0; i < fx.size(); ++i) {
            fx32[i] = make_float2((float)fx[i].x, (float)fx[i].y);
            fy32[i] = make_float2((float)fy[i].x, (float)fy[i].y);
        }
        upload((void **)&decE_, dec32.data(), dec32.size() * sizeof(float));
        upload((void **)&rx_, fx32.data(), fx32.size() * sizeof(float2));
        upload((void **)&ry_, fy32.data(), fy32.size() * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&spec_, (size_t)2 * ns * nbin_ * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&work_, (size_t)std::max(1, r) * 2 * ns * nbin_ * sizeof(float2));
        if (e == hipSuccess && r > 1)
            e = hipMalloc(&ghost_, (size_t)r * 2 * ns * n2 * s_.pitch * sizeof(float));
    }
    if (e != hipSuccess) {
        err = std::string("air boundary buffers: ") + hipGetErrorString(e);
        return false;
    }
    return true;
}

bool AirBoundary::fill_E(float *E1, hipStream_t st, std::string &err) {
    const int r = s_.r, ns = s_.nsrc;
    if (r < 2) return true;
    if (direct_) {
        const int n1 = s_.n1, n2 = s_.n2, n1h = n1 / 2 + 1;
        hipLaunchKernelGGL(air_rows_fwd, dim3(n2, 2 * ns), dim3(AT), n1 * (2 * sizeof(double2) + sizeof(float)), st,
                           E1, s_.fstride, (long long)s_.ks * s_.plane, s_.pitch, n1, f1_, n2, tw1_, sp64_);
        hipLaunchKernelGGL(air_cols<false>, dim3(n1h, 2 * ns, r - 1), dim3(AT), 3 * n2 * sizeof(double2), st, sp64_,
                           wk64_, dec64_, rx64_, ry64_, tw2_, n1h, n2, f2_, ns);
        hipLaunchKernelGGL(air_rows_inv, dim3(n2, (r - 1) * 2 * ns), dim3(AT), 3 * n1 * sizeof(double2), st, wk64_,
                           E1, s_.fstride, s_.plane, s_.ks, 2 * ns, s_.pitch, n1, f1_, n2, tw1_);
        return true;
    }
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
    if (direct_) {
        const int n1 = s_.n1, n2 = s_.n2, n1h = n1 / 2 + 1;
        hipLaunchKernelGGL(air_rows_fwd, dim3(n2, ns), dim3(AT), n1 * (2 * sizeof(double2) + sizeof(float)), st, H3,
                           s_.fstride, (long long)s_.ks * s_.plane, s_.pitch, n1, f1_, n2, tw1_, sp64_);
        hipLaunchKernelGGL(air_cols<true>, dim3(n1h, ns, 2 * r), dim3(AT), 3 * n2 * sizeof(double2), st, sp64_,
                           wk64_, dec64_, rx64_, ry64_, tw2_, n1h, n2, f2_, ns);
        hipLaunchKernelGGL(air_rows_inv, dim3(n2, r * 2 * ns), dim3(AT), 3 * n1 * sizeof(double2), st, wk64_, H1,
                           s_.fstride, s_.plane, s_.ks, 2 * ns, s_.pitch, n1, f1_, n2, tw1_);
        return true;
    }
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
