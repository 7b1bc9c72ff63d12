// Air above the sea surface (Section 3.3): ghost planes above the surface
// node filled by 2-D FFTs after each half step.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <string>
#include <vector>

namespace emm {

// largest plane axis of the direct (non-FFT) ghost-fill transforms
constexpr int kDftMax = 512;

struct AirSpec {
    int n1, n2, n3, pitch;     // padded grid; fields [n3][n2][pitch]
    int ks, r, nsrc;           // surface node, half stencil, sources
    long long plane, fstride;  // n2 * pitch, one source's field array
    double dx, dy;             // uniform horizontal spacings
    std::vector<double> hE;    // heights of the E ghost nodes ks - m, m = 1 .. r - 1
    std::vector<double> hH;    // heights of the H ghost half nodes ks - m, m = 1 .. r
    int method = 0;            // transforms: 0 = by plane size, 1 = hipFFT, 2 = direct kernels
};

class AirBoundary {
  public:
    AirBoundary() = default;
    AirBoundary(const AirBoundary &) = delete;
    AirBoundary &operator=(const AirBoundary &) = delete;
    ~AirBoundary();
    // plans, spectral tables and work buffers; false with `err` set on failure
    bool init(const AirSpec &spec, std::string &err);
    const AirSpec &spec() const { return s_; }
    // true: the fills use the direct transform kernels, false: hipFFT
    bool direct() const { return direct_; }
    // E1 (component 0, source 0; E2 follows after nsrc field arrays):
    // E1, E2 ghost nodes from the surface plane
    bool fill_E(float *E1, hipStream_t st, std::string &err);
    // H1 (H2 follows), H3: H1, H2 ghost half nodes from H3 at the surface
    bool fill_H(float *H1, const float *H3, hipStream_t st, std::string &err);

  private:
    AirSpec s_{};
    int nbin_ = 0;                       // n2 * (n1/2 + 1)
    // direct transforms in FP64 (no FFT plans): three kernels per fill, the
    // rows of the surface plane, the columns with the spectral factors, the
    // inverse rows into the ghost planes; n = f m splits per axis and
    // twiddle tables
    bool direct_ = false;
    int f1_ = 1, f2_ = 1;
    double2 *tw1_ = nullptr, *tw2_ = nullptr;
    double *dec64_ = nullptr;                // FP64 spectral factors, same layout as decE_, rx_, ry_
    double2 *rx64_ = nullptr, *ry64_ = nullptr;
    double2 *sp64_ = nullptr;                // [batch][n2][n1/2 + 1] row transforms of a fill
    double2 *wk64_ = nullptr;                // [outputs][n2][n1/2 + 1] column results of a fill
    hipfftHandle fwdE_ = 0, fwdH_ = 0, invE_ = 0, invH_ = 0;
    bool have_fwdE_ = false, have_fwdH_ = false, have_invE_ = false, have_invH_ = false;
    // inverse transforms of all ghost planes of a fill in one execution, into
    // ghost_ (planes [m - 1][component][source], rows `pitch` apart), then one
    // scatter kernel; used when a fill has more than one plane per component
    hipfftHandle invEall_ = 0, invHall_ = 0;
    bool have_invEall_ = false, have_invHall_ = false;
    float *ghost_ = nullptr;
    float2 *spec_ = nullptr, *work_ = nullptr;
    float *decE_ = nullptr;              // [r-1][nbin] exp(-|k| h) / (n1 n2)
    float2 *rx_ = nullptr, *ry_ = nullptr;   // [r][nbin]
};

}  // namespace emm
