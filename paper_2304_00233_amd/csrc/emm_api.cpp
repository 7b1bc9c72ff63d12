// C ABI of libemm: validation, set-up, device buffers and the time loop.
// Declarations and argument conventions: include/emm.h.
#include "emm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "emm_internal.h"
#include "emm_setup.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;

thread_local std::string g_last_error;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct emm_model {
    emm_options opt{};
    int n[3] = {0, 0, 0};     // interior nodes
    int np[3] = {0, 0, 0};    // padded nodes
    int pitch = 0;
    int r = 2, nb = 0, nbe = 0;
    double dt = 0.0, omega0 = 0.0;
    std::vector<double> axes[3], half[3];
    std::vector<double> cm[3], cp[3];
    double rho_slab_max[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int device = 0;
    hipStream_t own_stream = nullptr;
    // model-lifetime device data
    float *ce[3] = {nullptr, nullptr, nullptr};
    float *tab[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // cmx cmy cmz cpx cpy cpz
    // forward-lifetime device data (grown on demand, kept between forwards)
    DevBuf fields, psi, acc, cpml, srcinfo, srcq, wav, items, itemw, phase;
    hipEvent_t ev_loop[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ring;       // profiling: start/end pairs
    emm_info info{};
    std::string err;
};

namespace {

emm_status fail(emm_model *m, emm_status s, const std::string &msg) {
    g_last_error = msg;
    if (m) m->err = msg;
    return s;
}

#define HIP_OK(m, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((m), EMM_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

emm_status ensure(emm_model *m, DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return EMM_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t fr = 0, tot = 0;
    HIP_OK(m, hipMemGetInfo(&fr, &tot));
    if (bytes > fr) return fail(m, EMM_ERR_OOM, "device memory request of " + std::to_string(bytes) +
                                                     " bytes exceeds the " + std::to_string(fr) + " free");
    HIP_OK(m, hipMalloc(&b.p, std::max<size_t>(bytes, 256)));
    b.bytes = bytes;
    return EMM_OK;
}

bool finite_increasing(const double *x, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x[i]) || (i && !(x[i] > x[i - 1]))) return false;
    return true;
}

// Algorithmic bytes of one step for one source: E step reads H1..3, E1..3,
// ce1..3 and writes E1..3 (48 B/cell); H step reads E1..3, H1..3 and writes
// H1..3 (36 B/cell); each CPML slab cell reads and writes two memory
// variables per axis per half step (16 B).
void step_bytes(const emm_model *m, double &eb, double &hb) {
    const double N = double(m->np[0]) * m->np[1] * m->np[2];
    double ncpml = 0.0;
    if (m->nb > 0)
        for (int a = 0; a < 3; ++a) ncpml += 2.0 * m->nb * N / m->np[a];
    eb = 48.0 * N + 16.0 * ncpml;
    hb = 36.0 * N + 16.0 * ncpml;
}

int choose_kz(const emm_model *m, int xt, int yt, int nsrc) {
    const int nzv = m->np[2] - 2 * m->r;
    if (m->opt.tile_kz > 0) return std::min(m->opt.tile_kz, nzv);
    const long long per_chunk = (long long)xt * yt * nsrc;
    long long zc = std::max<long long>(1, (4096 + per_chunk - 1) / per_chunk);
    zc = std::min<long long>(zc, std::max(1, nzv / 8));
    return (int)((nzv + zc - 1) / zc);
}

}  // namespace

extern "C" {

emm_status emm_default_options(emm_options *o) {
    if (!o) return fail(nullptr, EMM_ERR_ARG, "options pointer is NULL");
    std::memset(o, 0, sizeof(*o));
    o->rd = 2;
    o->nb = 10;
    o->ne = -1;
    o->f0 = 1.0;
    o->cfl = 0.99;
    o->dt_override = 0.0;
    o->nt = 0;
    o->dft_mode = 0;
    o->cpml_R = 1e-5;
    o->cpml_npow = 2.0;
    o->cpml_alpha_max = 0.0;
    o->wavelet_fpeak = 0.0;
    o->allow_unstable = 0;
    o->profile = 0;
    o->tile_kz = 0;
    return EMM_OK;
}

const char *emm_status_str(emm_status s) {
    switch (s) {
    case EMM_OK: return "EMM_OK";
    case EMM_ERR_ARG: return "EMM_ERR_ARG";
    case EMM_ERR_GRID: return "EMM_ERR_GRID";
    case EMM_ERR_MODEL: return "EMM_ERR_MODEL";
    case EMM_ERR_GEOMETRY: return "EMM_ERR_GEOMETRY";
    case EMM_ERR_FREQ: return "EMM_ERR_FREQ";
    case EMM_ERR_CFL: return "EMM_ERR_CFL";
    case EMM_ERR_NONFINITE: return "EMM_ERR_NONFINITE";
    case EMM_ERR_OOM: return "EMM_ERR_OOM";
    case EMM_ERR_DEVICE: return "EMM_ERR_DEVICE";
    }
    return "EMM_ERR_UNKNOWN";
}

const char *emm_last_error(const emm_model *m) {
    if (m) return m->err.c_str();
    return g_last_error.c_str();
}

void emm_destroy(emm_model *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    if (m->own_stream) (void)hipStreamSynchronize(m->own_stream);
    for (float *p : m->ce) if (p) (void)hipFree(p);
    for (float *p : m->tab) if (p) (void)hipFree(p);
    for (DevBuf *b : {&m->fields, &m->psi, &m->acc, &m->cpml, &m->srcinfo, &m->srcq, &m->wav,
                      &m->items, &m->itemw, &m->phase})
        if (b->p) (void)hipFree(b->p);
    for (hipEvent_t e : m->ev_loop) if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : m->ring) if (e) (void)hipEventDestroy(e);
    if (m->own_stream) (void)hipStreamDestroy(m->own_stream);
    delete m;
}

emm_status emm_query(const emm_model *m, emm_info *info) {
    if (!m || !info) return fail(nullptr, EMM_ERR_ARG, "NULL model or info pointer");
    *info = m->info;
    return EMM_OK;
}

emm_status emm_create(const emm_grid *g, const emm_options *o, emm_model **out) {
    if (!out) return fail(nullptr, EMM_ERR_ARG, "out pointer is NULL");
    *out = nullptr;
    if (!g || !o) return fail(nullptr, EMM_ERR_ARG, "NULL grid or options");
    emm_options opt = *o;
    if (opt.rd < 1 || opt.rd > emm::kMaxR) return fail(nullptr, EMM_ERR_ARG, "rd must be 1..4");
    if (opt.ne < 0) opt.ne = opt.rd + 5;
    if (opt.nb < 0) return fail(nullptr, EMM_ERR_ARG, "nb must be >= 0");
    if (!(opt.f0 > 0.0) || !std::isfinite(opt.f0)) return fail(nullptr, EMM_ERR_ARG, "f0 must be > 0");
    if (!(opt.cfl > 0.0) || !std::isfinite(opt.cfl)) return fail(nullptr, EMM_ERR_ARG, "cfl must be > 0");
    if (opt.nt < 0 || opt.dft_mode < 0 || opt.dft_mode > 1 || opt.tile_kz < 0 ||
        !(opt.cpml_R > 0.0 && opt.cpml_R < 1.0) || !(opt.cpml_npow >= 0.0) ||
        !(opt.cpml_alpha_max >= 0.0) || !(opt.wavelet_fpeak >= 0.0) || !(opt.dt_override >= 0.0))
        return fail(nullptr, EMM_ERR_ARG, "option out of range");
    const int nd[3] = {g->n1, g->n2, g->n3};
    const double *xs[3] = {g->x1, g->x2, g->x3};
    const float *rho[3] = {g->rho11, g->rho22, g->rho33};
    for (int a = 0; a < 3; ++a) {
        if (!xs[a] || !rho[a]) return fail(nullptr, EMM_ERR_ARG, "NULL coordinate or resistivity array");
        if (nd[a] < 2 * opt.rd + 1)
            return fail(nullptr, EMM_ERR_GRID, "every axis needs at least 2*rd+1 nodes");
        if (!finite_increasing(xs[a], nd[a]))
            return fail(nullptr, EMM_ERR_GRID, "coordinates must be finite and strictly increasing");
    }
    const long long ncell = (long long)nd[0] * nd[1] * nd[2];
    for (int a = 0; a < 3; ++a)
        for (long long c = 0; c < ncell; ++c)
            if (!(rho[a][c] > 0.0f) || !std::isfinite(rho[a][c]))
                return fail(nullptr, EMM_ERR_MODEL, "resistivity must be finite and > 0");

    emm_model *m = new (std::nothrow) emm_model();
    if (!m) return fail(nullptr, EMM_ERR_OOM, "host allocation failed");
    m->opt = opt;
    m->r = opt.rd;
    m->nb = opt.nb;
    m->nbe = opt.nb + opt.ne;
    m->omega0 = 2.0 * kPi * opt.f0;
    for (int a = 0; a < 3; ++a) {
        m->n[a] = nd[a];
        m->axes[a] = emm::pad_axis(xs[a], nd[a], m->nbe);
        m->half[a] = emm::half_nodes(m->axes[a]);
        m->np[a] = (int)m->axes[a].size();
        emm::fd_tables(m->axes[a], m->r, m->cm[a], m->cp[a]);
    }
    m->pitch = (m->np[0] + emm::kTileX - 1) / emm::kTileX * emm::kTileX;

    // time step (Section 3.2): dt = cfl/eta, eta = 1/2 v_max sqrt(sum D_d^2)
    double rmax = 0.0;
    for (int a = 0; a < 3; ++a)
        for (long long c = 0; c < ncell; ++c) rmax = std::max(rmax, (double)rho[a][c]);
    const double vmax = std::sqrt(2.0 * m->omega0 * rmax / kMu0);
    double dsum = 0.0;
    const int L = 2 * m->r;
    for (int a = 0; a < 3; ++a) {
        double dmax = 0.0;
        for (int i = 0; i < m->np[a]; ++i) {
            double sm = 0.0, sp = 0.0;
            for (int q = 0; q < L; ++q) {
                sm += std::fabs(m->cm[a][i * L + q]);
                sp += std::fabs(m->cp[a][i * L + q]);
            }
            dmax = std::max(dmax, std::max(sm, sp));
        }
        dsum += dmax * dmax;
    }
    const double eta = 0.5 * vmax * std::sqrt(dsum);
    m->dt = opt.cfl / eta;
    if (opt.dt_override > 0.0) {
        if (opt.dt_override > 1.0 / eta && !opt.allow_unstable) {
            delete m;
            return fail(nullptr, EMM_ERR_CFL, "dt_override exceeds the stability limit 1/eta");
        }
        m->dt = opt.dt_override;
    }
    // largest resistivity in each CPML slab (the padded model replicates the
    // interior faces, so the slab of the low x side holds the values at i = 0)
    for (int a = 0; a < 3; ++a)
        for (int side = 0; side < 2; ++side) {
            const int fixed = side ? nd[a] - 1 : 0;
            int lo[3] = {0, 0, 0}, hi[3] = {nd[0], nd[1], nd[2]};
            lo[a] = fixed;
            hi[a] = fixed + 1;
            double mx = 0.0;
            for (int c3 = 0; c3 < 3; ++c3)
                for (int k = lo[2]; k < hi[2]; ++k)
                    for (int j = lo[1]; j < hi[1]; ++j)
                        for (int i = lo[0]; i < hi[0]; ++i)
                            mx = std::max(mx, (double)rho[c3][((long long)k * nd[1] + j) * nd[0] + i]);
            m->rho_slab_max[a][side] = mx;
        }

    // device
    HIP_OK(m, hipGetDevice(&m->device));
    {
        hipError_t e = hipStreamCreate(&m->own_stream);
        if (e != hipSuccess) {
            emm_status s = fail(m, EMM_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            delete m;
            return s;
        }
    }
    const long long N = (long long)m->pitch * m->np[1] * m->np[2];
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess || (size_t)(3 * N * 4) > fr) {
        emm_destroy(m);
        return fail(nullptr, EMM_ERR_OOM, "model does not fit in free device memory");
    }
    // dt/eps = dt * 2 omega0 rho on the padded grid (rho replicated into the padding)
    std::vector<float> buf(N, 0.0f);
    for (int c3 = 0; c3 < 3; ++c3) {
        for (int k = 0; k < m->np[2]; ++k) {
            const int kk = std::min(std::max(k - m->nbe, 0), nd[2] - 1);
            for (int j = 0; j < m->np[1]; ++j) {
                const int jj = std::min(std::max(j - m->nbe, 0), nd[1] - 1);
                float *row = &buf[((long long)k * m->np[1] + j) * m->pitch];
                const float *src = rho[c3] + ((long long)kk * nd[1] + jj) * nd[0];
                for (int i = 0; i < m->np[0]; ++i) {
                    const int ii = std::min(std::max(i - m->nbe, 0), nd[0] - 1);
                    row[i] = (float)(m->dt * 2.0 * m->omega0 * (double)src[ii]);
                }
            }
        }
        hipError_t e = hipMalloc(&m->ce[c3], N * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(m->ce[c3], buf.data(), N * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            emm_status s = fail(nullptr, EMM_ERR_DEVICE, std::string("ce upload: ") + hipGetErrorString(e));
            emm_destroy(m);
            return s;
        }
    }
    for (int t = 0; t < 6; ++t) {
        const std::vector<double> &src = t < 3 ? m->cm[t] : m->cp[t - 3];
        std::vector<float> f(src.begin(), src.end());
        hipError_t e = hipMalloc(&m->tab[t], f.size() * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(m->tab[t], f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            emm_status s = fail(nullptr, EMM_ERR_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
            emm_destroy(m);
            return s;
        }
    }
    m->info.dt = m->dt;
    m->info.nt = opt.nt;
    m->info.n1pad = m->np[0];
    m->info.n2pad = m->np[1];
    m->info.n3pad = m->np[2];
    m->info.cells = (long long)m->np[0] * m->np[1] * m->np[2];
    step_bytes(m, m->info.e_bytes, m->info.h_bytes);
    m->info.bytes_per_step = m->info.e_bytes + m->info.h_bytes;
    *out = m;
    return EMM_OK;
}

emm_status emm_forward(emm_model *m, const emm_source *src, int nsrc, const emm_receiver *rec,
                       int nrec, unsigned chan_mask, const double *freq_hz, int nfreq,
                       double *green, void *hip_stream) {
    if (!m) return fail(nullptr, EMM_ERR_ARG, "NULL model");
    m->err.clear();
    if (!src || !rec || !green || nsrc < 1 || nrec < 1 || chan_mask == 0 || (chan_mask & ~0x3Fu))
        return fail(m, EMM_ERR_ARG, "bad sources, receivers, output pointer or channel mask");
    if (!freq_hz || nfreq < 1) return fail(m, EMM_ERR_FREQ, "need at least one frequency");
    for (int f = 0; f < nfreq; ++f)
        if (!(freq_hz[f] > 0.0) || !std::isfinite(freq_hz[f]))
            return fail(m, EMM_ERR_FREQ, "frequencies must be finite and > 0");
    const int r = m->r, L = 2 * r, L3 = L * L * L;
    std::vector<int> chans;
    for (int c = 0; c < 6; ++c)
        if (chan_mask >> c & 1u) chans.push_back(c);
    const int nch = (int)chans.size();
    // staggering (half along x, y, z) of Ex, Ey, Ez, Hx, Hy, Hz
    static const int stag[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
    auto coords = [&](int a, int h) -> const std::vector<double> & { return h ? m->half[a] : m->axes[a]; };
    auto inside = [&](int a, int base) { return base >= m->nbe && base + L - 1 <= m->np[a] - 1 - m->nbe; };

    // sources: (2r)^3 stencil on the E_comp grid, J = moment w / V, scaled to max |q| = 1
    std::vector<int> sinfo(4 * nsrc);
    std::vector<float> sq((size_t)nsrc * L3);
    std::vector<double> sscale(nsrc);
    for (int s = 0; s < nsrc; ++s) {
        const emm_source &S = src[s];
        if (S.comp < 0 || S.comp > 2 || !std::isfinite(S.moment) || S.moment == 0.0 ||
            !std::isfinite(S.x) || !std::isfinite(S.y) || !std::isfinite(S.z))
            return fail(m, EMM_ERR_ARG, "source component must be 0..2 with a finite non-zero moment");
        const double p[3] = {S.x, S.y, S.z};
        double w[3][2 * emm::kMaxR];
        int base[3];
        for (int a = 0; a < 3; ++a) {
            base[a] = emm::point_stencil(coords(a, a == S.comp), p[a], r, w[a]);
            if (!inside(a, base[a])) return fail(m, EMM_ERR_GEOMETRY, "source stencil leaves the interior");
        }
        // control volume: primal interval along comp, dual intervals across
        double ext[3][2 * emm::kMaxR];
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < L; ++q) {
                const int idx = base[a] + q;
                ext[a][q] = a == S.comp ? m->axes[a][idx + 1] - m->axes[a][idx]
                                        : m->half[a][idx] - m->half[a][idx - 1];
            }
        std::vector<double> qd(L3);
        double qmax = 0.0;
        for (int c = 0; c < L; ++c)
            for (int b = 0; b < L; ++b)
                for (int a = 0; a < L; ++a) {
                    const double v = S.moment * w[0][a] * w[1][b] * w[2][c] / (ext[0][a] * ext[1][b] * ext[2][c]);
                    qd[(c * L + b) * L + a] = v;
                    qmax = std::max(qmax, std::fabs(v));
                }
        sscale[s] = 1.0 / qmax;
        for (int q = 0; q < L3; ++q) sq[(size_t)s * L3 + q] = (float)(qd[q] * sscale[s]);
        sinfo[4 * s] = S.comp;
        sinfo[4 * s + 1] = base[0];
        sinfo[4 * s + 2] = base[1];
        sinfo[4 * s + 3] = base[2];
    }
    // receiver items: E channels in the H-step launch, H channels in the E-step launch
    std::vector<int> info_e, info_h;     // {src, field, bx, by, bz, slot}
    std::vector<float> w_e, w_h;
    for (int i = 0; i < nrec; ++i) {
        const double p[3] = {rec[i].x, rec[i].y, rec[i].z};
        if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]))
            return fail(m, EMM_ERR_ARG, "receiver position not finite");
        for (int c = 0; c < nch; ++c) {
            const int ch = chans[c];
            double w[3][2 * emm::kMaxR];
            int base[3];
            for (int a = 0; a < 3; ++a) {
                base[a] = emm::point_stencil(coords(a, stag[ch][a]), p[a], r, w[a]);
                if (!inside(a, base[a])) return fail(m, EMM_ERR_GEOMETRY, "receiver stencil leaves the interior");
            }
            std::vector<int> &inf = ch < 3 ? info_h : info_e;   // E channels -> H-step launch
            std::vector<float> &wv = ch < 3 ? w_h : w_e;
            for (int s = 0; s < nsrc; ++s) {
                const int slot = (s * nrec + i) * nch + c;
                inf.insert(inf.end(), {s, ch % 3, base[0], base[1], base[2], slot});
                for (int a = 0; a < 3; ++a)
                    for (int q = 0; q < L; ++q) wv.push_back((float)w[a][q]);
            }
        }
    }
    // recorded in the H step: E^{n+1}; in the E step: H^{n+1/2}
    std::vector<int> &items_hstep = info_h;  // holds E channels
    std::vector<int> &items_estep = info_e;  // holds H channels
    std::vector<float> &wts_hstep = w_h, &wts_estep = w_e;

    // time axis, wavelet, DTFT phases, CPML
    double fmax = 0.0, fmin = 1e300;
    for (int f = 0; f < nfreq; ++f) {
        fmax = std::max(fmax, freq_hz[f]);
        fmin = std::min(fmin, freq_hz[f]);
    }
    const double fp = m->opt.wavelet_fpeak > 0.0 ? m->opt.wavelet_fpeak : 2.0 * std::sqrt(fmax * m->opt.f0);
    int nt = m->opt.nt;
    if (nt == 0) {
        const double tau = 1.0 / (kPi * fp);
        const double decay = emm::omega_prime(fmin, m->omega0).imag();
        const double T = 7.0 * tau + std::log(1e6) / decay;
        nt = (int)(std::ceil(T / m->dt / 100.0) * 100.0);
    }
    const std::vector<double> sw = emm::wavelet(nt, m->dt, fp);
    std::vector<float> swf(sw.begin(), sw.end());
    std::vector<std::complex<double>> Shat(nfreq, 0.0), wp(nfreq);
    std::vector<double2> ph((size_t)2 * nt * nfreq);   // [0]: E-step (H stamps), [1]: H-step (E stamps)
    for (int f = 0; f < nfreq; ++f) {
        wp[f] = emm::omega_prime(freq_hz[f], m->omega0);
        for (int n = 0; n < nt; ++n) {
            const std::complex<double> zh = std::exp(std::complex<double>(0, 1) * wp[f] * ((n + 0.5) * m->dt));
            const std::complex<double> ze = std::exp(std::complex<double>(0, 1) * wp[f] * ((n + 1.0) * m->dt));
            Shat[f] += (double)swf[n] * zh;
            ph[(size_t)n * nfreq + f] = make_double2(zh.real(), zh.imag());
            ph[(size_t)nt * nfreq + (size_t)n * nfreq + f] = make_double2(ze.real(), ze.imag());
        }
    }
    const double alpha_max = m->opt.cpml_alpha_max > 0.0 ? m->opt.cpml_alpha_max : kPi * fp;
    std::vector<float> cpml;   // per axis: a_int, b_int, a_half, b_half
    std::vector<size_t> cpml_off(12);
    for (int a = 0; a < 3; ++a) {
        auto v = [&](double rho) { return std::sqrt(2.0 * m->omega0 * rho / kMu0); };
        const emm::CpmlAxis c = emm::cpml_axis(m->axes[a], m->nb, m->dt, v(m->rho_slab_max[a][0]),
                                               v(m->rho_slab_max[a][1]), alpha_max, m->opt.cpml_npow,
                                               m->opt.cpml_R);
        const std::vector<double> *parts[4] = {&c.a_int, &c.b_int, &c.a_half, &c.b_half};
        for (int q = 0; q < 4; ++q) {
            cpml_off[a * 4 + q] = cpml.size();
            cpml.insert(cpml.end(), parts[q]->begin(), parts[q]->end());
        }
    }

    // device buffers
    emm_status st;
    HIP_OK(m, hipSetDevice(m->device));
    hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : m->own_stream;
    const long long plane = (long long)m->pitch * m->np[1];
    const long long fstride = plane * m->np[2];
    const int nb = m->nb;
    const long long psxs = nb ? (long long)m->np[2] * m->np[1] * 2 * nb : 0;
    const long long psys = nb ? (long long)m->np[2] * 2 * nb * m->pitch : 0;
    const long long pszs = nb ? (long long)2 * nb * plane : 0;
    const long long ps_per_src = 4 * (psxs + psys + pszs);      // 2 per axis per half step
    const int nslot = nsrc * nrec * nch;
    if ((st = ensure(m, m->fields, (size_t)6 * nsrc * fstride * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->psi, (size_t)std::max<long long>(1, nsrc * ps_per_src) * sizeof(float))) != EMM_OK) return st;
    const size_t acc_elem = m->opt.dft_mode ? sizeof(float4) : sizeof(double2);
    if ((st = ensure(m, m->acc, (size_t)nslot * nfreq * acc_elem)) != EMM_OK) return st;
    if ((st = ensure(m, m->cpml, cpml.size() * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->srcinfo, sinfo.size() * sizeof(int))) != EMM_OK) return st;
    if ((st = ensure(m, m->srcq, sq.size() * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->wav, swf.size() * sizeof(float))) != EMM_OK) return st;
    const size_t ni_e = items_estep.size() / 6, ni_h = items_hstep.size() / 6;
    if ((st = ensure(m, m->items, (items_estep.size() + items_hstep.size()) * sizeof(int))) != EMM_OK) return st;
    if ((st = ensure(m, m->itemw, (wts_estep.size() + wts_hstep.size()) * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->phase, ph.size() * sizeof(double2))) != EMM_OK) return st;

    char *items_d = (char *)m->items.p;
    char *itemw_d = (char *)m->itemw.p;
    HIP_OK(m, hipMemcpyAsync(m->cpml.p, cpml.data(), cpml.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->srcinfo.p, sinfo.data(), sinfo.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->srcq.p, sq.data(), sq.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->wav.p, swf.data(), swf.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    if (!items_estep.empty())
        HIP_OK(m, hipMemcpyAsync(items_d, items_estep.data(), items_estep.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (!items_hstep.empty())
        HIP_OK(m, hipMemcpyAsync(items_d + items_estep.size() * sizeof(int), items_hstep.data(),
                                 items_hstep.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (!wts_estep.empty())
        HIP_OK(m, hipMemcpyAsync(itemw_d, wts_estep.data(), wts_estep.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    if (!wts_hstep.empty())
        HIP_OK(m, hipMemcpyAsync(itemw_d + wts_estep.size() * sizeof(float), wts_hstep.data(),
                                 wts_hstep.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->phase.p, ph.data(), ph.size() * sizeof(double2), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemsetAsync(m->fields.p, 0, (size_t)6 * nsrc * fstride * sizeof(float), stream));
    if (nb) HIP_OK(m, hipMemsetAsync(m->psi.p, 0, (size_t)nsrc * ps_per_src * sizeof(float), stream));
    HIP_OK(m, hipMemsetAsync(m->acc.p, 0, (size_t)nslot * nfreq * acc_elem, stream));

    // kernel parameters
    emm::StepParams P{};
    P.n1 = m->np[0];
    P.n2 = m->np[1];
    P.n3 = m->np[2];
    P.pitch = m->pitch;
    P.plane = plane;
    P.fstride = fstride;
    P.nb = nb;
    P.xt = m->pitch / emm::kTileX;
    P.yt = (m->np[1] - 2 * r + 3) / 4;
    P.kz = choose_kz(m, P.xt, P.yt, nsrc);
    P.zc = (m->np[2] - 2 * r + P.kz - 1) / P.kz;
    P.nsrc = nsrc;
    P.nstencil = P.xt * P.yt * P.zc * nsrc;
    float *F = (float *)m->fields.p;
    P.E1 = F;
    P.E2 = F + (size_t)nsrc * fstride;
    P.E3 = F + (size_t)2 * nsrc * fstride;
    P.H1 = F + (size_t)3 * nsrc * fstride;
    P.H2 = F + (size_t)4 * nsrc * fstride;
    P.H3 = F + (size_t)5 * nsrc * fstride;
    // per-source field arrays are interleaved as [comp][src][...]: source s at + s * fstride
    P.ce1 = m->ce[0];
    P.ce2 = m->ce[1];
    P.ce3 = m->ce[2];
    P.ch = (float)(m->dt / kMu0);
    P.cmx = m->tab[0];
    P.cmy = m->tab[1];
    P.cmz = m->tab[2];
    P.cpx = m->tab[3];
    P.cpy = m->tab[4];
    P.cpz = m->tab[5];
    const float *cp = (const float *)m->cpml.p;
    P.axi = cp + cpml_off[0];
    P.bxi = cp + cpml_off[1];
    P.axh = cp + cpml_off[2];
    P.bxh = cp + cpml_off[3];
    P.ayi = cp + cpml_off[4];
    P.byi = cp + cpml_off[5];
    P.ayh = cp + cpml_off[6];
    P.byh = cp + cpml_off[7];
    P.azi = cp + cpml_off[8];
    P.bzi = cp + cpml_off[9];
    P.azh = cp + cpml_off[10];
    P.bzh = cp + cpml_off[11];
    P.psxs = psxs;
    P.psys = psys;
    P.pszs = pszs;
    P.src_info = (const int *)m->srcinfo.p;
    P.src_q = (const float *)m->srcq.p;
    P.wavelet = (const float *)m->wav.p;
    P.nf = nfreq;
    P.dft_mode = m->opt.dft_mode;
    P.acc = (double2 *)m->acc.p;
    P.acck = (float4 *)m->acc.p;

    emm::StepParams Pe = P, Ph = P;
    float *ps = (float *)m->psi.p;
    // psi layout per half step: x0 x1 (all sources), y0 y1, z0 z1
    const long long bx_ = nsrc * psxs, by_ = nsrc * psys, bz_ = nsrc * pszs;
    Pe.psx0 = ps;
    Pe.psx1 = ps + bx_;
    Pe.psy0 = ps + 2 * bx_;
    Pe.psy1 = ps + 2 * bx_ + by_;
    Pe.psz0 = ps + 2 * bx_ + 2 * by_;
    Pe.psz1 = ps + 2 * bx_ + 2 * by_ + bz_;
    float *ps2 = ps + 2 * (bx_ + by_ + bz_);
    Ph.psx0 = ps2;
    Ph.psx1 = ps2 + bx_;
    Ph.psy0 = ps2 + 2 * bx_;
    Ph.psy1 = ps2 + 2 * bx_ + by_;
    Ph.psz0 = ps2 + 2 * bx_ + 2 * by_;
    Ph.psz1 = ps2 + 2 * bx_ + 2 * by_ + bz_;
    const int waves = emm::block_threads() / 64;
    Pe.nitems = (int)ni_e;
    Pe.item_info = (const int *)items_d;
    Pe.item_w = (const float *)itemw_d;
    Pe.phase = (const double2 *)m->phase.p;
    Pe.nrecblk = (int)((ni_e + waves - 1) / waves + 7) / 8 * 8;
    Ph.nitems = (int)ni_h;
    Ph.item_info = (const int *)(items_d + items_estep.size() * sizeof(int));
    Ph.item_w = (const float *)(itemw_d + wts_estep.size() * sizeof(float));
    Ph.phase = (const double2 *)m->phase.p + (size_t)nt * nfreq;
    Ph.nrecblk = (int)((ni_h + waves - 1) / waves + 7) / 8 * 8;

    // time loop: per step E step (+ H-channel DTFT) then H step (+ E-channel DTFT)
    const bool prof = m->opt.profile != 0;
    const int ring_pairs = 128;
    if (prof && m->ring.empty()) {
        m->ring.assign(4 * ring_pairs, nullptr);
        for (hipEvent_t &e : m->ring) HIP_OK(m, hipEventCreate(&e));
    }
    if (!m->ev_loop[0]) {
        HIP_OK(m, hipEventCreate(&m->ev_loop[0]));
        HIP_OK(m, hipEventCreate(&m->ev_loop[1]));
    }
    double ems = 0.0, hms = 0.0;
    auto harvest = [&](int slot) -> emm_status {
        float a = 0.f, b = 0.f;
        HIP_OK(m, hipEventSynchronize(m->ring[4 * slot + 3]));
        HIP_OK(m, hipEventElapsedTime(&a, m->ring[4 * slot + 0], m->ring[4 * slot + 1]));
        HIP_OK(m, hipEventElapsedTime(&b, m->ring[4 * slot + 2], m->ring[4 * slot + 3]));
        ems += a;
        hms += b;
        return EMM_OK;
    };
    HIP_OK(m, hipEventRecord(m->ev_loop[0], stream));
    for (int n = 0; n < nt; ++n) {
        const int slot = n % ring_pairs;
        if (prof) {
            if (n >= ring_pairs && (st = harvest(slot)) != EMM_OK) return st;
            HIP_OK(m, hipEventRecord(m->ring[4 * slot + 0], stream));
        }
        emm::launch_e_step(r, Pe, n, stream);
        if (prof) {
            HIP_OK(m, hipEventRecord(m->ring[4 * slot + 1], stream));
            HIP_OK(m, hipEventRecord(m->ring[4 * slot + 2], stream));
        }
        emm::launch_h_step(r, Ph, n, stream);
        if (prof) HIP_OK(m, hipEventRecord(m->ring[4 * slot + 3], stream));
    }
    HIP_OK(m, hipGetLastError());
    HIP_OK(m, hipEventRecord(m->ev_loop[1], stream));
    if (prof)
        for (int n = std::max(0, nt - ring_pairs); n < nt; ++n)
            if ((st = harvest(n % ring_pairs)) != EMM_OK) return st;

    // accumulators back, then Green's functions (Section 2.2):
    // G^EE = (omega/omega') E'/J',  G^HE = H'/J',  J' = moment * S_f
    std::vector<double> acc_h((size_t)nslot * nfreq * (acc_elem / sizeof(double)));
    HIP_OK(m, hipMemcpyAsync(acc_h.data(), m->acc.p, (size_t)nslot * nfreq * acc_elem, hipMemcpyDeviceToHost, stream));
    HIP_OK(m, hipStreamSynchronize(stream));
    float loop_ms = 0.f;
    HIP_OK(m, hipEventElapsedTime(&loop_ms, m->ev_loop[0], m->ev_loop[1]));
    bool nonfinite = false;
    for (int s = 0; s < nsrc; ++s)
        for (int i = 0; i < nrec; ++i)
            for (int c = 0; c < nch; ++c)
                for (int f = 0; f < nfreq; ++f) {
                    const size_t k = ((size_t)(s * nrec + i) * nch + c) * nfreq + f;
                    std::complex<double> a;
                    if (m->opt.dft_mode == 0) {
                        a = {acc_h[2 * k], acc_h[2 * k + 1]};
                    } else {
                        const float *q = reinterpret_cast<const float *>(acc_h.data()) + 4 * k;
                        a = {(double)q[0] - (double)q[1], (double)q[2] - (double)q[3]};
                    }
                    std::complex<double> G = a / (sscale[s] * src[s].moment * Shat[f]);
                    if (chans[c] < 3) G *= (2.0 * kPi * freq_hz[f]) / wp[f];
                    if (!std::isfinite(G.real()) || !std::isfinite(G.imag())) nonfinite = true;
                    green[2 * k] = G.real();
                    green[2 * k + 1] = G.imag();
                }
    m->info.nt = nt;
    m->info.forward_ms = loop_ms;
    m->info.tile_kz = P.kz;
    m->info.e_kernel_ms = prof ? ems : 0.0;
    m->info.h_kernel_ms = prof ? hms : 0.0;
    m->info.e_launches = prof ? nt : 0;
    m->info.h_launches = prof ? nt : 0;
    if (nonfinite) return fail(m, EMM_ERR_NONFINITE, "a DTFT accumulator is not finite (unstable run?)");
    return EMM_OK;
}

}  // extern "C"
