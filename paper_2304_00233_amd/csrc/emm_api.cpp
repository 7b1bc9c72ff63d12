// C ABI of libemm: validation, set-up, device buffers and the time loop.
// Declarations and argument conventions: include/emm.h.
#include "emm.h"
#include "emm_air.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <string>
#include <vector>

#include "emm_adjoint.h"
#include "emm_internal.h"
#include "emm_setup.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr int kFlush = 16;       // steps per FP32 partial sum of the gradient

thread_local std::string g_last_error;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;     // carved from the static workspace: never freed
};

// Static device workspace of emm_forward_noalloc (callers that cannot
// allocate device memory): every per-call buffer of such a forward (fields,
// CPML memories, DTFT accumulators, source, receiver, CPML and phase tables)
// is carved from it.  Each device that loads the library holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
    bool done = false;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;
};
std::mutex g_scratch_mu;
std::map<int, ScratchSlot> g_scratch;

// Once per device, with that device current: the device address of its copy
// of `scratch`.
hipError_t scratch_address(int device, void **ptr) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot &slot = g_scratch[device];
    if (!slot.done) {
        slot.err = hipGetSymbolAddress(&slot.ptr, HIP_SYMBOL(scratch));
        if (slot.err != hipSuccess) slot.ptr = nullptr;
        slot.done = true;
    }
    *ptr = slot.ptr;
    return slot.err;
}

}  // namespace

// Host-side description of the acquisition of the last forward run and the
// kernel parameters built for it.
struct Acq {
    int nsrc = 0, nrec = 0, nch = 0, nf = 0, nt = 0;
    unsigned chan_mask = 0;
    std::vector<emm_source> src;
    std::vector<emm_receiver> rec;
    std::vector<double> freqs;
    std::vector<int> chans;
    std::vector<double> sscale;                     // source amplitude scale
    std::vector<std::complex<double>> Shat, wp;     // source spectrum, omega'
    // receiver items {src, field, bx, by, bz, slot} and their weights wx|wy|wz:
    // H channels are sampled in the E-step launch, E channels in the H-step one
    std::vector<int> items_estep, items_hstep;
    std::vector<float> w_estep, w_hstep;
    emm::StepParams Pe{}, Ph{};
    int ckpt = 0;                                   // checkpoint interval of the stored run (0: none)
    int nslot = 0;                                  // receiver slots (src, rec, chan)
    int ncorner = 0;                                // convergence-check slots after them (8 per source)
    int fmin_index = 0;                             // lowest frequency
    std::vector<float> wavelet;                     // s_n as stepped (FP32)
    bool valid = false;
};

// launch choices the autotuner measured best for one source count
struct Tune {
    int kz = 0;        // z planes per block
    int stream = 0;    // nontemporal hints
    int compact = 0;   // compact dt/eps in the E step
    int tx = 64;       // tile width of the step kernels
    int ry = 1;        // rows per wavefront (2, 4: register-blocked 64-wide tiles)
    int sorder = 0;    // tile order of the sources (0: fastest, 1: slowest)
};

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
    unsigned *cei = nullptr;  // compact dt/eps of the E step: index words
    float *cet = nullptr;     //   and the table of distinct values (nullptr: not built)
    int ncet = 0;
    float *tab[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // cmx cmy cmz cpx cpy cpz
    // forward-lifetime device data (grown on demand, kept between forwards)
    DevBuf fields, psi, acc, cpml, srcinfo, srcq, wav, items, itemw, phase;
    DevBuf fieldsB, psiB;                           // second buffers of the fused step (ping-pong)
    DevBuf ckpts;                                   // full-state checkpoints of the last run
    DevBuf ickpts;                                  // inner checkpoints of one outer segment
    DevBuf stepdev;                                 // device step counter of graph replays
    // adjoint: Et|Hb fields, Q (12 slab arrays), T (6), E snapshots, per-source
    // gradients, transposed tables, injection lists and coefficients
    DevBuf adjf, adjq, adjt, snaps, grad, grad32, tabT, inj, injA, adjcpml;
    DevBuf gsum;                                    // dL/dlog sigma on the input cells, summed over sources
    // receiver injection lists of the last emm_gradient (CSR over target
    // cells, in m->inj), kept while the acquisition's receiver items, the
    // source count and the layout stay the same: building them sorts
    // (2r)^3 entries per item (~5 M for 8 sources x 400 receivers x 3
    // channels at 8th order, ~0.4 s)
    struct InjCache {
        bool valid = false;
        std::vector<int> items_e, items_h;
        std::vector<float> w_e, w_h;
        int nsrc = 0;
        long long fstride = 0;
        void *base = nullptr;
        int ncells[2] = {0, 0};
        const void *ptr[12] = {};
    } injc;
    Acq acq;
    std::map<int, Tune> tuned;                      // autotuned launch choices per source count
    std::unique_ptr<emm::AirBoundary> air;          // ghost planes above the surface (airwave)
    hipEvent_t ev_loop[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ring;       // profiling: start/end pairs
    // static workspace of emm_forward_noalloc on this model's device
    void *scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    // set only during emm_forward_noalloc: ensure() carves from here
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    emm_info info{};
    std::string err;
};

namespace {

emm_status fail(emm_model *m, emm_status s, const std::string &msg) {
    g_last_error = msg;
    if (m) m->err = msg;
    return s;
}

// HIP failures: out of memory maps to EMM_ERR_OOM, everything else to DEVICE
emm_status hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? EMM_ERR_OOM : EMM_ERR_DEVICE; }

#define HIP_OK(m, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((m), hip_status(e_), std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

emm_status ensure(emm_model *m, DevBuf &b, size_t bytes) {
    if (m->arena) {
        // no-alloc call: the next 256-byte aligned piece of the static workspace
        const size_t need = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        if (m->arena_used + need > m->arena_cap)
            return fail(m, EMM_ERR_OOM, "the forward needs more than the " + std::to_string(m->arena_cap) +
                                            "-byte static workspace of emm_forward_noalloc (" +
                                            std::to_string(m->arena_used + need) + " bytes so far)");
        b.p = m->arena + m->arena_used;
        b.bytes = bytes;
        b.borrowed = true;
        m->arena_used += need;
        return EMM_OK;
    }
    if (b.bytes >= bytes && b.p && !b.borrowed) return EMM_OK;
    if (b.p && b.borrowed) {
        b.p = nullptr;
        b.bytes = 0;
        b.borrowed = false;
    }
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

// Owns a captured graph and its executable; destroys them on every exit path.
struct GraphHold {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphHold() = default;
    GraphHold(const GraphHold &) = delete;
    GraphHold &operator=(const GraphHold &) = delete;
    ~GraphHold() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

bool finite_increasing(const double *x, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x[i]) || (i && !(x[i] > x[i - 1]))) return false;
    return true;
}

// Algorithmic bytes of one step for one source: E step reads H1..3, E1..3,
// ce1..3 and writes E1..3 (48 B/cell); H step reads E1..3, H1..3 and writes
// H1..3 (36 B/cell); each CPML slab cell reads and writes two memory
// variables per axis per half step (16 B).
// E step: E read + written, H read, dt/eps read (3 FP32 arrays, or one
// index word in the compact form); H step: H read + written, E read
void step_bytes(const emm_model *m, double &eb, double &hb, bool compact) {
    const double N = double(m->np[0]) * m->np[1] * m->np[2];
    double ncpml = 0.0;
    if (m->nb > 0)
        for (int a = 0; a < 3; ++a) ncpml += 2.0 * m->nb * N / m->np[a];
    eb = (compact ? 40.0 : 48.0) * N + 16.0 * ncpml;
    hb = 36.0 * N + 16.0 * ncpml;
}

// first updated z plane: r, or the surface node when air sits above it
int kmin_of(const emm_model *m) { return m->opt.airwave ? m->nbe : m->r; }
// z planes of the update set
int z_planes(const emm_model *m) { return m->np[2] - m->r - kmin_of(m); }

int choose_kz(const emm_model *m, int xt, int yt, int nsrc) {
    const int nzv = z_planes(m);
    if (m->opt.tile_kz > 0) return std::min(m->opt.tile_kz, nzv);
    if (m->opt.tile_kz < 0) {
        auto it = m->tuned.find(nsrc);
        if (it != m->tuned.end()) return it->second.kz;
    }
    const long long per_chunk = (long long)xt * yt * nsrc;
    long long zc = std::max<long long>(1, (4096 + per_chunk - 1) / per_chunk);
    zc = std::min<long long>(zc, std::max(1, nzv / 8));
    return (int)((nzv + zc - 1) / zc);
}

// Nontemporal hints when the arrays one step touches (fields of all sources
// and dt/eps) exceed 160 MiB, well inside the 256 MB Infinity Cache below
// that; the autotuner overrides this with a measurement.
int choose_stream(const emm_model *m, long long fstride, int nsrc) {
    if (m->opt.nontemporal >= 0) return m->opt.nontemporal;
    if (m->opt.tile_kz < 0) {
        auto it = m->tuned.find(nsrc);
        if (it != m->tuned.end()) return it->second.stream;
    }
    const double resident = (6.0 * nsrc + 3.0) * (double)fstride * sizeof(float);
    return resident > 160.0 * (1 << 20) ? 1 : 0;
}

// Compact dt/eps whenever the model has it (8 of the E step's 48 B per
// cell less; measured faster on grids in and beyond the Infinity Cache),
// unless the autotuner measured the FP32 arrays faster.
int choose_compact(const emm_model *m, int nsrc) {
    if (!m->cei || m->opt.ce_table == 0) return 0;
    if (m->opt.ce_table == -1 && m->opt.tile_kz < 0) {
        auto it = m->tuned.find(nsrc);
        if (it != m->tuned.end()) return it->second.compact;
    }
    return 1;
}

// Tile width of the step kernels (64 x 4 or 32 x 8 columns): the option,
// the autotuner's choice, else 32 where it leaves clearly fewer idle lanes
// in the last x tile of a row, or at r >= 3 (less y halo per cell).
int choose_tx(const emm_model *m, int nsrc) {
    if (m->opt.tile_x > 0) return m->opt.tile_x;
    if (m->opt.tile_kz < 0) {
        auto it = m->tuned.find(nsrc);
        if (it != m->tuned.end()) return it->second.tx;
    }
    const int valid = m->np[0] - 2 * m->r;
    auto lanes = [&](int w) { return (m->np[0] - m->r + w - 1) / w * w; };
    const double e64 = (double)valid / lanes(64), e32 = (double)valid / lanes(32);
    return (m->r >= 3 || e32 > e64 + 0.02) ? 32 : 64;
}

// Tile order of the sources: the option, the autotuner's choice, else
// source fastest.
int choose_sorder(const emm_model *m, int nsrc) {
    if (m->opt.src_order >= 0) return m->opt.src_order;
    if (m->opt.tile_kz < 0) {
        auto it = m->tuned.find(nsrc);
        if (it != m->tuned.end()) return it->second.sorder;
    }
    return 0;
}

// Rows per wavefront of the step kernels: the option, the autotuner's
// choice, else 1 (one row per wavefront, step_kernel).
int choose_ry(const emm_model *m, int nsrc) {
    if (m->opt.tile_rows > 0) return m->opt.tile_rows;
    if (m->opt.tile_kz < 0) {
        auto it = m->tuned.find(nsrc);
        if (it != m->tuned.end()) return it->second.ry;
    }
    return 1;
}

// x and y tiles over the update set i, j in [r, n - 1 - r] (x tiles start at 0);
// ry > 1: 64-wide tiles of 4 ry rows (register-blocked kernels)
void set_tiles(emm::StepParams &P, const emm_model *m, int tx, int ry = 1) {
    if (ry > 1) tx = 64;
    const int rows = ry > 1 ? (emm::kStepThreads / 64) * ry : emm::kStepThreads / tx;
    P.tx = tx;
    P.ry = ry > 1 ? ry : 1;
    P.xt = (m->np[0] - m->r + tx - 1) / tx;
    P.yt = (m->np[1] - 2 * m->r + rows - 1) / rows;
}

// launch choices of the last run, and the E step's bytes that follow from them
void note_run(emm_model *m, const emm::StepParams &Pe) {
    m->info.tile_kz = Pe.kz;
    m->info.tile_x = Pe.tx;
    m->info.tile_rows = Pe.ry;
    m->info.src_order = Pe.sorder;
    m->info.air_transform = m->air ? (m->air->direct() ? 2 : 1) : 0;
    m->info.nontemporal = Pe.stream;
    m->info.ce_table = Pe.cei != nullptr;
    step_bytes(m, m->info.e_bytes, m->info.h_bytes, Pe.cei != nullptr);
    m->info.bytes_per_step = m->info.e_bytes + m->info.h_bytes;
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
    o->checkpoint_every = 0;
    o->graph_steps = 0;
    o->checkpoint_inner = 0;
    o->nontemporal = -1;
    o->converge_tol = 0.0;
    o->converge_every = 100;
    o->ce_table = -1;
    o->src_group = 0;
    o->tile_x = 0;
    o->tile_rows = 0;
    o->src_order = -1;
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
    if (m->cei) (void)hipFree(m->cei);
    if (m->cet) (void)hipFree(m->cet);
    for (float *p : m->tab) if (p) (void)hipFree(p);
    for (DevBuf *b : {&m->fields, &m->psi, &m->acc, &m->cpml, &m->srcinfo, &m->srcq, &m->wav,
                      &m->items, &m->itemw, &m->phase, &m->fieldsB, &m->psiB, &m->ckpts, &m->ickpts, &m->adjf, &m->adjq, &m->adjt,
                      &m->snaps, &m->grad, &m->grad32, &m->tabT, &m->inj, &m->injA, &m->adjcpml, &m->stepdev})
        if (b->p && !b->borrowed) (void)hipFree(b->p);
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
    if (opt.nt < 0 || opt.dft_mode < 0 || opt.dft_mode > 1 || opt.tile_kz < -1 || opt.checkpoint_every < 0 || opt.graph_steps < 0 ||
        opt.checkpoint_inner < 0 || opt.nontemporal < -1 || opt.nontemporal > 1 ||
        opt.airwave < 0 || opt.airwave > 3 || !(opt.converge_tol >= 0.0) || opt.converge_every < 1 ||
        opt.fused < 0 || opt.fused > 1 || opt.ce_table < -1 || opt.ce_table > 1 || opt.src_group < -1 || (opt.tile_x != 0 && opt.tile_x != 32 && opt.tile_x != 64) ||
        (opt.tile_rows != 0 && opt.tile_rows != 1 && opt.tile_rows != 2 && opt.tile_rows != 4) ||
        (opt.tile_rows > 1 && opt.tile_x == 32) || opt.src_order < -1 || opt.src_order > 1 ||
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
    if (opt.airwave) {
        // the FFTs of the air boundary need uniform x and y spacing, and the
        // ghost planes must fit above the surface node
        for (int a = 0; a < 2; ++a) {
            const double d0 = xs[a][1] - xs[a][0];
            for (int i = 1; i < nd[a]; ++i)
                if (std::fabs((xs[a][i] - xs[a][i - 1]) - d0) > 1e-9 * std::fabs(d0))
                    return fail(nullptr, EMM_ERR_GRID, "the air boundary needs uniform x and y spacing");
        }
        if (opt.nb + opt.ne < opt.rd)
            return fail(nullptr, EMM_ERR_GRID, "the air boundary needs nb + ne >= rd planes above the surface");
    }
    {
        // the kernels address one source's field array with 32-bit offsets:
        // (n1 + 2 nbe, rounded up to 64) (n2 + 2 nbe) (n3 + 2 nbe) < 2^31
        const long long nbe2 = 2LL * (opt.nb + opt.ne);
        const long long pitch = (nd[0] + nbe2 + emm::kTileX - 1) / emm::kTileX * emm::kTileX;
        if (pitch * (nd[1] + nbe2) * (nd[2] + nbe2) > (long long)INT32_MAX)
            return fail(nullptr, EMM_ERR_GRID, "padded grid has more than 2^31 - 1 cells per field array "
                                               "(x rows padded to a multiple of 64)");
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
    {
        hipError_t e = hipGetDevice(&m->device);
        if (e == hipSuccess) e = hipStreamCreate(&m->own_stream);
        // set-up of the static workspace of emm_forward_noalloc on this device
        // (a failure is reported by that call, not here)
        if (e == hipSuccess) m->scratch_err = scratch_address(m->device, &m->scratch);
        if (e != hipSuccess) {
            emm_status s = fail(nullptr, EMM_ERR_DEVICE, std::string("device set-up: ") + hipGetErrorString(e));
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
    // compact form for the E step: the distinct FP32 values of the three
    // components (at most kCeTable) and per cell their indices, one byte per
    // component
    std::vector<unsigned> cidx;
    std::vector<float> ctab;
    std::unordered_map<uint32_t, unsigned> code;
    if (opt.ce_table != 0) cidx.assign(N, 0u);
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
        if (!cidx.empty()) {
            // cells past n1pad in a row (pitch padding) are never updated: index 0
            uint32_t last_bits = 0;
            unsigned last = 0;
            bool have_last = false;
            for (int k = 0; k < m->np[2] && !cidx.empty(); ++k)
                for (int j = 0; j < m->np[1] && !cidx.empty(); ++j) {
                    const long long row = ((long long)k * m->np[1] + j) * m->pitch;
                    for (int i = 0; i < m->np[0]; ++i) {
                        uint32_t bits;
                        std::memcpy(&bits, &buf[row + i], 4);
                        if (!have_last || bits != last_bits) {
                            auto it = code.find(bits);
                            if (it == code.end()) {
                                if ((int)code.size() == emm::kCeTable) {
                                    cidx.clear();    // too many values: FP32 arrays
                                    break;
                                }
                                ctab.push_back(buf[row + i]);
                                it = code.emplace(bits, (unsigned)code.size()).first;
                            }
                            last_bits = bits;
                            last = it->second;
                            have_last = true;
                        }
                        cidx[row + i] |= last << (8 * c3);
                    }
                }
        }
        hipError_t e = hipMalloc(&m->ce[c3], N * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(m->ce[c3], buf.data(), N * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            emm_status s = fail(nullptr, hip_status(e), std::string("ce upload: ") + hipGetErrorString(e));
            emm_destroy(m);
            return s;
        }
    }
    if (!cidx.empty()) {
        hipError_t e = hipMalloc(&m->cei, N * sizeof(unsigned));
        if (e == hipSuccess) e = hipMemcpy(m->cei, cidx.data(), N * sizeof(unsigned), hipMemcpyHostToDevice);
        m->ncet = (int)ctab.size();
        if (e == hipSuccess) e = hipMalloc(&m->cet, ctab.size() * sizeof(float));
        if (e == hipSuccess)
            e = hipMemcpy(m->cet, ctab.data(), ctab.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            emm_status s = fail(nullptr, hip_status(e), std::string("ce table upload: ") + hipGetErrorString(e));
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
            emm_status s = fail(nullptr, hip_status(e), std::string("table upload: ") + hipGetErrorString(e));
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
    step_bytes(m, m->info.e_bytes, m->info.h_bytes, false);   // until a run chooses
    m->info.bytes_per_step = m->info.e_bytes + m->info.h_bytes;
    // fused step: E, H and dt/eps (FP32 arrays) read once, E and H written
    // once (60 B/cell) plus the same CPML memory traffic as the two half steps
    double eb32 = 0.0, hb32 = 0.0;
    step_bytes(m, eb32, hb32, false);
    m->info.leap_bytes = eb32 + hb32 - 24.0 * (double)m->np[0] * m->np[1] * m->np[2];
    *out = m;
    return EMM_OK;
}

}  // extern "C"

namespace {

// staggering (half along x, y, z) of Ex, Ey, Ez, Hx, Hy, Hz
const int kStag[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

bool same_acquisition(const Acq &a, const emm_source *src, int nsrc, const emm_receiver *rec,
                      int nrec, unsigned chan_mask, const double *freq, int nfreq) {
    if (!a.valid || a.nsrc != nsrc || a.nrec != nrec || a.chan_mask != chan_mask || a.nf != nfreq)
        return false;
    for (int s = 0; s < nsrc; ++s)
        if (a.src[s].x != src[s].x || a.src[s].y != src[s].y || a.src[s].z != src[s].z ||
            a.src[s].comp != src[s].comp || a.src[s].moment != src[s].moment)
            return false;
    for (int i = 0; i < nrec; ++i)
        if (a.rec[i].x != rec[i].x || a.rec[i].y != rec[i].y || a.rec[i].z != rec[i].z) return false;
    for (int f = 0; f < nfreq; ++f)
        if (a.freqs[f] != freq[f]) return false;
    return true;
}

// Validate the acquisition, build the host tables (stencils, wavelet, DTFT
// phases, CPML), upload them and fill the kernel parameters (Sections 3.1,
// 3.4, 3.5; see emm_forward in emm.h).
// Time steps of a forward: the option, else (Section 3.5) the wavelet's
// duration plus the time for the lowest frequency's damped mode to decay by
// 1e6, rounded up to a multiple of 100.  Frequencies must be valid.
int steps_for(const emm_model *m, const double *freq_hz, int nfreq) {
    if (m->opt.nt > 0) return m->opt.nt;
    double fmax = 0.0, fmin = 1e300;
    for (int f = 0; f < nfreq; ++f) {
        fmax = std::max(fmax, freq_hz[f]);
        fmin = std::min(fmin, freq_hz[f]);
    }
    const double fp = m->opt.wavelet_fpeak > 0.0 ? m->opt.wavelet_fpeak : 2.0 * std::sqrt(fmax * m->opt.f0);
    const double tau = 1.0 / (kPi * fp);
    const double decay = emm::omega_prime(fmin, m->omega0).imag();
    const double T = 7.0 * tau + std::log(1e6) / decay;
    return (int)(std::ceil(T / m->dt / 100.0) * 100.0);
}

// A source's component, moment and position: its (2r)^3 stencil on the grid
// of its E component must lie inside the interior.
emm_status check_source(emm_model *m, const emm_source &S) {
    if (S.comp < 0 || S.comp > 2 || !std::isfinite(S.moment) || S.moment == 0.0 || !std::isfinite(S.x) ||
        !std::isfinite(S.y) || !std::isfinite(S.z))
        return fail(m, EMM_ERR_ARG, "source component must be 0..2 with a finite non-zero moment");
    const double p[3] = {S.x, S.y, S.z};
    const int L = 2 * m->r;
    for (int a = 0; a < 3; ++a) {
        double w[2 * emm::kMaxR];
        const int base = emm::point_stencil(a == S.comp ? m->half[a] : m->axes[a], p[a], m->r, w);
        if (!(base >= m->nbe && base + L - 1 <= m->np[a] - 1 - m->nbe))
            return fail(m, EMM_ERR_GEOMETRY, "source stencil leaves the interior");
    }
    return EMM_OK;
}

// bytes of one source's full time-stepping state (fields + CPML memories)
size_t state_floats(const emm_model *m) {
    const long long plane = (long long)m->pitch * m->np[1];
    const long long fstride = plane * m->np[2];
    const int nb = m->nb;
    const long long psxs = nb ? (long long)m->np[2] * m->np[1] * 2 * nb : 0;
    const long long psys = nb ? (long long)m->np[2] * 2 * nb * m->pitch : 0;
    const long long pszs = nb ? (long long)2 * nb * plane : 0;
    return (size_t)(6 * fstride + 4 * (psxs + psys + pszs));
}

// Sources per time loop of emm_forward: the src_group option, else (0) as
// many as keep the arrays of one step within 160 MiB, so that they stay in
// the 256 MB Infinity Cache from step to step (batching sources on such a
// grid measured slower than one source after another), or all of them when
// one source alone does not fit.
int source_group(const emm_model *m, int nsrc) {
    if (m->opt.src_group > 0) return std::min(m->opt.src_group, nsrc);
    if (m->opt.src_group < 0) return nsrc;
    const double budget = 160.0 * (1 << 20);
    const double per = 4.0 * (double)state_floats(m);
    const double shared = (double)m->pitch * m->np[1] * m->np[2] * (choose_compact(m, nsrc) ? 4.0 : 12.0);
    if (per + shared > budget) return nsrc;
    return std::max(1, std::min(nsrc, (int)((budget - shared) / per)));
}

emm_status prepare(emm_model *m, const emm_source *src, int nsrc, const emm_receiver *rec, int nrec,
                   unsigned chan_mask, const double *freq_hz, int nfreq, hipStream_t stream) {
    Acq &A = m->acq;
    A.valid = false;
    A.ckpt = 0;
    if (!src || !rec || nsrc < 1 || nrec < 1 || chan_mask == 0 || (chan_mask & ~0x3Fu))
        return fail(m, EMM_ERR_ARG, "bad sources, receivers or channel mask");
    if (!freq_hz || nfreq < 1) return fail(m, EMM_ERR_FREQ, "need at least one frequency");
    for (int f = 0; f < nfreq; ++f)
        if (!(freq_hz[f] > 0.0) || !std::isfinite(freq_hz[f]))
            return fail(m, EMM_ERR_FREQ, "frequencies must be finite and > 0");
    const int r = m->r, L = 2 * r, L3 = L * L * L;
    A.chans.clear();
    for (int c = 0; c < 6; ++c)
        if (chan_mask >> c & 1u) A.chans.push_back(c);
    const int nch = (int)A.chans.size();
    auto coords = [&](int a, int h) -> const std::vector<double> & { return h ? m->half[a] : m->axes[a]; };
    auto inside = [&](int a, int base) { return base >= m->nbe && base + L - 1 <= m->np[a] - 1 - m->nbe; };

    // sources: (2r)^3 stencil on the E_comp grid, J = moment w / V, scaled to max |q| = 1
    std::vector<int> sinfo(4 * nsrc);
    std::vector<float> sq((size_t)nsrc * L3);
    A.sscale.assign(nsrc, 1.0);
    for (int s = 0; s < nsrc; ++s) {
        const emm_source &S = src[s];
        emm_status cs = check_source(m, S);
        if (cs != EMM_OK) return cs;
        const double p[3] = {S.x, S.y, S.z};
        double w[3][2 * emm::kMaxR];
        int base[3];
        for (int a = 0; a < 3; ++a) base[a] = emm::point_stencil(coords(a, a == S.comp), p[a], r, w[a]);
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
        A.sscale[s] = 1.0 / qmax;
        for (int q = 0; q < L3; ++q) sq[(size_t)s * L3 + q] = (float)(qd[q] * A.sscale[s]);
        sinfo[4 * s] = S.comp;
        sinfo[4 * s + 1] = base[0];
        sinfo[4 * s + 2] = base[1];
        sinfo[4 * s + 3] = base[2];
    }
    // receiver items: E channels in the H-step launch, H channels in the E-step launch
    A.items_estep.clear();
    A.items_hstep.clear();
    A.w_estep.clear();
    A.w_hstep.clear();
    for (int i = 0; i < nrec; ++i) {
        const double p[3] = {rec[i].x, rec[i].y, rec[i].z};
        if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]))
            return fail(m, EMM_ERR_ARG, "receiver position not finite");
        for (int c = 0; c < nch; ++c) {
            const int ch = A.chans[c];
            double w[3][2 * emm::kMaxR];
            int base[3];
            for (int a = 0; a < 3; ++a) {
                base[a] = emm::point_stencil(coords(a, kStag[ch][a]), p[a], r, w[a]);
                if (!inside(a, base[a])) return fail(m, EMM_ERR_GEOMETRY, "receiver stencil leaves the interior");
            }
            std::vector<int> &inf = ch < 3 ? A.items_hstep : A.items_estep;
            std::vector<float> &wv = ch < 3 ? A.w_hstep : A.w_estep;
            for (int s = 0; s < nsrc; ++s) {
                const int slot = (s * nrec + i) * nch + c;
                inf.insert(inf.end(), {s, ch % 3, base[0], base[1], base[2], slot});
                for (int a = 0; a < 3; ++a)
                    for (int q = 0; q < L; ++q) wv.push_back((float)w[a][q]);
            }
        }
    }

    // convergence check: E1 exactly at the 8 corner nodes of the interior
    // (first and last interior index per axis; the top ones are the surface
    // nodes under air), one slot each per source after the receiver slots
    A.nslot = nsrc * nrec * nch;
    A.ncorner = m->opt.converge_tol > 0.0 ? 8 * nsrc : 0;
    if (A.ncorner) {
        const int lo[3] = {m->nbe, m->nbe, m->nbe};
        const int hi[3] = {m->np[0] - 2 - m->nbe, m->np[1] - 1 - m->nbe, m->np[2] - 1 - m->nbe};
        for (int s = 0; s < nsrc; ++s)
            for (int c = 0; c < 8; ++c) {
                int base[3];
                float w[3][2 * emm::kMaxR] = {};
                for (int a = 0; a < 3; ++a) {
                    const int idx = (c >> a & 1) ? hi[a] : lo[a];
                    const int q = idx + L - 1 <= m->np[a] - 1 ? 0 : L - 1;   // keep the stencil in the array
                    base[a] = idx - q;
                    w[a][q] = 1.f;
                }
                A.items_hstep.insert(A.items_hstep.end(), {s, 0, base[0], base[1], base[2], A.nslot + 8 * s + c});
                for (int a = 0; a < 3; ++a)
                    for (int q = 0; q < L; ++q) A.w_hstep.push_back(w[a][q]);
            }
    }

    // time axis, wavelet, DTFT phases, CPML
    double fmax = 0.0, fmin = 1e300;
    for (int f = 0; f < nfreq; ++f) {
        fmax = std::max(fmax, freq_hz[f]);
        if (freq_hz[f] < fmin) A.fmin_index = f;
        fmin = std::min(fmin, freq_hz[f]);
    }
    const double fp = m->opt.wavelet_fpeak > 0.0 ? m->opt.wavelet_fpeak : 2.0 * std::sqrt(fmax * m->opt.f0);
    const int nt = steps_for(m, freq_hz, nfreq);
    const std::vector<double> sw = emm::wavelet(nt, m->dt, fp);
    std::vector<float> swf(sw.begin(), sw.end());
    A.wavelet = swf;
    A.Shat.assign(nfreq, 0.0);
    A.wp.assign(nfreq, 0.0);
    std::vector<double2> ph((size_t)2 * nt * nfreq);   // [0]: E-step (H stamps), [1]: H-step (E stamps)
    for (int f = 0; f < nfreq; ++f) {
        A.wp[f] = emm::omega_prime(freq_hz[f], m->omega0);
        for (int n = 0; n < nt; ++n) {
            const std::complex<double> zh = std::exp(std::complex<double>(0, 1) * A.wp[f] * ((n + 0.5) * m->dt));
            const std::complex<double> ze = std::exp(std::complex<double>(0, 1) * A.wp[f] * ((n + 1.0) * m->dt));
            A.Shat[f] += (double)swf[n] * zh;
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
    const long long plane = (long long)m->pitch * m->np[1];
    const long long fstride = plane * m->np[2];
    const int nb = m->nb;
    const long long psxs = nb ? (long long)m->np[2] * m->np[1] * 2 * nb : 0;
    const long long psys = nb ? (long long)m->np[2] * 2 * nb * m->pitch : 0;
    const long long pszs = nb ? (long long)2 * nb * plane : 0;
    const long long ps_per_src = 4 * (psxs + psys + pszs);      // 2 per axis per half step
    const int nslot = A.nslot + A.ncorner;
    if ((st = ensure(m, m->fields, (size_t)6 * nsrc * fstride * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->psi, (size_t)std::max<long long>(1, nsrc * ps_per_src) * sizeof(float))) != EMM_OK) return st;
    const size_t acc_elem = m->opt.dft_mode ? sizeof(float4) : sizeof(double2);
    if ((st = ensure(m, m->acc, (size_t)nslot * nfreq * acc_elem)) != EMM_OK) return st;
    if ((st = ensure(m, m->cpml, cpml.size() * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->srcinfo, sinfo.size() * sizeof(int))) != EMM_OK) return st;
    if ((st = ensure(m, m->srcq, sq.size() * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->wav, swf.size() * sizeof(float))) != EMM_OK) return st;
    const size_t ni_e = A.items_estep.size() / 6, ni_h = A.items_hstep.size() / 6;
    if ((st = ensure(m, m->items, (A.items_estep.size() + A.items_hstep.size()) * sizeof(int))) != EMM_OK) return st;
    if ((st = ensure(m, m->itemw, (A.w_estep.size() + A.w_hstep.size()) * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->phase, ph.size() * sizeof(double2))) != EMM_OK) return st;

    char *items_d = (char *)m->items.p;
    char *itemw_d = (char *)m->itemw.p;
    HIP_OK(m, hipMemcpyAsync(m->cpml.p, cpml.data(), cpml.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->srcinfo.p, sinfo.data(), sinfo.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->srcq.p, sq.data(), sq.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->wav.p, swf.data(), swf.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    if (!A.items_estep.empty())
        HIP_OK(m, hipMemcpyAsync(items_d, A.items_estep.data(), A.items_estep.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (!A.items_hstep.empty())
        HIP_OK(m, hipMemcpyAsync(items_d + A.items_estep.size() * sizeof(int), A.items_hstep.data(),
                                 A.items_hstep.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (!A.w_estep.empty())
        HIP_OK(m, hipMemcpyAsync(itemw_d, A.w_estep.data(), A.w_estep.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    if (!A.w_hstep.empty())
        HIP_OK(m, hipMemcpyAsync(itemw_d + A.w_estep.size() * sizeof(float), A.w_hstep.data(),
                                 A.w_hstep.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_OK(m, hipMemcpyAsync(m->phase.p, ph.data(), ph.size() * sizeof(double2), hipMemcpyHostToDevice, stream));
    // the host vectors above die with this call: wait for the copies
    HIP_OK(m, hipStreamSynchronize(stream));

    // kernel parameters
    emm::StepParams P{};
    P.n1 = m->np[0];
    P.n2 = m->np[1];
    P.n3 = m->np[2];
    P.pitch = m->pitch;
    P.plane = plane;
    P.fstride = fstride;
    P.nb = nb;
    set_tiles(P, m, choose_tx(m, nsrc), choose_ry(m, nsrc));
    P.kz = choose_kz(m, P.xt, P.yt, nsrc);
    P.zc = (z_planes(m) + P.kz - 1) / P.kz;
    P.kmin = kmin_of(m);
    P.nsrc = nsrc;
    P.nstencil = P.xt * P.yt * P.zc * nsrc;
    P.sorder = choose_sorder(m, nsrc);
    P.stream = choose_stream(m, fstride, nsrc);
    float *F = (float *)m->fields.p;
    // per-source field arrays are laid out [comp][src][...]: source s at + s * fstride
    P.E1 = F;
    P.E2 = F + (size_t)nsrc * fstride;
    P.E3 = F + (size_t)2 * nsrc * fstride;
    P.H1 = F + (size_t)3 * nsrc * fstride;
    P.H2 = F + (size_t)4 * nsrc * fstride;
    P.H3 = F + (size_t)5 * nsrc * fstride;
    P.Eo1 = P.E1;
    P.Eo2 = P.E2;
    P.Eo3 = P.E3;
    P.ce1 = m->ce[0];
    P.ce2 = m->ce[1];
    P.ce3 = m->ce[2];
    P.cei = choose_compact(m, nsrc) ? m->cei : nullptr;
    P.cet = m->cet;
    P.ncet = m->ncet;
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
    Ph.item_info = (const int *)(items_d + A.items_estep.size() * sizeof(int));
    Ph.item_w = (const float *)(itemw_d + A.w_estep.size() * sizeof(float));
    Ph.phase = (const double2 *)m->phase.p + (size_t)nt * nfreq;
    Ph.nrecblk = (int)((ni_h + waves - 1) / waves + 7) / 8 * 8;
    A.Pe = Pe;
    A.Ph = Ph;
    A.nsrc = nsrc;
    A.nrec = nrec;
    A.nch = nch;
    A.nf = nfreq;
    A.nt = nt;
    A.chan_mask = chan_mask;
    A.src.assign(src, src + nsrc);
    A.rec.assign(rec, rec + nrec);
    A.freqs.assign(freq_hz, freq_hz + nfreq);
    if (m->opt.airwave && (!m->air || m->air->spec().nsrc != nsrc)) {
        // ghost-plane FFT plans and spectral tables of the air boundary
        emm::AirSpec as;
        as.n1 = m->np[0];
        as.n2 = m->np[1];
        as.n3 = m->np[2];
        as.pitch = m->pitch;
        as.ks = m->nbe;
        as.r = r;
        as.nsrc = nsrc;
        as.plane = plane;
        as.fstride = fstride;
        as.dx = m->axes[0][1] - m->axes[0][0];
        as.dy = m->axes[1][1] - m->axes[1][0];
        const std::vector<double> &z = m->axes[2];
        for (int q = 1; q < r; ++q) as.hE.push_back(z[as.ks] - z[as.ks - q]);
        for (int q = 1; q <= r; ++q) as.hH.push_back(z[as.ks] - 0.5 * (z[as.ks - q] + z[as.ks - q + 1]));
        as.method = m->opt.airwave - 1;
        m->air.reset();
        auto air = std::make_unique<emm::AirBoundary>();
        std::string err;
        if (!air->init(as, err)) return fail(m, EMM_ERR_DEVICE, err);
        m->air = std::move(air);
    }
    A.valid = true;
    return EMM_OK;
}

emm_status autotune(emm_model *m, hipStream_t stream);


// Checkpoint c of buffer `base` <-> live state copies (fields and CPML
// memories of all sources).
emm_status copy_state(emm_model *m, void *base, int c, bool save, hipStream_t stream) {
    const Acq &A = m->acq;
    const size_t ff = (size_t)6 * A.nsrc * A.Pe.fstride * sizeof(float);
    const size_t pf = state_floats(m) * A.nsrc * sizeof(float) - ff;
    char *ck = (char *)base + (size_t)c * (ff + pf);
    if (save) {
        HIP_OK(m, hipMemcpyAsync(ck, m->fields.p, ff, hipMemcpyDeviceToDevice, stream));
        if (pf) HIP_OK(m, hipMemcpyAsync(ck + ff, m->psi.p, pf, hipMemcpyDeviceToDevice, stream));
    } else {
        HIP_OK(m, hipMemcpyAsync(m->fields.p, ck, ff, hipMemcpyDeviceToDevice, stream));
        if (pf) HIP_OK(m, hipMemcpyAsync(m->psi.p, ck + ff, pf, hipMemcpyDeviceToDevice, stream));
    }
    return EMM_OK;
}

// Device bytes of the reverse sweep's checkpoints and E snapshots for outer
// interval c1 and inner interval c2 (c2 >= c1: one level), with S bytes per
// full state and F bytes per E snapshot (all sources).
size_t ckpt_memory(int nt, int c1, int c2, size_t S, size_t F) {
    const size_t outer = (size_t)((nt + c1 - 1) / c1) * S;
    if (c2 >= c1) return outer + (size_t)(c1 + 1) * F;
    return outer + (size_t)((c1 + c2 - 1) / c2) * S + (size_t)(c2 + 1) * F;
}

// Checkpoint schedule within `budget` bytes.  Given intervals (> 0) are
// kept.  Otherwise: the one-level interval of least memory, preferring a
// multiple of the graph length K (the forward then replays graphs); if none
// fits, the two-level pair of least memory.  false: nothing fits.
bool plan_checkpoints(int nt, int K, int c1_fix, int c2_fix, size_t S, size_t F, size_t budget,
                      int &c1, int &c2) {
    auto better = [](size_t mem, size_t &best_mem) {
        if (mem < best_mem) {
            best_mem = mem;
            return true;
        }
        return false;
    };
    if (c1_fix > 0 && c2_fix > 0) {
        c1 = c1_fix;
        c2 = std::min(c2_fix, c1_fix);
        return true;
    }
    if (c1_fix > 0) {                                  // inner interval only
        c1 = c2 = c1_fix;
        if (ckpt_memory(nt, c1, c1, S, F) <= budget) return true;
        size_t best = SIZE_MAX;
        for (int b = 1; b < c1_fix; ++b)
            if (better(ckpt_memory(nt, c1, b, S, F), best)) c2 = b;
        return best <= budget;
    }
    if (c2_fix > 0 && c2_fix < nt) {                   // outer interval for a given inner one
        size_t best = SIZE_MAX;
        c2 = c2_fix;
        c1 = nt;
        for (int a = 2 * c2_fix; a < nt + c2_fix; a += c2_fix)
            if (better(ckpt_memory(nt, a, c2_fix, S, F), best)) c1 = a;
        return best <= budget;
    }
    size_t best_k = SIZE_MAX, best_any = SIZE_MAX;
    int ck = 0, ca = 1;
    for (int c = 1; c <= nt; ++c) {
        const size_t mem = ckpt_memory(nt, c, c, S, F);
        if (K > 0 && c % K == 0 && better(mem, best_k)) ck = c;
        if (better(mem, best_any)) ca = c;
    }
    if (best_k <= budget) {
        c1 = c2 = ck;
        return true;
    }
    if (best_any <= budget) {
        c1 = c2 = ca;
        return true;
    }
    size_t best = SIZE_MAX;
    c1 = c2 = ca;
    for (int b = 1; b <= std::min(nt, 4096); ++b)
        for (int a = 2 * b; a < nt + b; a += b)
            if (better(ckpt_memory(nt, a, b, S, F), best)) {
                c1 = a;
                c2 = b;
            }
    return best <= budget;
}

// Zero fields, CPML memories and DTFT accumulators of all sources.
emm_status zero_state(emm_model *m, hipStream_t stream) {
    const Acq &A = m->acq;
    const long long fstride = A.Pe.fstride;
    const size_t acc_elem = m->opt.dft_mode ? sizeof(float4) : sizeof(double2);
    const int nslot = A.nslot + A.ncorner;
    const size_t fbytes = (size_t)6 * A.nsrc * fstride * sizeof(float);
    const size_t psi_bytes = (state_floats(m) - 6 * fstride) * A.nsrc * sizeof(float);
    const size_t abytes = (size_t)nslot * A.nf * acc_elem;
    if (m->arena) {
        // the static workspace keeps the last call's contents; cleared with a
        // fill kernel (no memset node if the caller captures the stream)
        emm::launch_zero(m->fields.p, fbytes, stream);
        if (psi_bytes) emm::launch_zero(m->psi.p, psi_bytes, stream);
        emm::launch_zero(m->acc.p, abytes, stream);
        HIP_OK(m, hipGetLastError());
        return EMM_OK;
    }
    HIP_OK(m, hipMemsetAsync(m->fields.p, 0, fbytes, stream));
    if (psi_bytes) HIP_OK(m, hipMemsetAsync(m->psi.p, 0, psi_bytes, stream));
    HIP_OK(m, hipMemsetAsync(m->acc.p, 0, abytes, stream));
    return EMM_OK;
}

// Events of the profiling path, created once and kept with the model: grow
// the set to `count`.
emm_status ensure_events(emm_model *m, size_t count) {
    while (m->ring.size() < count) {
        hipEvent_t e = nullptr;
        HIP_OK(m, hipEventCreate(&e));
        m->ring.push_back(e);
    }
    return EMM_OK;
}

// Zero the state and run all time steps: per step the E step (+ H-channel
// DTFT) then the H step (+ E-channel DTFT).  ckpt > 0 stores the full state
// before every step n with n % ckpt == 0.
emm_status time_loop(emm_model *m, hipStream_t stream, int ckpt) {
    Acq &A = m->acq;
    emm_status st;
    const int nsrc = A.nsrc, nt = A.nt, r = m->r;
    if ((st = zero_state(m, stream)) != EMM_OK) return st;
    if (ckpt > 0) {
        const int nck = (nt + ckpt - 1) / ckpt;
        if ((st = ensure(m, m->ckpts, (size_t)nck * state_floats(m) * nsrc * sizeof(float))) != EMM_OK) return st;
    }
    // Profiling: HIP events stamped by the dispatch of one E step and one H
    // step out of every `sample` direct launches give those kernels' start
    // and end.  With graph replays (event nodes in graphs
    // carry no timestamps here), every 8th block of K steps is launched
    // directly instead -- the same kernels with the absolute step index --
    // and sampled, so the timing is taken inside the timed loop.
    const bool prof = m->opt.profile != 0;
    const int sample = 16;
    if (prof) {
        // every timed E/H pair of this forward gets its own four events: no
        // event is recorded twice before the end of the loop reads it
        const int Kg = m->opt.graph_steps;
        const long long blocks = Kg > 0 ? (nt / Kg + 7) / 8 : 0;
        const long long timed_max = blocks * ((Kg + 3) / 4) + (nt + sample - 1) / sample + 1;
        if ((st = ensure_events(m, (size_t)(4 * timed_max))) != EMM_OK) return st;
    }
    const bool loop_events = !m->arena;     // a no-alloc call creates no events
    if (loop_events && !m->ev_loop[0]) {
        HIP_OK(m, hipEventCreate(&m->ev_loop[0]));
        HIP_OK(m, hipEventCreate(&m->ev_loop[1]));
    }
    double ems = 0.0, hms = 0.0;
    long long nsamp = 0;
    int nslots_used = 0;
    auto harvest = [&](int slot) -> emm_status {
        float a = 0.f, b = 0.f;
        HIP_OK(m, hipEventSynchronize(m->ring[4 * slot + 3]));
        HIP_OK(m, hipEventElapsedTime(&a, m->ring[4 * slot + 0], m->ring[4 * slot + 1]));
        HIP_OK(m, hipEventElapsedTime(&b, m->ring[4 * slot + 2], m->ring[4 * slot + 3]));
        ems += a;
        hms += b;
        ++nsamp;
        return EMM_OK;
    };
    // one direct step, bracketed by events when `timed`
    auto step = [&](int n, bool timed) -> emm_status {
        int slot = -1;
        if (timed) {
            slot = nslots_used++;
            if ((size_t)(4 * slot + 3) >= m->ring.size()) return fail(m, EMM_ERR_ARG, "profiling events exhausted");
        }
        // timed launches carry their events in the dispatch itself (kernel
        // start and end, as a kernel trace reports them)
        std::string aerr;
        emm::launch_e_step(r, A.Pe, n, stream, timed ? m->ring[4 * slot + 0] : nullptr,
                           timed ? m->ring[4 * slot + 1] : nullptr);
        if (m->air && !m->air->fill_E(A.Pe.E1, stream, aerr)) return fail(m, EMM_ERR_DEVICE, aerr);
        emm::launch_h_step(r, A.Ph, n, stream, timed ? m->ring[4 * slot + 2] : nullptr,
                           timed ? m->ring[4 * slot + 3] : nullptr);
        if (m->air && !m->air->fill_H(A.Ph.H1, A.Ph.H3, stream, aerr)) return fail(m, EMM_ERR_DEVICE, aerr);
        HIP_OK(m, hipGetLastError());
        return EMM_OK;
    };
    // convergence stop (converge_tol > 0): every `every` steps, the lowest-
    // frequency DTFT of E1 at the interior corners against the last check
    const bool conv = A.ncorner > 0;
    const int every = m->opt.converge_every;
    const size_t acc_elem = m->opt.dft_mode ? sizeof(float4) : sizeof(double2);
    std::vector<std::complex<double>> prev(A.ncorner, 0.0);
    std::vector<double> craw((size_t)A.ncorner * A.nf * (acc_elem / sizeof(double)));
    bool converged = false;
    int n_done = nt;
    auto check = [&](int nd) -> emm_status {
        HIP_OK(m, hipMemcpyAsync(craw.data(), (char *)m->acc.p + (size_t)A.nslot * A.nf * acc_elem,
                                 craw.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
        HIP_OK(m, hipStreamSynchronize(stream));
        bool all = true;
        for (int s = 0; s < A.nsrc; ++s) {
            double num = 0.0, den = 0.0;
            for (int c = 0; c < 8; ++c) {
                const size_t k = (size_t)(8 * s + c) * A.nf + A.fmin_index;
                std::complex<double> v;
                if (m->opt.dft_mode == 0) {
                    v = {craw[2 * k], craw[2 * k + 1]};
                } else {
                    const float *q = reinterpret_cast<const float *>(craw.data()) + 4 * k;
                    v = {(double)q[0] - (double)q[1], (double)q[2] - (double)q[3]};
                }
                num = std::max(num, std::abs(v - prev[8 * s + c]));
                den = std::max(den, std::abs(v));
                prev[8 * s + c] = v;
            }
            if (!(den > 0.0 && num <= m->opt.converge_tol * den)) all = false;
        }
        if (all) {
            converged = true;
            n_done = nd;
        }
        return EMM_OK;
    };
    if (loop_events) HIP_OK(m, hipEventRecord(m->ev_loop[0], stream));
    int n_begin = 0;
    // K steps per captured hipGraph, replayed with a device step counter;
    // checkpoints and convergence checks must fall on replay edges
    const int K = m->opt.graph_steps;
    if (K > 0 && nt >= K && (ckpt == 0 || ckpt % K == 0) && (!conv || every % K == 0)) {
        if ((st = ensure(m, m->stepdev, 256)) != EMM_OK) return st;
        int *stepd = (int *)m->stepdev.p;
        HIP_OK(m, hipMemsetAsync(stepd, 0, sizeof(int), stream));
        emm::StepParams Pe = A.Pe, Ph = A.Ph;
        Pe.step_base = Ph.step_base = stepd;
        GraphHold gh;
        HIP_OK(m, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        // the air boundary's FFTs and spectral kernels are captured with the steps
        std::string aerr;
        bool aok = true;
        for (int j = 0; j < K && aok; ++j) {
            emm::launch_e_step(r, Pe, j, stream);
            if (m->air) aok = m->air->fill_E(A.Pe.E1, stream, aerr);
            emm::launch_h_step(r, Ph, j, stream);
            if (m->air && aok) aok = m->air->fill_H(A.Ph.H1, A.Ph.H3, stream, aerr);
        }
        emm::launch_advance(stepd, K, stream);
        hipError_t ce = hipStreamEndCapture(stream, &gh.graph);
        if (!aok || ce != hipSuccess)
            return fail(m, EMM_ERR_DEVICE, "graph capture: " + (aok ? std::string(hipGetErrorString(ce)) : aerr));
        hipError_t e = hipGraphInstantiate(&gh.exec, gh.graph, nullptr, nullptr, 0);
        if (e != hipSuccess)
            return fail(m, EMM_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        const int reps = nt / K;
        for (int q = 0; q < reps; ++q) {
            const int n = q * K;
            if (ckpt > 0 && n % ckpt == 0 && (st = copy_state(m, m->ckpts.p, n / ckpt, true, stream)) != EMM_OK) return st;
            if (prof && q % 8 == 0) {
                for (int j = 0; j < K; ++j)
                    if ((st = step(n + j, j % 4 == 0)) != EMM_OK) return st;
                emm::launch_advance(stepd, K, stream);
            } else {
                HIP_OK(m, hipGraphLaunch(gh.exec, stream));
            }
            if (conv && (n + K) % every == 0) {
                if ((st = check(n + K)) != EMM_OK) return st;
                if (converged) break;
            }
        }
        HIP_OK(m, hipStreamSynchronize(stream));
        n_begin = converged ? nt : reps * K;
    }
    for (int n = n_begin; n < nt; ++n) {
        if (ckpt > 0 && n % ckpt == 0 && (st = copy_state(m, m->ckpts.p, n / ckpt, true, stream)) != EMM_OK) return st;
        if ((st = step(n, prof && (n - n_begin) % sample == 0)) != EMM_OK) return st;
        if (conv && (n + 1) % every == 0) {
            if ((st = check(n + 1)) != EMM_OK) return st;
            if (converged) break;
        }
    }
    if (converged) {
        // source spectrum over the steps actually run (same order of sums as
        // a run of that many steps)
        for (int f = 0; f < A.nf; ++f) {
            A.Shat[f] = 0.0;
            for (int n = 0; n < n_done; ++n)
                A.Shat[f] += (double)A.wavelet[n] *
                             std::exp(std::complex<double>(0, 1) * A.wp[f] * ((n + 0.5) * m->dt));
        }
    }
    HIP_OK(m, hipGetLastError());
    if (loop_events) HIP_OK(m, hipEventRecord(m->ev_loop[1], stream));
    if (prof)
        for (int u = 0; u < nslots_used; ++u)
            if ((st = harvest(u)) != EMM_OK) return st;
    HIP_OK(m, hipStreamSynchronize(stream));
    float loop_ms = 0.f;
    if (loop_events) HIP_OK(m, hipEventElapsedTime(&loop_ms, m->ev_loop[0], m->ev_loop[1]));
    A.ckpt = converged ? 0 : ckpt;
    m->info.nt = n_done;
    m->info.converged = converged ? 1 : 0;
    m->info.forward_ms = loop_ms;
    note_run(m, A.Pe);
    m->info.fused = 0;
    m->info.e_kernel_ms = prof ? ems : 0.0;
    m->info.h_kernel_ms = prof ? hms : 0.0;
    m->info.e_launches = prof ? nsamp : 0;
    m->info.h_launches = prof ? nsamp : 0;
    return EMM_OK;
}

// Accumulators back to the host (complex, per slot and frequency).
emm_status read_acc(emm_model *m, hipStream_t stream, std::vector<std::complex<double>> &acc) {
    const Acq &A = m->acq;
    const size_t n = (size_t)A.nsrc * A.nrec * A.nch * A.nf;
    const size_t acc_elem = m->opt.dft_mode ? sizeof(float4) : sizeof(double2);
    std::vector<double> raw(n * (acc_elem / sizeof(double)));
    HIP_OK(m, hipMemcpyAsync(raw.data(), m->acc.p, n * acc_elem, hipMemcpyDeviceToHost, stream));
    HIP_OK(m, hipStreamSynchronize(stream));
    acc.resize(n);
    for (size_t k = 0; k < n; ++k) {
        if (m->opt.dft_mode == 0) {
            acc[k] = {raw[2 * k], raw[2 * k + 1]};
        } else {
            const float *q = reinterpret_cast<const float *>(raw.data()) + 4 * k;
            acc[k] = {(double)q[0] - (double)q[1], (double)q[2] - (double)q[3]};
        }
    }
    return EMM_OK;
}

// d G / d acc for slot k: G = c * acc with c = (omega/omega' for E channels) / (scale moment S_f)
std::complex<double> green_factor(const emm_model *m, size_t k) {
    const Acq &A = m->acq;
    const int f = (int)(k % A.nf);
    const int c = (int)((k / A.nf) % A.nch);
    const int s = (int)(k / ((size_t)A.nf * A.nch * A.nrec));
    std::complex<double> g = 1.0 / (A.sscale[s] * A.src[s].moment * A.Shat[f]);
    if (A.chans[c] < 3) g *= (2.0 * kPi * A.freqs[f]) / A.wp[f];
    return g;
}

// All time steps with the fused step kernel: E, H and the E-step CPML
// memories alternate between two buffers (step n reads set n % 2 and writes
// the other); the DTFT waves of step n record H^{n+1/2} and E^n, and one last
// launch without stencil blocks records E^{nt}.
emm_status leap_loop(emm_model *m, hipStream_t stream) {
    Acq &A = m->acq;
    emm_status st;
    const int nsrc = A.nsrc, nt = A.nt, r = m->r, L = 2 * r;
    const long long fstride = A.Pe.fstride;
    if ((st = zero_state(m, stream)) != EMM_OK) return st;
    const size_t fbytes = (size_t)6 * nsrc * fstride * sizeof(float);
    const size_t psi_e = (state_floats(m) - 6 * fstride) * nsrc / 2 * sizeof(float);   // E-step half
    if ((st = ensure(m, m->fieldsB, fbytes)) != EMM_OK) return st;
    if ((st = ensure(m, m->psiB, std::max<size_t>(psi_e, 256))) != EMM_OK) return st;
    HIP_OK(m, hipMemsetAsync(m->fieldsB.p, 0, fbytes, stream));
    if (psi_e) HIP_OK(m, hipMemsetAsync(m->psiB.p, 0, psi_e, stream));
    // tiling: outputs (65 - 2r) x (rows + 1 - 2r) per block, z chunks of kz
    emm::LeapParams X{};
    const int TXO = emm::kTileX - (L - 1), TYO = emm::kLeapRows - (L - 1);
    X.xt = (m->np[0] - 2 * r + TXO - 1) / TXO;
    X.yt = (m->np[1] - 2 * r + TYO - 1) / TYO;
    const int nzv = m->np[2] - 2 * r;
    X.kz = std::min(std::max(m->opt.tile_kz > 0 ? m->opt.tile_kz : 16, 1), nzv);
    X.zc = (nzv + X.kz - 1) / X.kz;
    X.nstencil = X.xt * X.yt * X.zc * nsrc;
    const int waves = emm::leap_threads() / 64;
    X.nrech = (int)((A.Pe.nitems + waves - 1) / waves + 7) / 8 * 8;
    X.nrece = (int)((A.Ph.nitems + waves - 1) / waves + 7) / 8 * 8;
    // the two parameter sets: parity 0 reads (fields, psi) and writes (fieldsB, psiB)
    float *FA = (float *)m->fields.p, *FB = (float *)m->fieldsB.p;
    const size_t cs = (size_t)nsrc * fstride;
    emm::StepParams pe[2], ph[2];
    emm::LeapParams xp[2];
    for (int par = 0; par < 2; ++par) {
        float *in = par ? FB : FA, *out = par ? FA : FB;
        pe[par] = A.Pe;
        ph[par] = A.Ph;
        for (emm::StepParams *P : {&pe[par], &ph[par]}) {
            P->E1 = in;
            P->E2 = in + cs;
            P->E3 = in + 2 * cs;
            P->H1 = in + 3 * cs;
            P->H2 = in + 4 * cs;
            P->H3 = in + 5 * cs;
        }
        xp[par] = X;
        xp[par].Eo1 = out;
        xp[par].Eo2 = out + cs;
        xp[par].Eo3 = out + 2 * cs;
        xp[par].Ho1 = out + 3 * cs;
        xp[par].Ho2 = out + 4 * cs;
        xp[par].Ho3 = out + 5 * cs;
        // E-step memories: x0 x1 y0 y1 z0 z1 of all sources, in A.Pe's layout
        float *qa = (float *)m->psi.p, *qb = (float *)m->psiB.p;
        float *rd_ = par ? qb : qa, *wr_ = par ? qa : qb;
        auto at = [&](float *base, const float *ref) { return base + (ref - (const float *)m->psi.p); };
        pe[par].psx0 = at(rd_, A.Pe.psx0);
        pe[par].psx1 = at(rd_, A.Pe.psx1);
        pe[par].psy0 = at(rd_, A.Pe.psy0);
        pe[par].psy1 = at(rd_, A.Pe.psy1);
        pe[par].psz0 = at(rd_, A.Pe.psz0);
        pe[par].psz1 = at(rd_, A.Pe.psz1);
        xp[par].qx0 = at(wr_, A.Pe.psx0);
        xp[par].qx1 = at(wr_, A.Pe.psx1);
        xp[par].qy0 = at(wr_, A.Pe.psy0);
        xp[par].qy1 = at(wr_, A.Pe.psy1);
        xp[par].qz0 = at(wr_, A.Pe.psz0);
        xp[par].qz1 = at(wr_, A.Pe.psz1);
    }
    const bool prof = m->opt.profile != 0;
    if (prof) {
        // one event pair per timed launch of this forward (none recorded twice)
        const int Kg = m->opt.graph_steps;
        const long long blocks = Kg > 0 ? (nt / Kg + 7) / 8 : 0;
        const long long timed_max = blocks * ((Kg + 3) / 4) + (nt + 15) / 16 + 1;
        if ((st = ensure_events(m, (size_t)(2 * timed_max))) != EMM_OK) return st;
    }
    if (!m->ev_loop[0]) {
        HIP_OK(m, hipEventCreate(&m->ev_loop[0]));
        HIP_OK(m, hipEventCreate(&m->ev_loop[1]));
    }
    double lms = 0.0;
    long long nsamp = 0;
    int used = 0;
    auto harvest = [&](int slot) -> emm_status {
        float a = 0.f;
        HIP_OK(m, hipEventSynchronize(m->ring[2 * slot + 1]));
        HIP_OK(m, hipEventElapsedTime(&a, m->ring[2 * slot], m->ring[2 * slot + 1]));
        lms += a;
        ++nsamp;
        return EMM_OK;
    };
    auto step = [&](int n, bool timed) -> emm_status {
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (timed) {
            const int slot = used++;
            if ((size_t)(2 * slot + 1) >= m->ring.size()) return fail(m, EMM_ERR_ARG, "profiling events exhausted");
            t0 = m->ring[2 * slot];
            t1 = m->ring[2 * slot + 1];
        }
        emm::launch_leap(r, pe[n & 1], ph[n & 1], xp[n & 1], n, stream, t0, t1);
        HIP_OK(m, hipGetLastError());
        return EMM_OK;
    };
    HIP_OK(m, hipEventRecord(m->ev_loop[0], stream));
    int n_begin = 0;
    const int K = m->opt.graph_steps;
    if (K > 0 && K % 2 == 0 && nt >= K) {
        if ((st = ensure(m, m->stepdev, 256)) != EMM_OK) return st;
        int *stepd = (int *)m->stepdev.p;
        HIP_OK(m, hipMemsetAsync(stepd, 0, sizeof(int), stream));
        emm::StepParams ge[2] = {pe[0], pe[1]}, gh[2] = {ph[0], ph[1]};
        for (int par = 0; par < 2; ++par) ge[par].step_base = gh[par].step_base = stepd;
        GraphHold hold;
        HIP_OK(m, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < K; ++j) emm::launch_leap(r, ge[j & 1], gh[j & 1], xp[j & 1], j, stream);
        emm::launch_advance(stepd, K, stream);
        HIP_OK(m, hipStreamEndCapture(stream, &hold.graph));
        hipError_t e = hipGraphInstantiate(&hold.exec, hold.graph, nullptr, nullptr, 0);
        if (e != hipSuccess)
            return fail(m, EMM_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        const int reps = nt / K;
        for (int q = 0; q < reps; ++q) {
            if (prof && q % 8 == 0) {
                for (int j = 0; j < K; ++j)
                    if ((st = step(q * K + j, j % 4 == 0)) != EMM_OK) return st;
                emm::launch_advance(stepd, K, stream);
            } else {
                HIP_OK(m, hipGraphLaunch(hold.exec, stream));
            }
        }
        HIP_OK(m, hipStreamSynchronize(stream));
        n_begin = reps * K;
    }
    for (int n = n_begin; n < nt; ++n)
        if ((st = step(n, prof && (n - n_begin) % 16 == 0)) != EMM_OK) return st;
    // E^{nt}: DTFT waves of the E channels only
    emm::LeapParams xf = xp[nt & 1];
    xf.nstencil = 0;
    xf.nrech = 0;
    emm::launch_leap(r, pe[nt & 1], ph[nt & 1], xf, nt, stream);
    HIP_OK(m, hipGetLastError());
    HIP_OK(m, hipEventRecord(m->ev_loop[1], stream));
    if (prof)
        for (int u = 0; u < used; ++u)
            if ((st = harvest(u)) != EMM_OK) return st;
    HIP_OK(m, hipStreamSynchronize(stream));
    float loop_ms = 0.f;
    HIP_OK(m, hipEventElapsedTime(&loop_ms, m->ev_loop[0], m->ev_loop[1]));
    A.ckpt = 0;
    m->info.nt = nt;
    m->info.converged = 0;
    m->info.fused = 1;
    m->info.forward_ms = loop_ms;
    note_run(m, A.Pe);
    m->info.tile_kz = X.kz;
    m->info.ce_table = 0;                      // the fused kernel reads the FP32 arrays
    m->info.e_kernel_ms = prof ? lms : 0.0;
    m->info.h_kernel_ms = 0.0;
    m->info.e_launches = prof ? nsamp : 0;
    m->info.h_launches = 0;
    return EMM_OK;
}

// G from the accumulators of the last forward (Section 2.2 normalisation).
emm_status write_green(emm_model *m, hipStream_t stream, double *green) {
    emm_status st;
    std::vector<std::complex<double>> acc;
    if ((st = read_acc(m, stream, acc)) != EMM_OK) return st;
    bool nonfinite = false;
    for (size_t k = 0; k < acc.size(); ++k) {
        const std::complex<double> G = acc[k] * green_factor(m, k);
        if (!std::isfinite(G.real()) || !std::isfinite(G.imag())) nonfinite = true;
        green[2 * k] = G.real();
        green[2 * k + 1] = G.imag();
    }
    if (nonfinite) return fail(m, EMM_ERR_NONFINITE, "a DTFT accumulator is not finite (unstable run?)");
    return EMM_OK;
}

// Time loops of several models (one job each) side by side: every job has
// its own stream and its own captured hipGraph of K steps (replayed with the
// model's device step counter), the replays of all jobs are issued in turn,
// and a job's last nt % K steps run as direct launches on its stream.  The
// jobs' streams start after the work already queued on `stream` and
// `stream` waits for all of them at the end, so small grids share the chip
// (eight 74^3 grids: 2.4x faster than one after another).
emm_status time_loop_jobs(const std::vector<emm_model *> &ms, int K, hipStream_t stream) {
    emm_status st = EMM_OK;
    emm_model *m0 = ms[0];
    const int nj = (int)ms.size();
    for (emm_model *m : ms) {
        if ((st = zero_state(m, stream)) != EMM_OK) return st;
        if ((st = ensure(m, m->stepdev, 256)) != EMM_OK) return st;
        HIP_OK(m, hipMemsetAsync(m->stepdev.p, 0, sizeof(int), stream));
        m->acq.ckpt = 0;
    }
    std::vector<hipStream_t> side(nj, nullptr);
    std::vector<hipEvent_t> join(nj, nullptr);
    std::vector<hipGraph_t> graph(nj, nullptr);
    std::vector<hipGraphExec_t> exec(nj, nullptr);
    hipEvent_t fork = nullptr, t0 = nullptr, t1 = nullptr;
    auto cleanup = [&]() {
        for (hipStream_t q : side) if (q) (void)hipStreamSynchronize(q);
        for (hipGraphExec_t x : exec) if (x) (void)hipGraphExecDestroy(x);
        for (hipGraph_t g : graph) if (g) (void)hipGraphDestroy(g);
        for (hipStream_t q : side) if (q) (void)hipStreamDestroy(q);
        for (hipEvent_t e : join) if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : {fork, t0, t1}) if (e) (void)hipEventDestroy(e);
    };
    auto run = [&]() -> emm_status {
        HIP_OK(m0, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        HIP_OK(m0, hipEventCreate(&t0));
        HIP_OK(m0, hipEventCreate(&t1));
        std::vector<int> whole(nj);
        int most = 0;
        for (int j = 0; j < nj; ++j) {
            HIP_OK(m0, hipStreamCreateWithFlags(&side[j], hipStreamNonBlocking));
            HIP_OK(m0, hipEventCreateWithFlags(&join[j], hipEventDisableTiming));
            emm_model *m = ms[j];
            whole[j] = m->acq.nt / K;
            most = std::max(most, whole[j]);
            if (whole[j] == 0) continue;
            emm::StepParams Pe = m->acq.Pe, Ph = m->acq.Ph;
            Pe.step_base = Ph.step_base = (const int *)m->stepdev.p;
            HIP_OK(m0, hipStreamBeginCapture(side[j], hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < K; ++i) {
                emm::launch_e_step(m->r, Pe, i, side[j]);
                emm::launch_h_step(m->r, Ph, i, side[j]);
            }
            emm::launch_advance((int *)m->stepdev.p, K, side[j]);
            hipError_t ce = hipStreamEndCapture(side[j], &graph[j]);
            if (ce != hipSuccess) return fail(m0, EMM_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
            ce = hipGraphInstantiate(&exec[j], graph[j], nullptr, nullptr, 0);
            if (ce != hipSuccess)
                return fail(m0, EMM_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ce));
        }
        // the jobs start after what is queued on `stream` (state set-up)
        HIP_OK(m0, hipEventRecord(t0, stream));
        HIP_OK(m0, hipEventRecord(fork, stream));
        for (int j = 0; j < nj; ++j) HIP_OK(m0, hipStreamWaitEvent(side[j], fork, 0));
        for (int u = 0; u < most; ++u)
            for (int j = 0; j < nj; ++j)
                if (u < whole[j]) HIP_OK(m0, hipGraphLaunch(exec[j], side[j]));
        for (int j = 0; j < nj; ++j) {
            const Acq &A = ms[j]->acq;
            for (int n = whole[j] * K; n < A.nt; ++n) {
                emm::launch_e_step(ms[j]->r, A.Pe, n, side[j]);
                emm::launch_h_step(ms[j]->r, A.Ph, n, side[j]);
            }
            HIP_OK(m0, hipEventRecord(join[j], side[j]));
            HIP_OK(m0, hipStreamWaitEvent(stream, join[j], 0));
        }
        HIP_OK(m0, hipGetLastError());
        HIP_OK(m0, hipEventRecord(t1, stream));
        HIP_OK(m0, hipStreamSynchronize(stream));
        float ms_loop = 0.f;
        HIP_OK(m0, hipEventElapsedTime(&ms_loop, t0, t1));
        for (emm_model *m : ms) {
            m->info.nt = m->acq.nt;
            m->info.forward_ms = ms_loop;
            note_run(m, m->acq.Pe);
            m->info.fused = 0;
            m->info.e_kernel_ms = m->info.h_kernel_ms = 0.0;
            m->info.e_launches = m->info.h_launches = 0;
        }
        return EMM_OK;
    };
    st = run();
    cleanup();
    return st;
}

// Autotuner of the z chunk per thread block and of the nontemporal hint
// (tile_kz = -1): time a few steps of both stencil kernels for each
// candidate (z planes per block x nontemporal hint x compact dt/eps) on this
// model and acquisition, then time the four fastest again over more steps
// and keep the best (cached per source count).  The
// state it leaves behind is discarded: the time loop starts from zero
// fields.
emm_status autotune(emm_model *m, hipStream_t stream) {
    Acq &A = m->acq;
    if (m->opt.tile_kz >= 0 || m->tuned.count(A.nsrc)) return EMM_OK;
    const int nzv = z_planes(m);
    // every distinct z chunking with at least 3 planes per block (the
    // smallest kz of each chunk count): how many waves of blocks a launch
    // needs on the chip moves the time by several per cent between
    // neighbouring kz, and on deep grids one to three chunks per column
    // save the z-queue refills of the others
    std::vector<int> cand;
    for (int zc = 1; zc <= nzv; ++zc) {
        const int kz = (nzv + zc - 1) / zc;
        if (kz < 3) break;
        if (cand.empty() || cand.back() != kz) cand.push_back(kz);
    }
    if (std::find(cand.begin(), cand.end(), A.Pe.kz) == cand.end()) cand.push_back(A.Pe.kz);
    std::vector<int> hints = {0, 1}, compacts = {0};
    // tile shapes (width, rows per wavefront): 64 x 4 and 32 x 8; the
    // register-blocked 64 x 8 and 64 x 16 only when tile_rows asks for them
    // (measured slower on every grid here: 2-3 waves per SIMD instead of 4-6)
    std::vector<std::pair<int, int>> shapes = {{64, 1}, {32, 1}};
    if (m->opt.nontemporal >= 0) hints = {m->opt.nontemporal};
    if (m->opt.tile_x > 0 || m->opt.tile_rows > 0) {
        std::vector<std::pair<int, int>> keep;
        for (auto sh : {std::make_pair(64, 1), std::make_pair(32, 1), std::make_pair(64, 2),
                        std::make_pair(64, 4)})
            if ((m->opt.tile_x == 0 || sh.first == m->opt.tile_x) &&
                (m->opt.tile_rows == 0 || sh.second == m->opt.tile_rows))
                keep.push_back(sh);
        shapes = keep;
    }
    if (m->cei && m->opt.ce_table == -1) compacts = {0, 1};
    else if (m->cei && m->opt.ce_table == 1) compacts = {1};
    hipEvent_t e0, e1;
    HIP_OK(m, hipEventCreate(&e0));
    HIP_OK(m, hipEventCreate(&e1));
    auto time_it = [&](const Tune &c, int steps, float &ms) -> emm_status {
        emm::StepParams Pe = A.Pe, Ph = A.Ph;
        set_tiles(Pe, m, c.tx, c.ry);
        set_tiles(Ph, m, c.tx, c.ry);
        Pe.kz = Ph.kz = c.kz;
        Pe.zc = Ph.zc = (nzv + c.kz - 1) / c.kz;
        Pe.nstencil = Ph.nstencil = Pe.xt * Pe.yt * Pe.zc * A.nsrc;
        Pe.stream = Ph.stream = c.stream;
        Pe.sorder = Ph.sorder = c.sorder;
        Pe.cei = c.compact ? m->cei : nullptr;
        for (int n = 0; n < 2; ++n) {              // warm-up
            emm::launch_e_step(m->r, Pe, n, stream);
            emm::launch_h_step(m->r, Ph, n, stream);
        }
        HIP_OK(m, hipEventRecord(e0, stream));
        for (int n = 0; n < steps; ++n) {
            emm::launch_e_step(m->r, Pe, n, stream);
            emm::launch_h_step(m->r, Ph, n, stream);
        }
        HIP_OK(m, hipEventRecord(e1, stream));
        HIP_OK(m, hipEventSynchronize(e1));
        HIP_OK(m, hipEventElapsedTime(&ms, e0, e1));
        return EMM_OK;
    };
    std::vector<std::pair<float, int>> first;   // (ms, index into tried)
    std::vector<Tune> tried;
    emm_status st;
    std::vector<int> orders = {0};
    if (A.nsrc > 1) orders = {0, 1};
    if (m->opt.src_order >= 0) orders = {m->opt.src_order};
    for (int so : orders)
    for (auto shape : shapes)
        for (int cp : compacts)
            for (int sh : hints)
                for (int kz : cand) {
                    Tune c;
                    c.kz = kz;
                    c.stream = sh;
                    c.compact = cp;
                    c.tx = shape.first;
                    c.ry = shape.second;
                    c.sorder = so;
                    float ms = 0.f;
                    if ((st = time_it(c, 6, ms)) != EMM_OK) return st;
                    first.push_back({ms, (int)tried.size()});
                    tried.push_back(c);
                }
    std::sort(first.begin(), first.end());
    float best = 1e30f;
    Tune pick;
    pick.kz = A.Pe.kz;
    pick.stream = A.Pe.stream;
    pick.compact = A.Pe.cei != nullptr;
    pick.tx = A.Pe.tx;
    pick.ry = A.Pe.ry;
    pick.sorder = A.Pe.sorder;
    if (!first.empty()) pick = tried[first[0].second];
    for (size_t c = 0; c < std::min<size_t>(4, first.size()); ++c) {
        float ms = 0.f;
        if ((st = time_it(tried[first[c].second], 16, ms)) != EMM_OK) return st;
        if (ms < best) {
            best = ms;
            pick = tried[first[c].second];
        }
    }

    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_OK(m, hipGetLastError());
    m->tuned[A.nsrc] = pick;
    for (emm::StepParams *P : {&A.Pe, &A.Ph}) {
        set_tiles(*P, m, pick.tx, pick.ry);
        P->kz = pick.kz;
        P->zc = (nzv + pick.kz - 1) / pick.kz;
        P->nstencil = P->xt * P->yt * P->zc * A.nsrc;
        P->stream = pick.stream;
        P->sorder = pick.sorder;
    }
    A.Pe.cei = pick.compact ? m->cei : nullptr;
    return EMM_OK;
}

}  // namespace

extern "C" {

emm_status emm_forward(emm_model *m, const emm_source *src, int nsrc, const emm_receiver *rec,
                       int nrec, unsigned chan_mask, const double *freq_hz, int nfreq,
                       double *green, void *hip_stream) {
    if (!m) return fail(nullptr, EMM_ERR_ARG, "NULL model");
    m->err.clear();
    if (!green) return fail(m, EMM_ERR_ARG, "NULL output pointer");
    emm_status st;
    hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : m->own_stream;
    const bool leap = m->opt.fused && m->opt.checkpoint_every == 0 && !m->opt.airwave &&
                      !(m->opt.converge_tol > 0.0);
    // sources in groups, one time loop per group; the checkpoints that a
    // gradient reuses and a batch-wide convergence stop need every source in
    // one loop.  Every source is checked before the first group runs.
    const int g = (src && nsrc > 1 && m->opt.checkpoint_every == 0 && !(m->opt.converge_tol > 0.0))
                      ? source_group(m, nsrc) : nsrc;
    if (g < nsrc)
        for (int s = 0; s < nsrc; ++s)
            if ((st = check_source(m, src[s])) != EMM_OK) return st;
    double fwd_ms = 0.0, e_ms = 0.0, h_ms = 0.0;
    long long e_n = 0, h_n = 0;
    for (int g0 = 0; g0 < nsrc || g0 == 0; g0 += std::max(g, 1)) {
        const int ng = std::min(g, nsrc - g0);
        if ((st = prepare(m, src ? src + g0 : src, ng, rec, nrec, chan_mask, freq_hz, nfreq, stream)) != EMM_OK)
            return st;
        if ((st = autotune(m, stream)) != EMM_OK) return st;
        if ((st = leap ? leap_loop(m, stream) : time_loop(m, stream, m->opt.checkpoint_every)) != EMM_OK) return st;
        const size_t per_src = (size_t)m->acq.nrec * m->acq.nch * m->acq.nf * 2;
        if ((st = write_green(m, stream, green + (size_t)g0 * per_src)) != EMM_OK) return st;
        fwd_ms += m->info.forward_ms;
        e_ms += m->info.e_kernel_ms;
        h_ms += m->info.h_kernel_ms;
        e_n += m->info.e_launches;
        h_n += m->info.h_launches;
    }
    m->info.forward_ms = fwd_ms;
    m->info.e_kernel_ms = e_ms;
    m->info.h_kernel_ms = h_ms;
    m->info.e_launches = e_n;
    m->info.h_launches = h_n;
    m->info.src_group = g;
    return EMM_OK;
}

emm_status emm_forward_noalloc(emm_model *m, const emm_source *src, int nsrc,
                               const emm_receiver *rec, int nrec, unsigned chan_mask,
                               const double *freq_hz, int nfreq, double *green, void *hip_stream) {
    if (!m) return fail(nullptr, EMM_ERR_ARG, "NULL model");
    m->err.clear();
    if (!green) return fail(m, EMM_ERR_ARG, "NULL output pointer");
    if (m->opt.airwave || m->opt.checkpoint_every > 0)
        return fail(m, EMM_ERR_ARG, "emm_forward_noalloc runs neither the air boundary nor "
                                    "checkpointed forwards (their buffers need allocation)");
    if (m->scratch_err != hipSuccess || !m->scratch)
        return fail(m, EMM_ERR_DEVICE, std::string("static workspace address: ") + hipGetErrorString(m->scratch_err));
    hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : m->own_stream;
    // the forward-lifetime buffers of earlier emm_forward calls stay aside
    // (and allocated) while this call carves its own from the workspace
    DevBuf *bufs[] = {&m->fields, &m->psi, &m->acc, &m->cpml, &m->srcinfo, &m->srcq,
                      &m->wav, &m->items, &m->itemw, &m->phase, &m->stepdev};
    constexpr int kBufs = sizeof(bufs) / sizeof(bufs[0]);
    DevBuf saved[kBufs];
    for (int b = 0; b < kBufs; ++b) {
        saved[b] = *bufs[b];
        *bufs[b] = DevBuf{};
    }
    const emm_options opt_saved = m->opt;
    m->opt.graph_steps = 0;        // direct launches: no graph to instantiate
    m->opt.profile = 0;            // no timing events
    m->arena = (char *)m->scratch;
    m->arena_cap = kScratchBytes;
    m->arena_used = 0;
    emm_status st = prepare(m, src, nsrc, rec, nrec, chan_mask, freq_hz, nfreq, stream);
    if (st == EMM_OK) st = time_loop(m, stream, 0);
    if (st == EMM_OK) st = write_green(m, stream, green);
    if (st != EMM_OK) (void)hipStreamSynchronize(stream);
    m->arena = nullptr;
    m->arena_cap = m->arena_used = 0;
    m->opt = opt_saved;
    for (int b = 0; b < kBufs; ++b) *bufs[b] = saved[b];
    m->acq.valid = false;          // its parameters point into the workspace
    m->acq.ckpt = 0;
    if (st != EMM_OK) return st;
    m->info.src_group = nsrc;
    m->info.e_kernel_ms = m->info.h_kernel_ms = 0.0;
    m->info.e_launches = m->info.h_launches = 0;
    return EMM_OK;
}

emm_status emm_forward_batch(const emm_job *jobs, int njobs, int graph_steps, void *hip_stream) {
    if (!jobs || njobs <= 0) return fail(nullptr, EMM_ERR_ARG, "need at least one job");
    if (graph_steps < 0) return fail(nullptr, EMM_ERR_ARG, "graph_steps must be >= 0");
    std::vector<emm_model *> ms;
    for (int j = 0; j < njobs; ++j) {
        emm_model *m = jobs[j].model;
        if (!m) return fail(nullptr, EMM_ERR_ARG, "job " + std::to_string(j) + ": NULL model");
        if (!jobs[j].green) return fail(m, EMM_ERR_ARG, "job " + std::to_string(j) + ": NULL output pointer");
        if (std::find(ms.begin(), ms.end(), m) != ms.end())
            return fail(m, EMM_ERR_ARG, "job " + std::to_string(j) + ": a model may appear in one job only");
        if (m->device != jobs[0].model->device)
            return fail(m, EMM_ERR_ARG, "job " + std::to_string(j) + ": all models must be on one device");
        if (m->opt.airwave || m->opt.converge_tol > 0.0)
            return fail(m, EMM_ERR_ARG, "job " + std::to_string(j) +
                                            ": the air boundary and the convergence stop run through emm_forward only");
        m->err.clear();
        ms.push_back(m);
    }
    hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : ms[0]->own_stream;
    emm_status st;
    for (int j = 0; j < njobs; ++j) {
        const emm_job &J = jobs[j];
        if ((st = prepare(J.model, J.src, J.nsrc, J.rec, J.nrec, J.chan_mask, J.freq_hz, J.nfreq, stream)) != EMM_OK)
            return st;
        if ((st = autotune(J.model, stream)) != EMM_OK) return st;
    }
    // jobs in consecutive groups, one graph per group, group after group
    // (src_group of the first job's model: -1 all jobs in one graph, k > 0
    // k jobs per graph, 0 as many as keep their arrays within the cache
    // budget of source_group; a job that alone exceeds it runs by itself)
    const int rule = ms[0]->opt.src_group;
    const double budget = 160.0 * (1 << 20);
    const double fill = 4.0 * (1 << 20);             // cells that keep the chip busy on their own
    std::vector<emm_model *> group;
    double held = 0.0, cells = 0.0;
    for (int j = 0; j <= njobs; ++j) {
        double need = 0.0;
        if (j < njobs) {
            emm_model *m = ms[j];
            need = 4.0 * (double)state_floats(m) * jobs[j].nsrc +
                   (double)m->pitch * m->np[1] * m->np[2] * (m->acq.Pe.cei ? 4.0 : 12.0);
        }
        // a group closes when the next job would overflow the cache budget,
        // unless the group is still too small to fill the chip
        const bool full = rule < 0 ? false
                          : rule > 0 ? (int)group.size() == rule
                                     : held + need > budget && cells >= fill;
        if (!group.empty() && (j == njobs || full)) {
            if ((st = time_loop_jobs(group, graph_steps > 0 ? graph_steps : 64, stream)) != EMM_OK) return st;
            for (emm_model *m : group) m->info.src_group = (int)group.size();
            group.clear();
            held = cells = 0.0;
        }
        if (j < njobs) {
            group.push_back(ms[j]);
            held += need;
            cells += (double)ms[j]->np[0] * ms[j]->np[1] * ms[j]->np[2] * jobs[j].nsrc;
        }
    }
    for (int j = 0; j < njobs; ++j)
        if ((st = write_green(jobs[j].model, stream, jobs[j].green)) != EMM_OK) return st;
    return EMM_OK;
}

// Device memory left for the checkpoints of a sweep over g sources: the
// free memory plus what the checkpoint buffers already hold, minus what the
// time-stepping state and the adjoint arrays of g sources still need and a
// margin.
emm_status ckpt_budget(emm_model *m, int g, size_t &bud) {
    const long long fs = (long long)m->pitch * m->np[1] * m->np[2];
    const size_t slab_src = (state_floats(m) - 6 * fs) / 2;     // 6 slab arrays per source
    const size_t need[8] = {(size_t)6 * g * fs * sizeof(float),
                            std::max<size_t>(1, 2 * g * slab_src) * sizeof(float),
                            std::max<size_t>(1, g * slab_src) * sizeof(float),
                            (size_t)3 * g * fs * sizeof(double),
                            (size_t)3 * g * fs * sizeof(float),
                            (size_t)6 * g * fs * sizeof(float),
                            std::max<size_t>(1, 2 * g * slab_src) * sizeof(float),
                            (size_t)3 * m->n[0] * m->n[1] * m->n[2] * sizeof(double)};
    const DevBuf *have[8] = {&m->adjf, &m->adjq, &m->adjt, &m->grad, &m->grad32, &m->fields, &m->psi, &m->gsum};
    size_t fr = 0, tot = 0;
    HIP_OK(m, hipMemGetInfo(&fr, &tot));
    long long budget = (long long)fr + (long long)(m->ckpts.bytes + m->ickpts.bytes + m->snaps.bytes);
    for (int b = 0; b < 8; ++b) budget -= (long long)(need[b] > have[b]->bytes ? need[b] - have[b]->bytes : 0);
    budget -= (long long)(tot / 50) + (256LL << 20);
    bud = budget > 0 ? (size_t)budget : 0;
    return EMM_OK;
}

// One forward + reverse sweep over the sources given (see emm_gradient).
// accumulate: add dL/dlog sigma onto grad and the misfit onto chi in the
// order a single call over all sources would (so groups of sources give
// the same bits); else start both from zero.
emm_status gradient_run(emm_model *m, const emm_source *src, int nsrc, const emm_receiver *rec, int nrec,
                        unsigned chan_mask, const double *freq_hz, int nfreq, const double *g_obs,
                        const double *g_bar, double *green, double &chi_acc, double *grad, bool accumulate,
                        hipStream_t stream) {
    emm_status st;
    // forward with checkpoints, unless the last forward stored them for the same acquisition
    const bool reuse = m->acq.ckpt > 0 && same_acquisition(m->acq, src, nsrc, rec, nrec, chan_mask, freq_hz, nfreq);
    if (!reuse) {
        if ((st = prepare(m, src, nsrc, rec, nrec, chan_mask, freq_hz, nfreq, stream)) != EMM_OK) return st;
        if ((st = autotune(m, stream)) != EMM_OK) return st;
    }
    // checkpoint schedule within the memory left for it
    int c1 = 0, c2 = 0;
    {
        const Acq &A0 = m->acq;
        const long long fs = A0.Pe.fstride;
        const size_t S = state_floats(m) * A0.nsrc * sizeof(float);
        const size_t F = (size_t)3 * A0.nsrc * fs * sizeof(float);
        size_t bud = 0;
        if ((st = ckpt_budget(m, A0.nsrc, bud)) != EMM_OK) return st;
        if (!plan_checkpoints(A0.nt, m->opt.graph_steps, reuse ? A0.ckpt : m->opt.checkpoint_every,
                              m->opt.checkpoint_inner, S, F, bud, c1, c2))
            return fail(m, EMM_ERR_OOM, "no checkpoint schedule fits in " + std::to_string(bud) +
                                            " bytes of device memory; run fewer sources per call");
        m->info.ckpt_outer = c1;
        m->info.ckpt_inner = std::min(c1, c2);
        m->info.ckpt_bytes = (double)ckpt_memory(A0.nt, c1, c2, S, F);
    }
    if (!reuse && (st = time_loop(m, stream, c1)) != EMM_OK) return st;
    const Acq &A = m->acq;
    const int ckpt = A.ckpt;                 // outer interval
    const int cin = std::min(c2, ckpt);      // inner interval
    std::vector<std::complex<double>> acc;
    if ((st = read_acc(m, stream, acc)) != EMM_OK) return st;
    const size_t nd = acc.size();
    // adjoint-source coefficients per slot: dL/du_n = sum_f Re(Acoef_f z_f^n) with
    // Acoef = conj(gbar) dG/dacc, gbar = dL/dRe G + i dL/dIm G; for the log misfit
    // L = 1/2 sum |log(G/G_obs)|^2, gbar = r / conj(G), r = log(G/G_obs).
    std::vector<double2> Acoef(nd);
    double chi = accumulate ? chi_acc : 0.0;
    bool nonfinite = false, badcot = false;
    for (size_t k = 0; k < nd; ++k) {
        const std::complex<double> c = green_factor(m, k);
        const std::complex<double> G = acc[k] * c;
        if (!std::isfinite(G.real()) || !std::isfinite(G.imag())) nonfinite = true;
        if (green) {
            green[2 * k] = G.real();
            green[2 * k + 1] = G.imag();
        }
        std::complex<double> gb;
        if (g_obs) {
            const std::complex<double> Go(g_obs[2 * k], g_obs[2 * k + 1]);
            const std::complex<double> rr = std::log(G / Go);
            chi += 0.5 * std::norm(rr);
            gb = rr / std::conj(G);
        } else {
            gb = {g_bar[2 * k], g_bar[2 * k + 1]};
        }
        const std::complex<double> a = std::conj(gb) * c;
        if (!std::isfinite(a.real()) || !std::isfinite(a.imag())) badcot = true;
        Acoef[k] = make_double2(a.real(), a.imag());
    }
    if (nonfinite) return fail(m, EMM_ERR_NONFINITE, "a DTFT accumulator is not finite (unstable run?)");
    if (badcot)
        return fail(m, EMM_ERR_NONFINITE, g_obs ? "the misfit is not finite (a G or G_obs of zero or non-finite value)"
                                                : "g_bar holds a non-finite value");
    chi_acc = g_obs ? chi : 0.0;

    // ---- adjoint set-up ----
    const int r = m->r, L = 2 * r, nb = m->nb, nt = A.nt;
    const int n1 = m->np[0], n2 = m->np[1], n3 = m->np[2];
    const long long fstride = A.Pe.fstride, plane = A.Pe.plane;
    // transposed FD tables: (D-)^T has the D+ shape, (D+)^T the D- shape
    if (!m->tabT.p) {
        std::vector<float> t;
        std::vector<size_t> off;
        for (int kind = 0; kind < 2; ++kind)          // 0: transposed D-, 1: transposed D+
            for (int a = 0; a < 3; ++a) {
                const std::vector<double> &c = kind == 0 ? m->cm[a] : m->cp[a];
                const int n = m->np[a];
                off.push_back(t.size());
                for (int q = 0; q < n; ++q)
                    for (int mm = 0; mm < L; ++mm) {
                        // row q of the transpose: source row q - r + 1 + mm (D-) or q - r + mm (D+)
                        const int row = kind == 0 ? q - r + 1 + mm : q - r + mm;
                        t.push_back(row >= r && row <= n - 1 - r ? (float)c[(size_t)row * L + (L - 1 - mm)] : 0.f);
                    }
            }
        if ((st = ensure(m, m->tabT, t.size() * sizeof(float))) != EMM_OK) return st;
        HIP_OK(m, hipMemcpy(m->tabT.p, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    const float *tT = (const float *)m->tabT.p;
    const float *cmT[3] = {tT, tT + (size_t)n1 * L, tT + (size_t)(n1 + n2) * L};
    const float *cpT[3] = {tT + (size_t)(n1 + n2 + n3) * L, tT + (size_t)(2 * n1 + n2 + n3) * L,
                           tT + (size_t)(2 * n1 + 2 * n2 + n3) * L};
    // CPML tables concatenated per kind [x | y | z]
    {
        std::vector<float> c;
        // fetch the per-axis tables of this forward back from the device buffer
        std::vector<float> all((n1 + n2 + n3) * 4);
        HIP_OK(m, hipMemcpy(all.data(), m->cpml.p, all.size() * sizeof(float), hipMemcpyDeviceToHost));
        // device layout: axis a: a_int, b_int, a_half, b_half (each n_a)
        size_t o = 0;
        const int nn[3] = {n1, n2, n3};
        size_t base[3];
        for (int a = 0; a < 3; ++a) {
            base[a] = o;
            o += 4 * (size_t)nn[a];
        }
        for (int kind = 0; kind < 4; ++kind)
            for (int a = 0; a < 3; ++a)
                for (int i = 0; i < nn[a]; ++i) c.push_back(all[base[a] + (size_t)kind * nn[a] + i]);
        if ((st = ensure(m, m->adjcpml, c.size() * sizeof(float))) != EMM_OK) return st;
        HIP_OK(m, hipMemcpy(m->adjcpml.p, c.data(), c.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    const float *acp = (const float *)m->adjcpml.p;
    const size_t nsum = (size_t)n1 + n2 + n3;
    // slab arrays per source: x [n3][n2][2nb], y [n3][2nb][pitch], z [2nb][n2][pitch]
    const long long sxs = nb ? (long long)n3 * n2 * 2 * nb : 0;
    const long long sys = nb ? (long long)n3 * 2 * nb * m->pitch : 0;
    const long long szs = nb ? (long long)2 * nb * plane : 0;
    const long long slab_src = 2 * (sxs + sys + szs);          // 6 arrays
    if ((st = ensure(m, m->adjf, (size_t)6 * nsrc * fstride * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->adjq, (size_t)std::max<long long>(1, 2 * nsrc * slab_src) * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->adjt, (size_t)std::max<long long>(1, nsrc * slab_src) * sizeof(float))) != EMM_OK) return st;
    if ((st = ensure(m, m->snaps, (size_t)(cin + 1) * 3 * nsrc * fstride * sizeof(float))) != EMM_OK) return st;
    if (cin < ckpt &&
        (st = ensure(m, m->ickpts, (size_t)((ckpt + cin - 1) / cin) * state_floats(m) * nsrc * sizeof(float))) != EMM_OK)
        return st;
    if ((st = ensure(m, m->grad, (size_t)3 * nsrc * fstride * sizeof(double))) != EMM_OK) return st;
    if ((st = ensure(m, m->grad32, (size_t)3 * nsrc * fstride * sizeof(float))) != EMM_OK) return st;
    HIP_OK(m, hipMemsetAsync(m->adjf.p, 0, (size_t)6 * nsrc * fstride * sizeof(float), stream));
    if (nb) HIP_OK(m, hipMemsetAsync(m->adjq.p, 0, (size_t)2 * nsrc * slab_src * sizeof(float), stream));
    HIP_OK(m, hipMemsetAsync(m->grad.p, 0, (size_t)3 * nsrc * fstride * sizeof(double), stream));
    HIP_OK(m, hipMemsetAsync(m->grad32.p, 0, (size_t)3 * nsrc * fstride * sizeof(float), stream));

    // receiver injection lists (CSR over target cells, fixed order): E channels
    // target Et (scaled by dt/eps), H channels target Hb; rebuilt only when the
    // receiver items change
    emm_model::InjCache &ic = m->injc;
    const bool inj_cached = ic.valid && ic.nsrc == nsrc && ic.fstride == fstride && ic.base == m->inj.p &&
                            ic.items_e == A.items_hstep && ic.items_h == A.items_estep && ic.w_e == A.w_hstep &&
                            ic.w_h == A.w_estep;
    if ((st = ensure(m, m->injA, nd * sizeof(double2))) != EMM_OK) return st;
    HIP_OK(m, hipMemcpy(m->injA.p, Acoef.data(), nd * sizeof(double2), hipMemcpyHostToDevice));
    if (!inj_cached) {
        ic.valid = false;
        std::vector<int> rowE, rowH, itE, itH, compE, compH;
        std::vector<float> wE, wH;
        std::vector<long long> cellE, cellH, mcE, mcH;
        for (int kind = 0; kind < 2; ++kind) {            // 0: E channels (items_hstep), 1: H channels
            const std::vector<int> &items = kind == 0 ? A.items_hstep : A.items_estep;
            const std::vector<float> &wts = kind == 0 ? A.w_hstep : A.w_estep;
            std::vector<std::pair<long long, std::pair<int, float>>> ent;  // (target key, (slot, weight))
            const int nit = (int)items.size() / 6;
            for (int q = 0; q < nit; ++q) {
                const int *inf = &items[6 * q];
                const int s = inf[0], f = inf[1], bx = inf[2], by = inf[3], bz = inf[4], slot = inf[5];
                const float *w = &wts[(size_t)3 * L * q];
                for (int c3 = 0; c3 < L; ++c3)
                    for (int b = 0; b < L; ++b)
                        for (int a = 0; a < L; ++a) {
                            const long long mc = (long long)(bz + c3) * plane + (long long)(by + b) * m->pitch + bx + a;
                            const long long key = ((long long)f * nsrc + s) * fstride + mc;
                            ent.push_back({key, {slot, w[a] * w[L + b] * w[2 * L + c3]}});
                        }
            }
            std::stable_sort(ent.begin(), ent.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
            std::vector<int> &row = kind == 0 ? rowE : rowH;
            std::vector<int> &it = kind == 0 ? itE : itH;
            std::vector<int> &cp_ = kind == 0 ? compE : compH;
            std::vector<float> &ww = kind == 0 ? wE : wH;
            std::vector<long long> &cell = kind == 0 ? cellE : cellH;
            std::vector<long long> &mcell = kind == 0 ? mcE : mcH;
            for (size_t e = 0; e < ent.size(); ++e) {
                if (e == 0 || ent[e].first != ent[e - 1].first) {
                    row.push_back((int)it.size());
                    const long long key = ent[e].first;
                    const int f = (int)(key / ((long long)nsrc * fstride));
                    cp_.push_back(f);
                    cell.push_back(key - (long long)f * nsrc * fstride);    // within the component array
                    mcell.push_back(key % fstride);
                }
                it.push_back(ent[e].second.first);
                ww.push_back(ent[e].second.second);
            }
            row.push_back((int)it.size());
        }
        // one device buffer for both lists
        auto bytes_of = [](const auto &v) { return v.size() * sizeof(v[0]); };
        const size_t inj_bytes = bytes_of(rowE) + bytes_of(rowH) + bytes_of(itE) + bytes_of(itH) + bytes_of(wE) +
                                 bytes_of(wH) + bytes_of(cellE) + bytes_of(cellH) + bytes_of(mcE) + bytes_of(mcH) +
                                 bytes_of(compE) + bytes_of(compH) + 16 * 12;
        if ((st = ensure(m, m->inj, inj_bytes)) != EMM_OK) return st;
        char *ip = (char *)m->inj.p;
        size_t io = 0;
        auto up = [&](const auto &v) -> const void * {
            io = (io + 15) / 16 * 16;
            void *d = ip + io;
            if (!v.empty()) (void)hipMemcpy(d, v.data(), bytes_of(v), hipMemcpyHostToDevice);
            io += bytes_of(v);
            return d;
        };
        ic.ncells[0] = (int)cellE.size();
        ic.ncells[1] = (int)cellH.size();
        ic.ptr[0] = up(rowE);
        ic.ptr[1] = up(itE);
        ic.ptr[2] = up(wE);
        ic.ptr[3] = up(cellE);
        ic.ptr[4] = up(mcE);
        ic.ptr[5] = up(compE);
        ic.ptr[6] = up(rowH);
        ic.ptr[7] = up(itH);
        ic.ptr[8] = up(wH);
        ic.ptr[9] = up(cellH);
        ic.ptr[10] = up(mcH);
        ic.ptr[11] = up(compH);
        HIP_OK(m, hipDeviceSynchronize());       // the host lists die with this block
        ic.items_e = A.items_hstep;
        ic.items_h = A.items_estep;
        ic.w_e = A.w_hstep;
        ic.w_h = A.w_estep;
        ic.nsrc = nsrc;
        ic.fstride = fstride;
        ic.base = m->inj.p;
        ic.valid = true;
    }
    float *AF = (float *)m->adjf.p;
    float *Et[3] = {AF, AF + (size_t)nsrc * fstride, AF + (size_t)2 * nsrc * fstride};
    float *Hb[3] = {AF + (size_t)3 * nsrc * fstride, AF + (size_t)4 * nsrc * fstride, AF + (size_t)5 * nsrc * fstride};
    emm::InjectParams IE{}, IH{};
    IE.ncells = ic.ncells[0];
    IE.nf = A.nf;
    IE.row = (const int *)ic.ptr[0];
    IE.item = (const int *)ic.ptr[1];
    IE.w = (const float *)ic.ptr[2];
    IE.cell = (const long long *)ic.ptr[3];
    IE.mcell = (const long long *)ic.ptr[4];
    IE.comp = (const int *)ic.ptr[5];
    IE.A = (const double2 *)m->injA.p;
    IE.phase = A.Ph.phase;                    // E stamps (n + 1) dt
    IE.F1 = Et[0];
    IE.F2 = Et[1];
    IE.F3 = Et[2];
    IE.ce1 = m->ce[0];
    IE.ce2 = m->ce[1];
    IE.ce3 = m->ce[2];
    IE.scale_ce = 1;
    IH = IE;
    IH.ncells = ic.ncells[1];
    IH.row = (const int *)ic.ptr[6];
    IH.item = (const int *)ic.ptr[7];
    IH.w = (const float *)ic.ptr[8];
    IH.cell = (const long long *)ic.ptr[9];
    IH.mcell = (const long long *)ic.ptr[10];
    IH.comp = (const int *)ic.ptr[11];
    IH.phase = A.Pe.phase;                    // H stamps (n + 1/2) dt
    IH.F1 = Hb[0];
    IH.F2 = Hb[1];
    IH.F3 = Hb[2];
    IH.scale_ce = 0;

    // adjoint gather parameters
    float *AQ = (float *)m->adjq.p, *AT_ = (float *)m->adjt.p;
    auto slab_ptrs = [&](float *base, float **out) {
        // [x0 x1 | y0 y1 | z0 z1], each nsrc * stride
        out[0] = base;
        out[1] = base + nsrc * sxs;
        out[2] = base + 2 * nsrc * sxs;
        out[3] = base + 2 * nsrc * sxs + nsrc * sys;
        out[4] = base + 2 * nsrc * sxs + 2 * nsrc * sys;
        out[5] = base + 2 * nsrc * sxs + 2 * nsrc * sys + nsrc * szs;
    };
    emm::AdjParams PE{}, PH{};               // PE: reverse of the H update (-> Et), PH: of the E update (-> Hb)
    PE.n1 = n1;
    PE.n2 = n2;
    PE.n3 = n3;
    PE.pitch = m->pitch;
    PE.r = r;
    PE.nb = nb;
    PE.nsrc = nsrc;
    // z chunks and tile width of the forward kernels; the gathers' tiles are
    // one row per wavefront (tw x 256/tw columns), whatever rows per
    // wavefront the forward kernels used
    emm::StepParams gt{};
    set_tiles(gt, m, A.Pe.tx, 1);
    PE.kz = A.Pe.kz;
    PE.tw = gt.tx;
    PE.xt = gt.xt;
    PE.yt = gt.yt;
    PE.zc = A.Pe.zc;
    PE.sorder = A.Pe.sorder;
    PE.nstencil = PE.xt * PE.yt * PE.zc * nsrc;
    PE.fstride = fstride;
    PE.ce1 = m->ce[0];
    PE.ce2 = m->ce[1];
    PE.ce3 = m->ce[2];
    PE.cei = A.Pe.cei;                        // compact dt/eps when the forward used it
    PE.cet = m->cet;
    PE.ncet = m->ncet;
    PE.a_int = acp;
    PE.b_int = acp + nsum;
    PE.a_half = acp + 2 * nsum;
    PE.b_half = acp + 3 * nsum;
    PE.sxs = sxs;
    PE.sys = sys;
    PE.szs = szs;
    PE.gstride = fstride;
    PE.grad = (double *)m->grad.p;
    PE.grad32 = (float *)m->grad32.p;
    PH = PE;
    PE.in1 = Hb[0];
    PE.in2 = Hb[1];
    PE.in3 = Hb[2];
    PE.out1 = Et[0];
    PE.out2 = Et[1];
    PE.out3 = Et[2];
    PE.scale = (float)(m->dt / kMu0);
    PE.tx = cpT[0];
    PE.ty = cpT[1];
    PE.tz = cpT[2];
    slab_ptrs(AQ, PE.Q);
    slab_ptrs(AT_, PE.T);
    PH.in1 = Et[0];
    PH.in2 = Et[1];
    PH.in3 = Et[2];
    PH.out1 = Hb[0];
    PH.out2 = Hb[1];
    PH.out3 = Hb[2];
    PH.scale = 1.0f;
    PH.tx = cmT[0];
    PH.ty = cmT[1];
    PH.tz = cmT[2];
    slab_ptrs(AQ + nsrc * slab_src, PH.Q);
    slab_ptrs(AT_, PH.T);

    // forward recompute parameters: no receiver DTFT
    emm::StepParams Pe = A.Pe, Ph = A.Ph;
    Pe.nrecblk = Ph.nrecblk = 0;
    Pe.nitems = Ph.nitems = 0;
    float *snap = (float *)m->snaps.p;
    const size_t snap_bytes = (size_t)3 * nsrc * fstride * sizeof(float);
    // one segment [n0, nend) from checkpoint c of buffer `base`: recompute it
    // with the E step writing out of place into the next snapshot slot (so E
    // after every step is kept without copies), then reverse its steps
    auto reverse_segment = [&](void *base, int c, int n0, int nend) -> emm_status {
        emm_status s2;
        if ((s2 = copy_state(m, base, c, false, stream)) != EMM_OK) return s2;
        HIP_OK(m, hipMemcpyAsync(snap, m->fields.p, snap_bytes, hipMemcpyDeviceToDevice, stream));
        const size_t cs = (size_t)nsrc * fstride;               // component stride
        for (int n = n0; n < nend; ++n) {
            float *Ein = snap + (size_t)(n - n0) * 3 * cs, *Eout = snap + (size_t)(n - n0 + 1) * 3 * cs;
            emm::StepParams Pr = Pe, Qr = Ph;
            Pr.E1 = Ein;
            Pr.E2 = Ein + cs;
            Pr.E3 = Ein + 2 * cs;
            Pr.Eo1 = Qr.E1 = Qr.Eo1 = Eout;
            Pr.Eo2 = Qr.E2 = Qr.Eo2 = Eout + cs;
            Pr.Eo3 = Qr.E3 = Qr.Eo3 = Eout + 2 * cs;
            emm::launch_e_step(r, Pr, n, stream);
            emm::launch_h_step(r, Qr, n, stream);
        }
        for (int n = nend - 1; n >= n0; --n) {
            if (nb) emm::launch_adj_filter(true, PE, stream);
            emm::launch_adj_tile(r, true, PE, stream);
            emm::launch_adj_inject(IE, n, stream);
            PH.E_next = snap + (size_t)(n - n0 + 1) * 3 * nsrc * fstride;
            PH.E_prev = snap + (size_t)(n - n0) * 3 * nsrc * fstride;
            if (nb) emm::launch_adj_filter(false, PH, stream);
            emm::launch_adj_tile(r, false, PH, stream);
            emm::launch_adj_inject(IH, n, stream);
            // FP32 partial gradient sums cover the steps down to a multiple
            // of kFlush: the same steps under every checkpoint schedule
            if (n % kFlush == 0) emm::launch_adj_flush(PH, stream);
        }
        HIP_OK(m, hipGetLastError());
        return EMM_OK;
    };
    const int nseg = (nt + ckpt - 1) / ckpt;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int n0 = sgi * ckpt, nend = std::min(n0 + ckpt, nt);
        if (cin >= ckpt) {
            if ((st = reverse_segment(m->ckpts.p, sgi, n0, nend)) != EMM_OK) return st;
            continue;
        }
        // two levels: re-run the outer segment once, laying inner checkpoints
        const int nq = (nend - n0 + cin - 1) / cin;
        if ((st = copy_state(m, m->ckpts.p, sgi, false, stream)) != EMM_OK) return st;
        for (int q = 0; q < nq; ++q) {
            if ((st = copy_state(m, m->ickpts.p, q, true, stream)) != EMM_OK) return st;
            if (q == nq - 1) break;
            for (int n = n0 + q * cin; n < n0 + (q + 1) * cin; ++n) {
                emm::launch_e_step(r, Pe, n, stream);
                emm::launch_h_step(r, Ph, n, stream);
            }
        }
        for (int q = nq - 1; q >= 0; --q)
            if ((st = reverse_segment(m->ickpts.p, q, n0 + q * cin, std::min(n0 + (q + 1) * cin, nend))) != EMM_OK)
                return st;
    }
    // sum over sources, drop the pitch padding, fold the model padding back onto
    // the input cells, and change sign: d/d log sigma = -d/d log(dt/eps); on
    // the device (the running sum over source groups stays there), then one
    // copy of the input-cell gradient to the caller
    const int nd0 = m->n[0], nd1 = m->n[1], nd2 = m->n[2];
    const size_t nout = (size_t)3 * nd0 * nd1 * nd2;
    if ((st = ensure(m, m->gsum, nout * sizeof(double))) != EMM_OK) return st;
    emm::launch_adj_fold((const double *)m->grad.p, (double *)m->gsum.p, nsrc, fstride, plane, m->pitch, n1, n2,
                         n3, r, m->nbe, nd0, nd1, nd2, accumulate, stream);
    HIP_OK(m, hipGetLastError());
    HIP_OK(m, hipMemcpyAsync(grad, m->gsum.p, nout * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(m, hipStreamSynchronize(stream));
    return EMM_OK;
}

// Sources per forward + reverse sweep of emm_gradient: the src_group option,
// else (0) the most sources whose checkpoints fit one level (a second level
// costs one more forward pass, batching saves a few per cent), else the most
// that fit two levels; all of them with a fixed checkpoint interval.
int gradient_group(emm_model *m, int nsrc, int nt) {
    if (m->opt.src_group > 0) return std::min(m->opt.src_group, nsrc);
    if (m->opt.src_group < 0 || m->opt.checkpoint_every > 0) return nsrc;
    const long long fs = (long long)m->pitch * m->np[1] * m->np[2];
    int two = 0;
    for (int g = nsrc; g >= 1; --g) {
        size_t bud = 0;
        if (ckpt_budget(m, g, bud) != EMM_OK) return nsrc;
        int c1 = 0, c2 = 0;
        const size_t S = state_floats(m) * g * sizeof(float), F = (size_t)3 * g * fs * sizeof(float);
        if (!plan_checkpoints(nt, m->opt.graph_steps, 0, m->opt.checkpoint_inner, S, F, bud, c1, c2)) continue;
        if (c2 >= c1) return g;
        if (!two) two = g;
    }
    return two ? two : 1;
}

emm_status emm_gradient(emm_model *m, const emm_source *src, int nsrc, const emm_receiver *rec,
                        int nrec, unsigned chan_mask, const double *freq_hz, int nfreq,
                        const double *g_obs, const double *g_bar, double *green, double *misfit,
                        double *grad, void *hip_stream) {
    if (!m) return fail(nullptr, EMM_ERR_ARG, "NULL model");
    m->err.clear();
    if (!grad || (g_obs == nullptr) == (g_bar == nullptr))
        return fail(m, EMM_ERR_ARG, "need grad and exactly one of g_obs, g_bar");
    if (m->opt.airwave) return fail(m, EMM_ERR_ARG, "the adjoint of the air boundary is not built");
    if (m->opt.converge_tol > 0.0) return fail(m, EMM_ERR_ARG, "the gradient needs a fixed step count (converge_tol = 0)");
    hipStream_t stream = hip_stream ? (hipStream_t)hip_stream : m->own_stream;
    emm_status st;
    double chi = 0.0;
    // the checkpoints of the last forward serve only the same acquisition in one sweep
    const bool reuse = m->acq.ckpt > 0 && same_acquisition(m->acq, src, nsrc, rec, nrec, chan_mask, freq_hz, nfreq);
    bool freqs_ok = freq_hz && nfreq > 0;
    for (int f = 0; freqs_ok && f < nfreq; ++f) freqs_ok = freq_hz[f] > 0.0 && std::isfinite(freq_hz[f]);
    const int g = (!reuse && src && nsrc > 1 && freqs_ok) ? gradient_group(m, nsrc, steps_for(m, freq_hz, nfreq))
                                                          : nsrc;
    if (g < nsrc)
        for (int s = 0; s < nsrc; ++s)
            if ((st = check_source(m, src[s])) != EMM_OK) return st;
    const size_t per_src = (size_t)nrec * __builtin_popcount(chan_mask & 0x3Fu) * (nfreq > 0 ? nfreq : 0) * 2;
    for (int g0 = 0; g0 < nsrc || g0 == 0; g0 += std::max(g, 1)) {
        const int ng = std::min(g, nsrc - g0);
        const size_t o = (size_t)g0 * per_src;
        if ((st = gradient_run(m, src ? src + g0 : src, ng, rec, nrec, chan_mask, freq_hz, nfreq,
                               g_obs ? g_obs + o : nullptr, g_bar ? g_bar + o : nullptr, green ? green + o : nullptr,
                               chi, grad, g0 > 0, stream)) != EMM_OK)
            return st;
    }
    if (misfit) *misfit = chi;
    m->info.src_group = g;
    return EMM_OK;
}

}  // extern "C"
