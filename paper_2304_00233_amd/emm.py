"""Thin ctypes binding of the libemm C ABI (include/emm.h).

Argument marshalling only: every step of the modelling runs in the HIP
library.  The names mirror the C functions; `forward_workload` is a
convenience that takes a workload object (grid, model, acquisition,
options) and returns the Green's functions as complex128
[nsrc][nrec][nchan][nfreq].  If the compiled library is missing this module
raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# EMM_LIBRARY may point at another build of the same ABI (e.g. an older
# kernel version for an A/B timing); default: the in-tree build.
LIB_PATH = os.environ.get("EMM_LIBRARY") or os.path.join(_HERE, "libemm.so")

EMM_OK = 0
STATUS = {0: "EMM_OK", -1: "EMM_ERR_ARG", -2: "EMM_ERR_GRID", -3: "EMM_ERR_MODEL",
          -4: "EMM_ERR_GEOMETRY", -5: "EMM_ERR_FREQ", -6: "EMM_ERR_CFL",
          -7: "EMM_ERR_NONFINITE", -8: "EMM_ERR_OOM", -9: "EMM_ERR_DEVICE"}
EXPORTED = ("emm_default_options", "emm_create", "emm_query", "emm_forward",
            "emm_forward_noalloc", "emm_forward_batch", "emm_gradient", "emm_destroy",
            "emm_status_str", "emm_last_error")

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


class emm_grid(C.Structure):
    _fields_ = [("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int),
                ("x1", _dp), ("x2", _dp), ("x3", _dp),
                ("rho11", _fp), ("rho22", _fp), ("rho33", _fp)]


class emm_options(C.Structure):
    _fields_ = [("rd", C.c_int), ("nb", C.c_int), ("ne", C.c_int),
                ("f0", C.c_double), ("cfl", C.c_double), ("dt_override", C.c_double),
                ("nt", C.c_int), ("dft_mode", C.c_int),
                ("cpml_R", C.c_double), ("cpml_npow", C.c_double),
                ("cpml_alpha_max", C.c_double), ("wavelet_fpeak", C.c_double),
                ("allow_unstable", C.c_int), ("profile", C.c_int), ("tile_kz", C.c_int),
                ("checkpoint_every", C.c_int), ("graph_steps", C.c_int),
                ("checkpoint_inner", C.c_int), ("nontemporal", C.c_int), ("airwave", C.c_int),
                ("converge_tol", C.c_double), ("converge_every", C.c_int), ("fused", C.c_int),
                ("ce_table", C.c_int), ("src_group", C.c_int), ("tile_x", C.c_int),
                ("tile_rows", C.c_int), ("src_order", C.c_int)]


class emm_source(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double),
                ("comp", C.c_int), ("moment", C.c_double)]


class emm_receiver(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double)]


class emm_job(C.Structure):
    _fields_ = [("model", C.c_void_p), ("src", C.POINTER(emm_source)), ("nsrc", C.c_int),
                ("rec", C.POINTER(emm_receiver)), ("nrec", C.c_int), ("chan_mask", C.c_uint),
                ("freq_hz", _dp), ("nfreq", C.c_int), ("green", _dp)]


class emm_info(C.Structure):
    _fields_ = [("dt", C.c_double), ("nt", C.c_int),
                ("n1pad", C.c_int), ("n2pad", C.c_int), ("n3pad", C.c_int),
                ("cells", C.c_longlong), ("bytes_per_step", C.c_double),
                ("e_bytes", C.c_double), ("h_bytes", C.c_double),
                ("e_kernel_ms", C.c_double), ("h_kernel_ms", C.c_double),
                ("e_launches", C.c_longlong), ("h_launches", C.c_longlong),
                ("forward_ms", C.c_double), ("tile_kz", C.c_int),
                ("ckpt_outer", C.c_int), ("ckpt_inner", C.c_int), ("ckpt_bytes", C.c_double),
                ("nontemporal", C.c_int), ("converged", C.c_int), ("fused", C.c_int),
                ("leap_bytes", C.c_double), ("ce_table", C.c_int), ("src_group", C.c_int),
                ("tile_x", C.c_int), ("tile_rows", C.c_int), ("src_order", C.c_int),
                ("air_transform", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libemm is not built ({LIB_PATH} missing): run "
                          "`python -m paper_2304_00233_amd.build` (or __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    lib.emm_default_options.argtypes = [C.POINTER(emm_options)]
    lib.emm_default_options.restype = C.c_int
    lib.emm_create.argtypes = [C.POINTER(emm_grid), C.POINTER(emm_options), C.POINTER(C.c_void_p)]
    lib.emm_create.restype = C.c_int
    lib.emm_query.argtypes = [C.c_void_p, C.POINTER(emm_info)]
    lib.emm_query.restype = C.c_int
    lib.emm_forward.argtypes = [C.c_void_p, C.POINTER(emm_source), C.c_int,
                                C.POINTER(emm_receiver), C.c_int, C.c_uint, _dp, C.c_int,
                                _dp, C.c_void_p]
    lib.emm_forward.restype = C.c_int
    lib.emm_forward_noalloc.argtypes = lib.emm_forward.argtypes
    lib.emm_forward_noalloc.restype = C.c_int
    lib.emm_forward_batch.argtypes = [C.POINTER(emm_job), C.c_int, C.c_int, C.c_void_p]
    lib.emm_forward_batch.restype = C.c_int
    lib.emm_gradient.argtypes = [C.c_void_p, C.POINTER(emm_source), C.c_int,
                                 C.POINTER(emm_receiver), C.c_int, C.c_uint, _dp, C.c_int,
                                 _dp, _dp, _dp, _dp, _dp, C.c_void_p]
    lib.emm_gradient.restype = C.c_int
    lib.emm_destroy.argtypes = [C.c_void_p]
    lib.emm_destroy.restype = None
    lib.emm_status_str.argtypes = [C.c_int]
    lib.emm_status_str.restype = C.c_char_p
    lib.emm_last_error.argtypes = [C.c_void_p]
    lib.emm_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def hip_runtimes() -> list:
    """Paths of the HIP runtime libraries (libamdhip64) mapped into this
    process.  libemm binds to the first one loaded: a process that imports
    torch before this module shares torch's runtime with it (one entry here);
    importing this module first and torch afterwards maps two."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return sorted(paths)


class EmmError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


def _check(status: int, model=None):
    if status != EMM_OK:
        raise EmmError(status, emm_last_error(model))


# ---------------------------------------------------------------- 1:1 names
def emm_default_options() -> emm_options:
    o = emm_options()
    _check(_lib.emm_default_options(C.byref(o)))
    return o


def emm_status_str(status: int) -> str:
    return _lib.emm_status_str(status).decode()


def emm_last_error(model=None) -> str:
    return (_lib.emm_last_error(model) or b"").decode()


def emm_create(x1, x2, x3, rho11, rho22, rho33, opts: emm_options):
    """Returns an opaque model handle (c_void_p).  Arrays are copied."""
    xs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x1, x2, x3)]
    rs = [np.ascontiguousarray(a, dtype=np.float32) for a in (rho11, rho22, rho33)]
    n1, n2, n3 = (len(a) for a in xs)
    for r in rs:
        if r.shape != (n3, n2, n1):
            raise ValueError(f"resistivity shape {r.shape} != (n3, n2, n1) = {(n3, n2, n1)}")
    g = emm_grid(n1, n2, n3, *(a.ctypes.data_as(_dp) for a in xs),
                 *(a.ctypes.data_as(_fp) for a in rs))
    h = C.c_void_p()
    _check(_lib.emm_create(C.byref(g), C.byref(opts), C.byref(h)))
    return h


def emm_query(model) -> emm_info:
    info = emm_info()
    _check(_lib.emm_query(model, C.byref(info)), model)
    return info


def emm_forward(model, sources, receivers, chan_mask: int, freqs, src_comp=None,
                moments=None, stream=None, noalloc: bool = False) -> np.ndarray:
    """sources [nsrc][3], receivers [nrec][3] in metres; returns complex128
    [nsrc][nrec][popcount(chan_mask)][nfreq].  noalloc: call
    emm_forward_noalloc (per-call buffers in the library's static device
    workspace) instead of emm_forward."""
    sources = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    receivers = np.atleast_2d(np.asarray(receivers, dtype=np.float64))
    freqs = np.ascontiguousarray(freqs, dtype=np.float64)
    ns, nr, nf = len(sources), len(receivers), len(freqs)
    comp = np.zeros(ns, dtype=np.int32) if src_comp is None else np.asarray(src_comp)
    mom = np.ones(ns) if moments is None else np.asarray(moments, dtype=np.float64)
    S = (emm_source * max(ns, 1))(*[emm_source(*sources[i], int(comp[i]), float(mom[i]))
                                    for i in range(ns)])
    R = (emm_receiver * max(nr, 1))(*[emm_receiver(*receivers[i]) for i in range(nr)])
    nch = bin(chan_mask & 0x3F).count("1")
    out = np.zeros(2 * max(ns, 1) * max(nr, 1) * max(nch, 1) * max(nf, 1))
    fn = _lib.emm_forward_noalloc if noalloc else _lib.emm_forward
    _check(fn(model, S, ns, R, nr, C.c_uint(chan_mask), freqs.ctypes.data_as(_dp), nf,
              out.ctypes.data_as(_dp), stream), model)
    g = out[0::2] + 1j * out[1::2]
    return g.reshape(ns, nr, nch, nf)


def _acq(sources, receivers, freqs, src_comp, moments):
    sources = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    receivers = np.atleast_2d(np.asarray(receivers, dtype=np.float64))
    freqs = np.ascontiguousarray(freqs, dtype=np.float64)
    ns, nr = len(sources), len(receivers)
    comp = np.zeros(ns, dtype=np.int32) if src_comp is None else np.asarray(src_comp)
    mom = np.ones(ns) if moments is None else np.asarray(moments, dtype=np.float64)
    S = (emm_source * max(ns, 1))(*[emm_source(*sources[i], int(comp[i]), float(mom[i]))
                                    for i in range(ns)])
    R = (emm_receiver * max(nr, 1))(*[emm_receiver(*receivers[i]) for i in range(nr)])
    return S, ns, R, nr, freqs


def emm_gradient(model, shape, sources, receivers, chan_mask: int, freqs, g_obs=None,
                 g_bar=None, src_comp=None, moments=None, stream=None):
    """Discrete-adjoint gradient (see emm.h).  shape = (n1, n2, n3) of the
    model; g_obs or g_bar complex [nsrc][nrec][nchan][nfreq].  Returns
    (grad[3][n3][n2][n1] = dL/d log sigma, G, misfit)."""
    S, ns, R, nr, freqs = _acq(sources, receivers, freqs, src_comp, moments)
    nf = len(freqs)
    nch = bin(chan_mask & 0x3F).count("1")
    n1, n2, n3 = shape

    def pack(z):
        if z is None:
            return None
        z = np.asarray(z, dtype=np.complex128).reshape(-1)
        out = np.empty(2 * z.size)
        out[0::2], out[1::2] = z.real, z.imag
        return out
    go, gb = pack(g_obs), pack(g_bar)
    green = np.zeros(2 * ns * nr * nch * nf)
    grad = np.zeros(3 * n1 * n2 * n3)
    mis = C.c_double(0.0)
    _check(_lib.emm_gradient(model, S, ns, R, nr, C.c_uint(chan_mask), freqs.ctypes.data_as(_dp),
                             nf, go.ctypes.data_as(_dp) if go is not None else None,
                             gb.ctypes.data_as(_dp) if gb is not None else None,
                             green.ctypes.data_as(_dp), C.byref(mis), grad.ctypes.data_as(_dp),
                             stream), model)
    G = (green[0::2] + 1j * green[1::2]).reshape(ns, nr, nch, nf)
    return grad.reshape(3, n3, n2, n1), G, mis.value


def emm_forward_batch(jobs, graph_steps: int = 64, stream=None) -> list:
    """jobs: sequence of (model handle, sources, receivers, chan_mask, freqs,
    src_comp or None); all jobs run in one captured hipGraph (see emm.h).
    Returns one complex128 [nsrc][nrec][nchan][nfreq] array per job."""
    keep, outs, shapes = [], [], []
    J = (emm_job * len(jobs))()
    for j, (h, sources, receivers, chan_mask, freqs, src_comp) in enumerate(jobs):
        S, ns, R, nr, fr = _acq(sources, receivers, freqs, src_comp, None)
        nch = bin(chan_mask & 0x3F).count("1")
        out = np.zeros(2 * max(ns, 1) * max(nr, 1) * max(nch, 1) * max(len(fr), 1))
        keep += [S, R, fr]
        outs.append(out)
        shapes.append((ns, nr, nch, len(fr)))
        J[j] = emm_job(h, C.cast(S, C.POINTER(emm_source)), ns, C.cast(R, C.POINTER(emm_receiver)),
                       nr, C.c_uint(chan_mask), fr.ctypes.data_as(_dp), len(fr),
                       out.ctypes.data_as(_dp))
    st = _lib.emm_forward_batch(J, len(jobs), graph_steps, stream)
    if st != 0:
        # the failing job's model holds the detail
        detail = ""
        for h, *_ in jobs:
            detail = detail or emm_last_error(h)
        raise EmmError(st, detail)
    return [(o[0::2] + 1j * o[1::2]).reshape(sh) for o, sh in zip(outs, shapes)]


def forward_models(models, graph_steps: int = 64, stream=None) -> list:
    """Forward of several Model objects (their workloads' acquisitions) side
    by side (emm_forward_batch: each job its own stream and step graph)."""
    jobs = [(m.h, m.w.sources, m.w.receivers, m.w.chan_mask, m.w.freqs, m.w.src_comp)
            for m in models]
    return emm_forward_batch(jobs, graph_steps, stream)


def emm_destroy(model) -> None:
    _lib.emm_destroy(model)


# ------------------------------------------------------------ conveniences
def options_for(w, **overrides) -> emm_options:
    o = emm_default_options()
    o.rd, o.nb, o.ne, o.f0, o.cfl = w.rd, w.nb, w.ne, w.f0, w.cfl
    o.nt, o.dft_mode = w.nt, w.dft_mode
    o.airwave = int(getattr(w, "airwave", False))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


class Model:
    """RAII wrapper: Model(workload) creates, .forward() runs, .close() frees."""

    def __init__(self, w, **opt_overrides):
        self.w = w
        self.opts = options_for(w, **opt_overrides)
        self.h = emm_create(w.x1, w.x2, w.x3, w.rho11, w.rho22, w.rho33, self.opts)

    def forward(self, sources=None, receivers=None, freqs=None, chan_mask=None,
                src_comp=None, stream=None, noalloc: bool = False) -> np.ndarray:
        w = self.w
        return emm_forward(self.h, w.sources if sources is None else sources,
                           w.receivers if receivers is None else receivers,
                           w.chan_mask if chan_mask is None else chan_mask,
                           w.freqs if freqs is None else freqs,
                           w.src_comp if src_comp is None and sources is None else src_comp,
                           stream=stream, noalloc=noalloc)

    def gradient(self, g_obs=None, g_bar=None, sources=None, receivers=None, freqs=None,
                 chan_mask=None, src_comp=None, stream=None):
        w = self.w
        return emm_gradient(self.h, w.shape, w.sources if sources is None else sources,
                            w.receivers if receivers is None else receivers,
                            w.chan_mask if chan_mask is None else chan_mask,
                            w.freqs if freqs is None else freqs, g_obs=g_obs, g_bar=g_bar,
                            src_comp=w.src_comp if src_comp is None and sources is None else src_comp,
                            stream=stream)

    def info(self) -> dict:
        return emm_query(self.h).as_dict()

    def close(self):
        if self.h:
            emm_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward_workload(w, **opt_overrides):
    """Green's functions of every source of workload `w` plus model info."""
    with Model(w, **opt_overrides) as m:
        G = m.forward()
        return G, m.info()
