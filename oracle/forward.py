"""Oracle forward modelling: complex frequency-domain E/H Green's functions at
the receivers for a conductivity model on a rectilinear non-uniform mesh.

forward(workload) -> (G[nsrc][nrec][nchan][nfreq] complex128, info)

Call shape mirrors the C library (sources, receivers, channels and
frequencies in, Green's functions out) so tests can compare the two on the
same inputs.  Each source is an independent run (Section 5: one transmitter
per process in the paper).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import airwave as AW
from . import tables as T

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Params(C.Structure):
    _fields_ = [
        ("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int),
        ("r", C.c_int), ("nb", C.c_int), ("nt", C.c_int),
        ("ch", C.c_double),
        ("ce1", _dp), ("ce2", _dp), ("ce3", _dp),
        ("cm1", _dp), ("cm2", _dp), ("cm3", _dp),
        ("cp1", _dp), ("cp2", _dp), ("cp3", _dp),
        ("a1i", _dp), ("b1i", _dp), ("a2i", _dp), ("b2i", _dp), ("a3i", _dp), ("b3i", _dp),
        ("a1h", _dp), ("b1h", _dp), ("a2h", _dp), ("b2h", _dp), ("a3h", _dp), ("b3h", _dp),
        ("src_comp", C.c_int), ("src_base", C.c_int * 3), ("src_q", _dp),
        ("wavelet", _dp),
        ("nrec", C.c_int), ("nchan", C.c_int), ("chan", _ip),
        ("rec_base", _ip), ("rec_w", _dp),
        ("nfreq", C.c_int),
        ("phE_re", _dp), ("phE_im", _dp), ("phH_re", _dp), ("phH_im", _dp),
        ("acc_re", _dp), ("acc_im", _dp),
        ("nthreads", C.c_int),
        ("kmin", C.c_int),
        ("ghost", C.c_void_p),
        ("conv_tol", C.c_double),
        ("conv_every", C.c_int), ("conv_f", C.c_int),
        ("corner", _ip),
        ("nt_done", _ip),
        ("conv_measure", _dp),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        _lib = C.CDLL(LIB_PATH)
        _lib.oracle_run.argtypes = [C.POINTER(_Params)]
        _lib.oracle_run.restype = C.c_int
        _lib.oracle_gradient.argtypes = [C.POINTER(_Params), C.c_int, _dp, _dp, _dp]
        _lib.oracle_gradient.restype = C.c_int
        for f in (_lib.oracle_curl_h, _lib.oracle_curl_e):
            f.argtypes = [C.POINTER(_Params)] + [_dp] * 6
            f.restype = None
    return _lib


_GHOST_FN = C.CFUNCTYPE(None, C.c_int, C.POINTER(_dp))


def _ghost_callback(st: "Setup"):
    """Ghost-plane filler for the air above the surface node (Section 3.3),
    called by the stepper after each E and each H update."""
    ops = AW.make_ops(st.axes, st.nbe, st.r)
    n1, n2, n3 = st.n_pad

    def cb(which, fields):
        F = [np.ctypeslib.as_array(fields[c], shape=(n3, n2, n1)) for c in range(6)]
        if which == 0:
            AW.fill_E(F[0], F[1], ops)
        else:
            AW.fill_H(F[3], F[4], F[5], ops)
    return _GHOST_FN(cb)


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


@dataclass
class Setup:
    """Everything the time loop needs, computed once per model (Algorithm 1
    set-up phase)."""
    r: int
    nb: int
    nbe: int
    axes: tuple          # padded node coordinates
    n_pad: tuple         # (n1pad, n2pad, n3pad)
    rho: tuple           # padded resistivities
    fd: tuple            # ((cm1, cp1), (cm2, cp2), (cm3, cp3))
    dt: float
    omega0: float
    fp: float
    cpml: tuple          # per axis (a_int, b_int, a_half, b_half)
    ce: tuple            # dt/eps at E1/E2/E3


def make_setup(w, fp: float, dt_override: float = 0.0, frozen: "Setup | None" = None) -> Setup:
    """frozen: take dt and the CPML tables from this reference set-up (both
    depend on the largest resistivities; a derivative with respect to the
    model holds them fixed)."""
    r, nb = w.rd, w.nb
    nbe = w.nb + w.ne
    omega0 = 2.0 * np.pi * w.f0
    axes = tuple(T.pad_axis(x, nbe) for x in (w.x1, w.x2, w.x3))
    rho = tuple(T.pad_model(a, nbe) for a in (w.rho11, w.rho22, w.rho33))
    fd = tuple(T.fd_tables(x, r) for x in axes)
    dt = dt_override if dt_override > 0.0 else T.time_step(fd, rho, omega0, w.cfl)
    alpha_max = np.pi * fp
    cpml = []
    for a in range(3):
        v_lo, v_hi = T.slab_velocities(rho, a, nb, omega0)
        cpml.append(T.cpml_axis(axes[a], nb, dt, v_lo, v_hi, alpha_max))
    if frozen is not None:
        dt, cpml = frozen.dt, list(frozen.cpml)
    # dt * eps^-1 with eps = 1/(2 omega0 rho)  (Section 2.2: sigma = 2 omega0 eps)
    ce = tuple(np.ascontiguousarray(dt * 2.0 * omega0 * a) for a in rho)
    return Setup(r, nb, nbe, axes, tuple(len(x) for x in axes), rho, fd, dt,
                 omega0, fp, tuple(cpml), ce)


def _build_params(st: Setup, nt: int, src, comp: int, rec, chans, freqs,
                  threads: int | None = None, moment: float = 1.0):
    """ctypes parameter block for one source plus the arrays it points to."""
    r = st.r
    L = 2 * r
    n1, n2, n3 = st.n_pad
    s = T.wavelet(nt, st.dt, st.fp)
    # source stencil on the E_comp grid: J = moment * w / V  (Section 3.1)
    stag = [0, 0, 0]
    stag[comp] = 1
    sb, sw = T.point_stencil(st.axes, src, stag, r)
    if not T.inside(sb, st.n_pad, st.nbe, r):
        raise ValueError("source stencil leaves the interior")
    wt = sw[2][:, None, None] * sw[1][None, :, None] * sw[0][None, None, :]
    q = np.ascontiguousarray(moment * wt / T.dual_volume(st.axes, comp, sb, r))
    nrec, nch = len(rec), len(chans)
    rb = np.zeros((nrec, nch, 3), dtype=np.int32)
    rw = np.zeros((nrec, nch, L, L, L))
    for i, p in enumerate(rec):
        for c, ch in enumerate(chans):
            b, ww = T.point_stencil(st.axes, p, T.STAGGER[ch], r)
            if not T.inside(b, st.n_pad, st.nbe, r):
                raise ValueError("receiver stencil leaves the interior")
            rb[i, c] = b
            rw[i, c] = ww[2][:, None, None] * ww[1][None, :, None] * ww[0][None, None, :]
    phE, phH = T.dft_phases(freqs, st.omega0, st.dt, nt)
    phE_re, phE_im = np.ascontiguousarray(phE.real), np.ascontiguousarray(phE.imag)
    phH_re, phH_im = np.ascontiguousarray(phH.real), np.ascontiguousarray(phH.imag)
    nf = len(freqs)
    acc_re = np.zeros((nrec, nch, nf))
    acc_im = np.zeros((nrec, nch, nf))
    ch_arr = np.asarray(chans, dtype=np.int32)
    tabs = [np.ascontiguousarray(t) for pair in st.fd for t in pair]
    cp = [np.ascontiguousarray(t) for ax in st.cpml for t in ax]
    P = _Params()
    P.n1, P.n2, P.n3 = n1, n2, n3
    P.r, P.nb, P.nt = r, st.nb, nt
    P.ch = st.dt / T.MU0
    P.ce1, P.ce2, P.ce3 = (_ptr(a) for a in st.ce)
    P.cm1, P.cp1, P.cm2, P.cp2, P.cm3, P.cp3 = (_ptr(t) for t in tabs)
    (P.a1i, P.b1i, P.a1h, P.b1h, P.a2i, P.b2i, P.a2h, P.b2h,
     P.a3i, P.b3i, P.a3h, P.b3h) = (_ptr(t) for t in cp)
    P.src_comp = comp
    P.src_base[0], P.src_base[1], P.src_base[2] = (int(v) for v in sb)
    P.src_q = _ptr(q)
    P.wavelet = _ptr(s)
    P.nrec, P.nchan = nrec, nch
    P.chan = _ptr(ch_arr, C.c_int)
    P.rec_base = _ptr(rb, C.c_int)
    P.rec_w = _ptr(rw)
    P.nfreq = nf
    P.phE_re, P.phE_im, P.phH_re, P.phH_im = (_ptr(a) for a in (phE_re, phE_im, phH_re, phH_im))
    P.acc_re, P.acc_im = _ptr(acc_re), _ptr(acc_im)
    P.nthreads = int(threads or os.cpu_count() or 1)
    P.kmin = r
    P.ghost = None
    P.conv_tol = 0.0
    P.conv_every = 1
    keep = (tabs, cp, q, s, ch_arr, rb, rw, phE_re, phE_im, phH_re, phH_im, acc_re, acc_im)
    return P, keep, s


def corner_nodes(st: Setup) -> np.ndarray:
    """(i, j, k) of E1 at the 8 corners of the interior: first and last
    interior index on each axis (E1's x index i stands for x_{i+1/2})."""
    n1, n2, n3 = st.n_pad
    lo = (st.nbe, st.nbe, st.nbe)
    hi = (n1 - 2 - st.nbe, n2 - 1 - st.nbe, n3 - 1 - st.nbe)
    return np.array([[hi[a] if c >> a & 1 else lo[a] for a in range(3)] for c in range(8)],
                    dtype=np.int32)


def run_source(st: Setup, nt: int, src, comp: int, rec, chans, freqs,
               threads: int | None = None, moment: float = 1.0, airwave: bool = False,
               converge_tol: float = 0.0, converge_every: int = 100, report: dict | None = None):
    """Time-domain run for one source; returns the receiver DTFT
    acc[nrec][nchan][nfreq] and the source spectrum S_f (over the steps
    run).  airwave: the first interior z node is the sea surface with air
    above it.  converge_tol > 0: stop at the first check (every
    converge_every steps) where the lowest-frequency DTFT of E1 at the
    interior corners changed by at most converge_tol times its largest
    magnitude; `report` receives nt_done and the measure at each check."""
    lib = _load()
    P, keep, s = _build_params(st, nt, src, comp, rec, chans, freqs, threads, moment)
    cb = None
    if airwave:
        cb = _ghost_callback(st)
        P.kmin = st.nbe
        P.ghost = C.cast(cb, C.c_void_p)
    done = C.c_int(nt)
    corner = corner_nodes(st)
    measure = np.zeros(nt // max(1, converge_every) + 1)
    if converge_tol > 0.0:
        P.conv_tol = converge_tol
        P.conv_every = int(converge_every)
        P.conv_f = int(np.argmin(freqs))
        P.corner = _ptr(corner, C.c_int)
        P.nt_done = C.pointer(done)
        P.conv_measure = _ptr(measure)
    rc = lib.oracle_run(C.byref(P))
    del cb
    if rc < 0:
        raise MemoryError("oracle allocation failed")
    nd = done.value
    if report is not None:
        report["nt_done"] = nd
        report["measure"] = measure[:nd // max(1, converge_every)].copy()
    acc = keep[-2] + 1j * keep[-1]
    return acc, T.source_spectrum(s[:nd], freqs, st.omega0, st.dt), rc


def run_adjoint(st: Setup, nt: int, src, comp: int, rec, chans, freqs, A,
                ckpt: int = 50, threads: int | None = None):
    """Discrete adjoint of one source's run: returns d chi/d log(dt/eps_c)
    on the padded grid [3][n3][n2][n1], for a misfit whose derivative with
    respect to receiver sample u_n of item (rec, chan) is
    sum_f Re(A[rec][chan][f] exp(i w'_f t_n))."""
    lib = _load()
    P, keep, _ = _build_params(st, nt, src, comp, rec, chans, freqs, threads)
    A = np.asarray(A, dtype=np.complex128)
    a_re = np.ascontiguousarray(A.real)
    a_im = np.ascontiguousarray(A.imag)
    n1, n2, n3 = st.n_pad
    grad = np.zeros((3, n3, n2, n1))
    rc = lib.oracle_gradient(C.byref(P), int(ckpt), _ptr(a_re), _ptr(a_im), _ptr(grad))
    if rc < 0:
        raise MemoryError("oracle allocation failed")
    return grad


def fold_padding(g_pad: np.ndarray, nbe: int) -> np.ndarray:
    """Adjoint of the model extension (nearest-interior replication into the
    padding): every padded cell's value is added to the interior cell it
    copies.  [..., n3p, n2p, n1p] -> [..., n3, n2, n1]."""
    out = g_pad
    for ax in (-1, -2, -3):
        out = np.moveaxis(out, ax, 0)
        inner = out[nbe:out.shape[0] - nbe].copy()
        inner[0] += out[:nbe].sum(axis=0)
        inner[-1] += out[out.shape[0] - nbe:].sum(axis=0)
        out = np.moveaxis(inner, 0, ax)
    return out


def misfit_gradient(w, G_obs, threads: int | None = None, nt: int | None = None,
                    fpeak: float = 0.0, dt_override: float = 0.0, ckpt: int = 50,
                    frozen: Setup | None = None, with_gradient: bool = True):
    """chi = 1/2 sum over sources, receivers, channels, frequencies of
    |log(G/G_obs)|^2 (real part: log-amplitude residual, imaginary part:
    phase residual) and its gradient with respect to log sigma of every
    input cell, for each of the three staggered conductivity arrays:
    returns (chi, grad[3][n3][n2][n1], G).  dt, the step count and the CPML
    tables are held fixed (pass `frozen`, the set-up of the reference model,
    when evaluating perturbed models)."""
    if w.airwave:
        raise NotImplementedError("the adjoint of the air boundary is not built")
    freqs = np.asarray(w.freqs, dtype=np.float64)
    fp = T.peak_frequency(freqs, w.f0, fpeak)
    st = make_setup(w, fp, dt_override, frozen)
    if nt is None:
        nt = w.nt if w.nt > 0 else T.auto_nt(freqs, w.f0, st.dt, fp)
    chans = w.channels
    chi = 0.0
    g_pad = np.zeros((3,) + tuple(reversed(st.n_pad)))
    G_all = np.zeros((len(w.sources), len(w.receivers), len(chans), len(freqs)), np.complex128)
    for s_i, src in enumerate(w.sources):
        comp = int(w.src_comp[s_i])
        acc, S, _ = run_source(st, nt, src, comp, w.receivers, chans, freqs, threads)
        G = green(acc, S, freqs, st.omega0, chans)
        G_all[s_i] = G
        r = np.log(G / G_obs[s_i])
        chi += 0.5 * float(np.sum(np.abs(r) ** 2))
        # d chi/d u_n = Re(sum_f conj(r_f) / acc_f * exp(i w'_f t_n))
        if with_gradient:
            A = np.conj(r) / acc
            g_pad += run_adjoint(st, nt, src, comp, w.receivers, chans, freqs, A, ckpt, threads)
    # d/d log(dt/eps) = d/d log rho = -d/d log sigma
    return chi, -fold_padding(g_pad, st.nbe), G_all


def green(acc, S, freqs, omega0, chans, moment: float = 1.0):
    """G^EE = (omega/omega') E'/J',  G^HE = H'/J'  (eq. greenfunction, with
    sqrt(-i omega/2 omega0) = omega/omega' on the principal branch), per unit
    moment: J' = moment * S_f."""
    wp = T.omega_prime(freqs, omega0)
    w = 2.0 * np.pi * np.asarray(freqs)
    G = acc / (moment * S[None, None, :])
    for c, ch in enumerate(chans):
        if ch < 3:
            G[:, c, :] *= (w / wp)[None, :]
    return G


def forward(w, threads: int | None = None, nt: int | None = None,
            fpeak: float = 0.0, dt_override: float = 0.0, converge_tol: float = 0.0,
            converge_every: int = 100):
    """Green's functions for every source of workload `w`:
    complex128 [nsrc][nrec][nchan][nfreq], plus an info dict.  With
    converge_tol > 0 each source stops at its own convergence check
    (info["nt_done"] per source)."""
    freqs = np.asarray(w.freqs, dtype=np.float64)
    fp = T.peak_frequency(freqs, w.f0, fpeak)
    st = make_setup(w, fp, dt_override)
    if nt is None:
        nt = w.nt if w.nt > 0 else T.auto_nt(freqs, w.f0, st.dt, fp)
    chans = w.channels
    out = np.zeros((len(w.sources), len(w.receivers), len(chans), len(freqs)),
                   dtype=np.complex128)
    nonfinite = False
    done = []
    for s_i, src in enumerate(w.sources):
        rep = {}
        acc, S, rc = run_source(st, nt, src, int(w.src_comp[s_i]), w.receivers,
                                chans, freqs, threads, airwave=w.airwave,
                                converge_tol=converge_tol, converge_every=converge_every,
                                report=rep)
        nonfinite |= rc == 1
        done.append(rep["nt_done"])
        out[s_i] = green(acc, S, freqs, st.omega0, chans)
    info = dict(dt=st.dt, nt=nt, n_pad=st.n_pad, fp=fp, nonfinite=nonfinite, nt_done=done)
    return out, info


def curl_apply(st: Setup, which: str, F1, F2, F3, threads: int = 1):
    """Apply the stepper's own curl (no CPML history) to given fields."""
    lib = _load()
    P = _Params()
    P.n1, P.n2, P.n3 = st.n_pad
    P.r, P.nb = st.r, 0
    tabs = [np.ascontiguousarray(t) for pair in st.fd for t in pair]
    P.cm1, P.cp1, P.cm2, P.cp2, P.cm3, P.cp3 = (_ptr(t) for t in tabs)
    P.nthreads = threads
    F = [np.ascontiguousarray(a, dtype=np.float64) for a in (F1, F2, F3)]
    out = [np.zeros_like(F[0]) for _ in range(3)]
    fn = lib.oracle_curl_h if which == "H" else lib.oracle_curl_e
    fn(C.byref(P), *(_ptr(a) for a in F), *(_ptr(a) for a in out))
    return out
