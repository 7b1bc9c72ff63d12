"""C ABI checks that need no GPU: the library loads, exports every function
include/emm.h declares, the ctypes structures match the C layout, default
options, status strings, and every validation error that emm_create
reports before touching the device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emm.h")


@pytest.fixture(scope="module")
def emm():
    from paper_2304_00233_amd import emm as E
    return E


def test_exports_every_declared_function(emm):
    names = re.findall(r"^\s*(?:emm_status|void|const char\s*\*)\s*(emm_\w+)\s*\(",
                       open(HEADER).read(), re.M)
    assert set(names) == set(emm.EXPORTED)
    lib = C.CDLL(emm.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", emm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_struct_layout_matches_header(emm, tmp_path):
    src = tmp_path / "layout.c"
    structs = ["emm_grid", "emm_options", "emm_source", "emm_receiver", "emm_info", "emm_job"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "emm.h"', "int main(void){"]
    for s in structs:
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f, _ in getattr(emm, s)._fields_:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                        text=True).stdout.split("\n") if l)
    for s in structs:
        cls = getattr(emm, s)
        assert int(got[s]) == C.sizeof(cls), s
        for f, _ in cls._fields_:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)


def test_default_options(emm):
    o = emm.emm_default_options()
    assert (o.rd, o.nb, o.ne, o.f0, o.cfl, o.nt, o.dft_mode) == (2, 10, -1, 1.0, 0.99, 0, 0)
    assert o.cpml_R == 1e-5 and o.cpml_npow == 2.0 and o.profile == 0
    assert (o.checkpoint_every, o.checkpoint_inner, o.graph_steps, o.tile_kz) == (0, 0, 0, 0)
    assert o.nontemporal == -1 and o.airwave == 0
    assert o.converge_tol == 0.0 and o.converge_every == 100
    assert o.fused == 0 and o.ce_table == -1 and o.src_group == 0 and o.tile_x == 0
    assert o.tile_rows == 0 and o.src_order == -1


def test_status_strings(emm):
    for code, name in emm.STATUS.items():
        assert emm.emm_status_str(code) == name


def _grid(n=(12, 11, 10), rho=1.0):
    xs = [np.arange(k, dtype=np.float64) * 100.0 for k in n]
    r = np.full((n[2], n[1], n[0]), rho, np.float32)
    return xs, [r, r.copy(), r.copy()]


def _create_status(emm, xs, rs, **opt):
    o = emm.emm_default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    try:
        h = emm.emm_create(*xs, *rs, o)
    except emm.EmmError as e:
        return e.status, str(e)
    emm.emm_destroy(h)
    return 0, ""


def test_create_validation_errors(emm):
    xs, rs = _grid()
    assert _create_status(emm, xs, rs, rd=0)[0] == -1
    assert _create_status(emm, xs, rs, rd=5)[0] == -1
    assert _create_status(emm, xs, rs, nb=-1)[0] == -1
    assert _create_status(emm, xs, rs, f0=0.0)[0] == -1
    assert _create_status(emm, xs, rs, cpml_R=2.0)[0] == -1
    # too few nodes for the stencil
    xs2, rs2 = _grid((12, 11, 4))
    assert _create_status(emm, xs2, rs2, rd=2)[0] == -2
    # non-monotone and non-finite coordinates
    bad = [x.copy() for x in xs]
    bad[1][5] = bad[1][4]
    assert _create_status(emm, bad, rs)[0] == -2
    bad = [x.copy() for x in xs]
    bad[2][3] = np.nan
    assert _create_status(emm, bad, rs)[0] == -2
    # resistivity <= 0 or not finite
    for v in (0.0, -1.0, np.nan, np.inf):
        r2 = [a.copy() for a in rs]
        r2[2][1, 2, 3] = v
        assert _create_status(emm, xs, r2)[0] == -3, v
    # dt above the CFL limit
    st, msg = _create_status(emm, xs, rs, dt_override=1.0)
    assert st == -6 and "stability" in msg
    # convergence stop options
    assert _create_status(emm, xs, rs, converge_tol=-1.0)[0] == -1
    assert _create_status(emm, xs, rs, converge_every=0)[0] == -1
    # compact dt/eps: automatic (-1), off (0) or whenever possible (1)
    assert _create_status(emm, xs, rs, ce_table=2)[0] == -1
    assert _create_status(emm, xs, rs, ce_table=-2)[0] == -1
    assert _create_status(emm, xs, rs, src_group=-2)[0] == -1
    assert _create_status(emm, xs, rs, tile_x=48)[0] == -1
    assert _create_status(emm, xs, rs, tile_rows=3)[0] == -1
    assert _create_status(emm, xs, rs, tile_rows=4, tile_x=32)[0] == -1
    assert _create_status(emm, xs, rs, src_order=2)[0] == -1
    # the air boundary: option range, uniform x and y, room for the ghost planes
    assert _create_status(emm, xs, rs, airwave=4)[0] == -1
    nu = [x.copy() for x in xs]
    nu[0][3] += 1.0
    st, msg = _create_status(emm, nu, rs, airwave=1)
    assert st == -2 and "uniform" in msg
    st, msg = _create_status(emm, xs, rs, airwave=1, rd=3, nb=0, ne=2)
    assert st == -2 and "planes" in msg


def test_null_pointers(emm):
    lib = emm._lib
    h = C.c_void_p()
    assert lib.emm_create(None, None, C.byref(h)) == -1
    assert lib.emm_default_options(None) == -1
    assert lib.emm_query(None, None) == -1
    assert lib.emm_forward(None, None, 0, None, 0, 0, None, 0, None, None) == -1
    assert lib.emm_forward_noalloc(None, None, 0, None, 0, 0, None, 0, None, None) == -1
    assert lib.emm_forward_batch(None, 1, 0, None) == -1
    jobs = (emm.emm_job * 2)()
    assert lib.emm_forward_batch(jobs, 0, 0, None) == -1      # no jobs
    assert lib.emm_forward_batch(jobs, 2, 0, None) == -1      # NULL models
    assert lib.emm_forward_batch(jobs, 2, -1, None) == -1     # bad graph length
    lib.emm_destroy(None)                           # NULL-safe


def test_valid_create_without_gpu_reports_device(emm):
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU is present")
    xs, rs = _grid()
    st, msg = _create_status(emm, xs, rs)
    assert st == -9 and msg


@pytest.mark.parametrize("rd", [1, 2, 3, 4])
def test_host_stability_limit_matches_oracle(emm, rd):
    """emm_create computes eta = 1/2 v_max sqrt(sum D_d^2) (Section 3.2) from
    its Bjorck-Pereyra tables before any device call; the oracle computes it
    from Fornberg tables.  A dt_override a hair above the oracle's 1/eta must
    be rejected (CFL) and a hair below accepted by validation, on a
    non-uniform grid."""
    from oracle import forward as F
    from workloads import configs
    w = configs.small_case(seed=20 + rd, shape=(19, 17, 16), rd=rd,
                           nu_axes=(True, True, True))
    st = F.make_setup(w, fp=2.0)
    limit = st.dt / w.cfl
    xs = [w.x1, w.x2, w.x3]
    rs = [w.rho11, w.rho22, w.rho33]
    st_hi, _ = _create_status(emm, xs, rs, rd=rd, nb=w.nb, ne=w.ne, dt_override=limit * (1 + 1e-9))
    assert st_hi == -6
    st_lo, _ = _create_status(emm, xs, rs, rd=rd, nb=w.nb, ne=w.ne, dt_override=limit * (1 - 1e-9))
    assert st_lo != -6          # passes validation (then needs a device)


def test_create_rejects_grids_beyond_32_bit_offsets(emm):
    """The kernels address one field array with 32-bit offsets, so a padded
    grid of 2^31 cells or more (here 1290^3 nodes: (1290 + 34, rounded up to
    1344) x 1324 x 1324 = 2.36e9 cells) is refused with EMM_ERR_GRID before
    the resistivity arrays are read (a single value is passed) and before
    any device call."""
    lib = emm._lib

    def status(n, rho):
        xs = [np.arange(k, dtype=np.float64) * 10.0 for k in n]
        g = emm.emm_grid(n[0], n[1], n[2], *(a.ctypes.data_as(C.POINTER(C.c_double)) for a in xs),
                         *(a.ctypes.data_as(C.POINTER(C.c_float)) for a in rho))
        o = emm.emm_default_options()
        o.dt_override = 1e30          # a valid grid then fails the CFL check, still before the device
        h = C.c_void_p()
        return lib.emm_create(C.byref(g), C.byref(o), C.byref(h)), emm.emm_last_error(None)

    one = np.ones(1, np.float32)
    st, msg = status((1290, 1290, 1290), [one] * 3)
    assert st == -2 and "2^31" in msg
    n = (12, 11, 10)
    full = np.ones((n[2], n[1], n[0]), np.float32)
    st, _ = status(n, [full] * 3)
    assert st == -6
