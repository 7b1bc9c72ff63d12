"""Direct frequency-domain solve of the spatially discrete system (oracle pin).

z-transforming the leap-frog updates of Section 3.1 with z = exp(i w' dt),
the staggered stamps E^{m} -> m dt, H^{m+1/2} -> (m+1/2) dt, J^{m+1/2} ->
(m+1/2) dt and zero initial state gives exactly

    delta E^ = (dt/eps) (curlH~ H^ - J^),   delta H^ = -(dt/mu) curlE~ E^,
    delta = z^{-1/2} - z^{1/2} = -2 i sin(w' dt/2),

where the CPML memory variables psi^{n+1} = b psi^n + a d (Section 3.4)
turn each slab derivative D into D (1 + a/(1 - b z)).  So the time-domain run
followed by the receiver DTFT must equal, up to the truncation of the time
sum, the sparse solve of

    (delta^2 I + (dt/eps)(dt/mu) curlH~ M_H curlE~) E^ = -delta (dt/eps) J^

with J^ = q (the injection stencil times a unit source spectrum).  This pins
the time loop, the injection, the field stamps and the DTFT of the oracle
against a formulation that has no time loop at all.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import airwave as AW
from . import tables as T


def _axis_ops(st, axis: int, z: complex):
    """1D D-/D+ matrices along one axis with CPML factors folded in."""
    n = st.n_pad[axis]
    r = st.r
    cm, cp = st.fd[axis]
    a_i, b_i, a_h, b_h = st.cpml[axis]
    Dm = sp.lil_matrix((n, n), dtype=np.complex128)
    Dp = sp.lil_matrix((n, n), dtype=np.complex128)
    for i in range(r, n - r):
        fm = 1.0
        fp = 1.0
        if i < st.nb or i > n - 1 - st.nb:
            fm = 1.0 + a_i[i] / (1.0 - b_i[i] * z)
            fp = 1.0 + a_h[i] / (1.0 - b_h[i] * z)
        for m in range(2 * r):
            Dm[i, i - r + m] += fm * cm[i][m]
            Dp[i, i - r + 1 + m] += fp * cp[i][m]
    return Dm.tocsr(), Dp.tocsr()


def _lift(op, axis, n_pad):
    """Embed a 1D operator along `axis` into the [z][y][x] flattened grid."""
    n1, n2, n3 = n_pad
    I = [sp.identity(n, format="csr") for n in (n1, n2, n3)]
    mats = [I[2], I[1], I[0]]        # kron order: z, y, x
    mats[2 - axis] = op
    return sp.kron(mats[0], sp.kron(mats[1], mats[2], format="csr"), format="csr")


def _ghost_maps(st):
    """The air boundary's ghost fills as sparse maps on the [3][z][y][x]
    vectors: P_E = I + (E1, E2 ghost planes from the surface plane), P_H =
    I + (H1, H2 ghost half planes from H3 at the surface).  Built column by
    column by applying the fills of `airwave` to unit surface planes; the
    ghost fill is linear and uses only same-time-level values, so the
    z-transform carries it over unchanged."""
    n1, n2, n3 = st.n_pad
    N, M = n1 * n2 * n3, n1 * n2
    ops = AW.make_ops(st.axes, st.nbe, st.r)
    ks = st.nbe
    rowsE, colsE, valsE, rowsH, colsH, valsH = [], [], [], [], [], []
    for q in range(M):
        unit = np.zeros((n3, n2, n1))
        unit.reshape(n3, M)[ks, q] = 1.0
        a, b = unit.copy(), unit.copy()
        AW.fill_E(a, b, ops)
        h1, h2 = np.zeros((n3, n2, n1)), np.zeros((n3, n2, n1))
        AW.fill_H(h1, h2, unit, ops)
        for m in range(1, st.r + 1):
            for c, F in ((0, a), (1, b)):
                if m < st.r:
                    v = F.reshape(n3, M)[ks - m]
                    nz = np.nonzero(v)[0]
                    rowsE += list(c * N + (ks - m) * M + nz)
                    colsE += [c * N + ks * M + q] * len(nz)
                    valsE += list(v[nz])
            for c, F in ((0, h1), (1, h2)):
                v = F.reshape(n3, M)[ks - m]
                nz = np.nonzero(v)[0]
                rowsH += list(c * N + (ks - m) * M + nz)
                colsH += [2 * N + ks * M + q] * len(nz)
                valsH += list(v[nz])
    I = sp.identity(3 * N, format="csr")
    PE = I + sp.csr_matrix((valsE, (rowsE, colsE)), shape=(3 * N, 3 * N))
    PH = I + sp.csr_matrix((valsH, (rowsH, colsH)), shape=(3 * N, 3 * N))
    return PE, PH


def solve(st, freq: float, src, comp: int, rec, chans, moment: float = 1.0,
          airwave: bool = False):
    """Receiver values of E^ / H^ per unit source spectrum: [nrec][nchan].
    airwave: the first interior z node is the sea surface with air above
    (updates start there; ghost planes above it, `airwave`)."""
    n1, n2, n3 = st.n_pad
    N = n1 * n2 * n3
    r = st.r
    wp = T.omega_prime([freq], st.omega0)[0]
    z = np.exp(1j * wp * st.dt)
    delta = np.exp(-0.5j * wp * st.dt) - np.exp(0.5j * wp * st.dt)
    Dm, Dp = [], []
    for a in range(3):
        m, p = _axis_ops(st, a, z)
        Dm.append(_lift(m, a, st.n_pad))
        Dp.append(_lift(p, a, st.n_pad))
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    kmin = st.nbe if airwave else r
    upd = ((i >= r) & (i <= n1 - 1 - r) & (j >= r) & (j <= n2 - 1 - r) &
           (k >= kmin) & (k <= n3 - 1 - r)).ravel().astype(np.float64)
    U = sp.diags(upd)
    Z = sp.csr_matrix((N, N))
    # curl H~ -> E positions; curl E~ -> H positions (rows masked to the update set)
    curlH = sp.bmat([[Z, -Dm[2], Dm[1]], [Dm[2], Z, -Dm[0]], [-Dm[1], Dm[0], Z]], format="csr")
    curlE = sp.bmat([[Z, -Dp[2], Dp[1]], [Dp[2], Z, -Dp[0]], [-Dp[1], Dp[0], Z]], format="csr")
    U3 = sp.block_diag([U, U, U], format="csr")
    curlH = U3 @ curlH
    curlE = U3 @ curlE
    if airwave:
        PE, PH = _ghost_maps(st)
        curlH = (curlH @ PH).tocsr()
        curlE = (curlE @ PE).tocsr()
    ce = np.concatenate([c.ravel() for c in st.ce])
    ch = st.dt / T.MU0
    Ce = sp.diags(ce)
    A = delta * delta * sp.identity(3 * N) + ch * (Ce @ (curlH @ curlE))
    # non-updated E cells stay zero: identity rows there
    upd3 = np.concatenate([upd, upd, upd])
    keep = sp.diags(upd3)
    drop = sp.diags(1.0 - upd3)
    A = (keep @ A + drop).tocsc()
    # source stencil J^ = moment * w / V on the E_comp grid
    stag = [0, 0, 0]
    stag[comp] = 1
    sb, sw = T.point_stencil(st.axes, src, stag, r)
    wt = sw[2][:, None, None] * sw[1][None, :, None] * sw[0][None, None, :]
    q = moment * wt / T.dual_volume(st.axes, comp, sb, r)
    J = np.zeros((3, n3, n2, n1), dtype=np.complex128)
    L = 2 * r
    J[comp, sb[2]:sb[2] + L, sb[1]:sb[1] + L, sb[0]:sb[0] + L] = q
    rhs = -delta * ce * J.ravel() * upd3
    E = spla.spsolve(A, rhs)
    Hh = -(ch / delta) * (curlE @ E)
    E = E.reshape(3, n3, n2, n1)
    Hh = Hh.reshape(3, n3, n2, n1)
    out = np.zeros((len(rec), len(chans)), dtype=np.complex128)
    for a, p in enumerate(rec):
        for c, chn in enumerate(chans):
            b, w = T.point_stencil(st.axes, p, T.STAGGER[chn], r)
            F = E[chn] if chn < 3 else Hh[chn - 3]
            blk = F[b[2]:b[2] + L, b[1]:b[1] + L, b[0]:b[0] + L]
            out[a, c] = np.einsum("k,j,i,kji->", w[2], w[1], w[0], blk)
    return out
