"""Neighbour access with boundary ghosts, the isotropic finite-difference
gradient and divergence, and pull streaming with bounce-back.

Array layout: 2D arrays are [ny, nx], 3D arrays are [nz, ny, nx]; a lattice
vector e = (e_x, e_y[, e_z]) therefore acts on array axis ``ndim-1-a`` for
physical axis a.  Boundary kinds per physical axis: "periodic" (wrap),
"wall" (zero flux), "inlet_outflow" (flow only; treated as a wall by the
pull and fixed afterwards by the flow step).
"""

from __future__ import annotations

import numpy as np

from .lattice import stencil_lattice


def _arr_axis(ndim: int, phys_axis: int) -> int:
    return ndim - 1 - phys_axis


def pad1(a: np.ndarray, bc, negate_phys_axis: int | None = None) -> np.ndarray:
    """Pad ``a`` by one ghost layer on every axis.

    periodic axes wrap; other axes copy the edge value (the even mirror about
    the half-way wall: the ghost at -1 equals the node at 0).  If
    ``negate_phys_axis`` is given, the ghost layers across that axis are
    negated (odd mirror of the normal component of a vector field, reading of
    the compact divergence at zero-flux walls)."""
    out = a
    nd = a.ndim
    for pa in range(nd):
        ax = _arr_axis(nd, pa)
        mode = "wrap" if bc[pa] == "periodic" else "edge"
        width = [(0, 0)] * nd
        width[ax] = (1, 1)
        out = np.pad(out, width, mode=mode)
        if negate_phys_axis == pa and bc[pa] != "periodic":
            lo = [slice(None)] * nd
            hi = [slice(None)] * nd
            lo[ax] = slice(0, 1)
            hi[ax] = slice(-1, None)
            out[tuple(lo)] = -out[tuple(lo)]
            out[tuple(hi)] = -out[tuple(hi)]
    return out


def at_offset(padded: np.ndarray, e) -> np.ndarray:
    """Given a 1-padded array, return b with b[x] = a[x + e] (|e_a| <= 1)."""
    nd = padded.ndim
    sl = []
    for ax in range(nd):
        pa = nd - 1 - ax
        o = int(e[pa])
        n = padded.shape[ax] - 2
        sl.append(slice(1 + o, 1 + o + n))
    return padded[tuple(sl)]


def grad_iso(phi: np.ndarray, bc) -> np.ndarray:
    """Isotropic gradient: d_a phi = (1/c_s^2) sum_i w_i e_ia phi(x + e_i)
    with the D2Q9 (2D) or D3Q19 (3D) weights; in 2D this is
    (phi_E - phi_W)/3 + (phi_NE - phi_NW - phi_SW + phi_SE)/12 for d_x.
    Ghosts: even mirror at walls, wrap on periodic axes.  Returns [d, ...]."""
    lat = stencil_lattice(phi.ndim)
    p = pad1(phi, bc)
    g = np.zeros((lat.d,) + phi.shape)
    for i in range(1, lat.Q):
        nb = at_offset(p, lat.e[i])
        for a in range(lat.d):
            if lat.e[i, a] != 0:
                g[a] += 3.0 * lat.w[i] * lat.e[i, a] * nb
    return g


def div_iso(J: np.ndarray, bc) -> np.ndarray:
    """Compact isotropic divergence: div J = 3 sum_i w_i e_i . J(x + e_i)
    (D2Q9/D3Q19 weights).  At zero-flux walls the ghost J is the mirror
    image: normal component negated, tangential components kept."""
    d = J.shape[0]
    lat = stencil_lattice(d)
    out = np.zeros(J.shape[1:])
    padded = [pad1(J[a], bc, negate_phys_axis=a) for a in range(d)]
    for i in range(1, lat.Q):
        for a in range(d):
            if lat.e[i, a] != 0:
                out += 3.0 * lat.w[i] * lat.e[i, a] * at_offset(padded[a], lat.e[i])
    return out


def source_outside(shape, e, bc) -> np.ndarray:
    """Mask of sites y whose upstream neighbour y - e lies outside the domain
    along a non-periodic axis."""
    nd = len(shape)
    mask = np.zeros(shape, dtype=bool)
    for pa in range(nd):
        if bc[pa] == "periodic" or e[pa] == 0:
            continue
        ax = nd - 1 - pa
        n = shape[ax]
        idx = np.arange(n) - int(e[pa])
        bad = (idx < 0) | (idx >= n)
        sh = [1] * nd
        sh[ax] = n
        mask |= bad.reshape(sh)
    return mask


def pull(post: np.ndarray, lat, bc) -> np.ndarray:
    """Pull streaming: out_i(y) = post_i(y - e_i).  If y - e_i is outside a
    non-periodic boundary, half-way bounce-back supplies post_ibar(y)."""
    out = np.empty_like(post)
    for i in range(lat.Q):
        p = pad1(post[i], bc)
        out[i] = at_offset(p, -lat.e[i])
        m = source_outside(post.shape[1:], lat.e[i], bc)
        if m.any():
            out[i][m] = post[lat.opp[i]][m]
    return out


def upstream(a: np.ndarray, e, bc) -> np.ndarray:
    """a(y - e) with even-mirror ghosts (used for the liquid fraction at the
    link midpoint of the partial bounce-back)."""
    return at_offset(pad1(a, bc), -np.asarray(e))
