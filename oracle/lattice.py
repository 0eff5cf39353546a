"""Discrete velocity sets, weights and moment bases.

* D2Q9: velocities and weights of Eq. (15), transformation matrix of
  Eq. (16) (Section 3.1).
* D2Q5: not printed in the paper.  Reading used here: weights 1/3 (rest) and
  1/6 (axes), so c_s^2 = 1/3 and the factor 3 of Eqs. (19), (21), (24), (40)
  is unchanged; orthogonal rows [1,1,1,1,1], [0,1,0,-1,0], [0,0,1,0,-1],
  [-4,1,1,1,1], [0,1,-1,1,-1]; the flux rows (1, 2) relax with 1/tau and all
  other rows with 1, mirroring Eq. (23).
* D3Q7 (3D extension, not in the paper): weights 1/4 and 1/8, c_s^2 = 1/4;
  rows 1, x, y, z, 6-weighted |e|^2 row and two anisotropic second moments.
* D3Q19 (3D extension, not in the paper): orthogonal basis obtained by
  Gram-Schmidt from the monomial list 1, e_x, e_y, e_z, |e|^2, |e|^4,
  3e_x^2-|e|^2, e_y^2-e_z^2, e_xe_y, e_ye_z, e_xe_z, |e|^2 e_x, |e|^2 e_y,
  |e|^2 e_z, and the cubic ghost moments.

Index order of every array below is the population index i.
"""

from __future__ import annotations

import numpy as np


class Lattice:
    def __init__(self, name, e, w, M, flux_rows, cs2):
        self.name = name
        self.e = np.asarray(e, dtype=np.int64)          # [Q, d]
        self.w = np.asarray(w, dtype=np.float64)        # [Q]
        self.M = np.asarray(M, dtype=np.float64)        # [Q, Q]
        self.Minv = np.linalg.inv(self.M)
        self.Q, self.d = self.e.shape
        self.flux_rows = tuple(flux_rows)               # rows relaxed with 1/tau
        self.cs2 = float(cs2)
        opp = []
        for i in range(self.Q):
            j = [k for k in range(self.Q) if np.all(self.e[k] == -self.e[i])]
            opp.append(j[0])
        self.opp = np.asarray(opp)

    def __repr__(self):
        return f"Lattice({self.name})"


# Eq. (15), Eq. (16)
D2Q9 = Lattice(
    "D2Q9",
    e=[(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
    w=[4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
    M=[
        [1, 1, 1, 1, 1, 1, 1, 1, 1],
        [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [4, -2, -2, -2, -2, 1, 1, 1, 1],
        [0, 1, 0, -1, 0, 1, -1, -1, 1],
        [0, -2, 0, 2, 0, 1, -1, -1, 1],
        [0, 0, 1, 0, -1, 1, 1, -1, -1],
        [0, 0, -2, 0, 2, 1, 1, -1, -1],
        [0, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 1, -1, 1, -1],
    ],
    flux_rows=(3, 5),   # Eq. (23): s3 = s5 = 1/tau
    cs2=1 / 3,
)

D2Q5 = Lattice(
    "D2Q5",
    e=[(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)],
    w=[1 / 3] + [1 / 6] * 4,
    M=[
        [1, 1, 1, 1, 1],
        [0, 1, 0, -1, 0],
        [0, 0, 1, 0, -1],
        [-4, 1, 1, 1, 1],
        [0, 1, -1, 1, -1],
    ],
    flux_rows=(1, 2),
    cs2=1 / 3,
)

D3Q7 = Lattice(
    "D3Q7",
    e=[(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
    w=[1 / 4] + [1 / 8] * 6,
    M=[
        [1, 1, 1, 1, 1, 1, 1],
        [0, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 1, -1, 0, 0],
        [0, 0, 0, 0, 0, 1, -1],
        [-6, 1, 1, 1, 1, 1, 1],
        [0, 2, 2, -1, -1, -1, -1],
        [0, 0, 0, 1, 1, -1, -1],
    ],
    flux_rows=(1, 2, 3),
    cs2=1 / 4,
)


def _d3q19():
    e = [(0, 0, 0),
         (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    E = np.asarray(e, dtype=np.float64)
    x, y, z = E[:, 0], E[:, 1], E[:, 2]
    r2 = x * x + y * y + z * z
    mono = [
        np.ones(19), x, y, z, r2, r2 * r2,
        3 * x * x - r2, y * y - z * z, x * y, y * z, x * z,
        r2 * x, r2 * y, r2 * z,
        (3 * x * x - r2) * r2, (y * y - z * z) * r2,
        x * (y * y - z * z), y * (z * z - x * x), z * (x * x - y * y),
    ]
    rows = []
    for v in mono:
        u = v.copy()
        for r in rows:
            u = u - (u @ r) / (r @ r) * r
        rows.append(u)
    M = np.array(rows)
    # scale rows to small integers where possible (orthogonality is unaffected)
    for k in range(19):
        nz = np.abs(M[k])[np.abs(M[k]) > 1e-12]
        M[k] = np.round(M[k] / nz.min(), 12)
    return e, w, M


_e19, _w19, _M19 = _d3q19()
D3Q19 = Lattice("D3Q19", e=_e19, w=_w19, M=_M19, flux_rows=(1, 2, 3), cs2=1 / 3)


def scalar_lattice(q: int) -> Lattice:
    return {5: D2Q5, 9: D2Q9, 7: D3Q7}[q]


def flow_lattice(dim: int) -> Lattice:
    return D2Q9 if dim == 2 else D3Q19


def stencil_lattice(dim: int) -> Lattice:
    """Weights of the isotropic finite-difference stencils (D2Q9 in 2D,
    D3Q19 in 3D)."""
    return D2Q9 if dim == 2 else D3Q19
