"""Diagnostics of a domain: tip positions, solid fraction, total solute,
enthalpy, mass, and the coupling pulses S_phi and J_U (Section 4.1 tip
histories; Section 4.4 ablation measures).

Tip reading: from each seed centre, march along the four crystal axes
(angles theta_c + m 90 deg) at unit spacing, sampling phi by bilinear
interpolation (clamped at the domain edge).  The tip lies between the last
sample with phi >= 0 and the first sample with phi < 0; its position is the
linear interpolation of the zero crossing.
"""

from __future__ import annotations

import math

import numpy as np

from . import params as P


def bilinear(phi: np.ndarray, x: float, y: float) -> float:
    ny, nx = phi.shape
    x = min(max(x, 0.0), nx - 1.0)
    y = min(max(y, 0.0), ny - 1.0)
    x0 = min(int(math.floor(x)), nx - 2)
    y0 = min(int(math.floor(y)), ny - 2)
    tx, ty = x - x0, y - y0
    return ((1 - tx) * (1 - ty) * phi[y0, x0] + tx * (1 - ty) * phi[y0, x0 + 1]
            + (1 - tx) * ty * phi[y0 + 1, x0] + tx * ty * phi[y0 + 1, x0 + 1])


def tip_distance(phi: np.ndarray, cx: float, cy: float, angle: float, rmax: int) -> float:
    """Distance from (cx, cy) to the phi = 0 crossing along ``angle``."""
    c, s = math.cos(angle), math.sin(angle)
    prev = bilinear(phi, cx, cy)
    if prev < 0:
        return 0.0
    for r in range(1, rmax + 1):
        cur = bilinear(phi, cx + r * c, cy + r * s)
        if cur < 0:
            return (r - 1) + prev / (prev - cur)
        prev = cur
    return float(rmax)


def tips(dom) -> np.ndarray:
    """[n_seeds, 4] tip distances along +x', +y', -x', -y' (2D only)."""
    d = dom.d
    th = d.get("theta_c", 0.0)
    rmax = int(max(dom.shape))
    out = []
    for s in d["seeds"]:
        out.append([tip_distance(dom.phi, s[0], s[1], th + m * math.pi / 2, rmax) for m in range(4)])
    return np.asarray(out)


def totals(dom) -> dict:
    """Whole-domain sums in float64."""
    d = dom.d
    phi = dom.phi
    out = dict(solid=float(np.sum((1.0 + phi) / 2.0)))
    if d["has_U"]:
        out["M_C"] = float(np.sum(P.concentration(d, phi, dom.U)))
        out["sum_U"] = float(np.sum(dom.U))
    if d["has_T"]:
        out["enthalpy"] = float(np.sum(dom.T - d["rho_L"] * d["L_h"] * phi / (2.0 * d["rhoCp_L"])))
        out["sum_T"] = float(np.sum(dom.T))
    if d["has_flow"]:
        out["mass"] = float(np.sum(dom.rho))
    out["S_phi"] = dom.S_phi
    out["J_U"] = dom.J_U
    out["finite"] = bool(np.all(np.isfinite(phi)))
    return out
