"""Derived parameters: the algebra that turns a parameter set into relaxation
times, effective coefficients and the maps of Eq. (5).

Each function states the equation it writes out.  The per-site functions take
NumPy arrays of phi and broadcast.
"""

from __future__ import annotations

import numpy as np  # noqa: F401  (arrays broadcast through every function)


# ---------------------------------------------------------------- time steps
def dt_field(d: dict, field: str) -> float:
    """Eq. (34): dt_chi = N_chi * dt_base."""
    return {"phi": d["N_phi"], "U": d["N_U"], "T": d["N_T"], "F": d["N_F"]}[field] * d["dt_base"]


# ------------------------------------------------------------ phase field
def lambda_coupling(a1: float, W0: float, d0: float) -> float:
    """lambda = a1 W0 / d0 (Sections 4.1-4.3, Table 1)."""
    return a1 * W0 / d0


def capillary_length(Gamma: float, m_L: float, k: float, C_inf: float) -> float:
    """d0 = Gamma / (|m_L| (1 - k) C_inf) (Table 1)."""
    return Gamma / (abs(m_L) * (1.0 - k) * C_inf)


def solutal_coupling(m_L: float, k: float, C_inf: float, L_h: float, Cp_L: float) -> float:
    """M_c = -m_L (1 - k) C_inf / (L_h / C_pL) (Eq. 5, Table 1)."""
    return -m_L * (1.0 - k) * C_inf / (L_h / Cp_L)


def theta_of_T(d: dict, T):
    """Eq. (5): theta = (T - T_m - m_L C_inf) / (L_h / C_pL)."""
    return (T - d["T_m"] - d["m_L"] * d["C_inf"]) / (d["L_h"] / d["Cp_L"])


def tau_phi(d: dict, A):
    """Eq. (24): tau_phi = 3 dt_phi a_s^2 W0^2 / tau0 + 1/2 (A = a_s^2).
    The factor 3 is 1/c_s^2 of the scalar lattice (4 on D3Q7)."""
    inv_cs2 = 4.0 if d.get("q_scalar", 5) == 7 else 3.0
    return inv_cs2 * dt_field(d, "phi") * A * d["W0"] ** 2 / d["tau0"] + 0.5


# ------------------------------------------------------------ solute
def kfac(d: dict, phi):
    """(1 + k) - (1 - k) phi, the denominator of Eqs. (7), (8), (38)."""
    return (1.0 + d["k"]) - (1.0 - d["k"]) * phi


def D_eff(d: dict, phi):
    """Eq. (7)."""
    return ((1.0 + phi) * d["D_S"] + (1.0 - phi) * d["D_L"]) / kfac(d, phi)


def tau_U(d: dict, phi):
    """Eq. (24): tau_U = 3 dt_U D_eff + 1/2."""
    inv_cs2 = 4.0 if d.get("q_scalar", 5) == 7 else 3.0
    return inv_cs2 * dt_field(d, "U") * D_eff(d, phi) + 0.5


def concentration(d: dict, phi, U):
    """Inverse of the U map of Eq. (5): C = C_inf kfac(phi) [1 + (1-k) U] / 2."""
    return d["C_inf"] * kfac(d, phi) * (1.0 + (1.0 - d["k"]) * U) / 2.0


# ------------------------------------------------------------ heat
def kappa_eff(d: dict, phi):
    """Eq. (11), first line."""
    return (1.0 + phi) / 2.0 * d["kappa_S"] + (1.0 - phi) / 2.0 * d["kappa_L"]


def rhoCp_eff(d: dict, phi):
    """Eq. (11), second line (rho_S C_pS and rho_L C_pL given as products)."""
    return (1.0 + phi) / 2.0 * d["rhoCp_S"] + (1.0 - phi) / 2.0 * d["rhoCp_L"]


def alpha_eff(d: dict, phi):
    """alpha_eff = kappa_eff / (rho C_p)_eff (Section 2.3)."""
    return kappa_eff(d, phi) / rhoCp_eff(d, phi)


def tau_T(d: dict, phi):
    """Eq. (24): tau_T = 3 dt_T alpha_eff + 1/2."""
    inv_cs2 = 4.0 if d.get("q_scalar", 5) == 7 else 3.0
    return inv_cs2 * dt_field(d, "T") * alpha_eff(d, phi) + 0.5


# ------------------------------------------------------------ flow
def tau_F(d: dict) -> float:
    """Eq. (32): tau_F = 3 dt_F nu + 1/2."""
    return 3.0 * dt_field(d, "F") * d["nu"] + 0.5


# ------------------------------------------------------------ Table 1
def lattice_from_physical(phys: dict, dx: float, dt: float, dm: float, dT: float) -> dict:
    """Physical-to-lattice conversion of Section 4.4 / Table 1.

    Units: length dx [m], time dt [s], mass dm [kg], temperature dT [K].
    Energy per mass  J/kg      -> dx^2/dt^2
    Specific heat    J/(kg K)  -> dx^2/(dt^2 dT)
    Conductivity     W/(m K)   -> dm dx/(dt^3 dT)
    Diffusivities    m^2/s     -> dx^2/dt
    Gamma            K m       -> dT dx
    Densities: rho = dm/dx^3 (taken as 1, so the lattice density is
    phys_rho * dx^3 / dm; with rho = 1000 kg/m^3, dx = 1e-7, dm = 1e-18 it is 1).
    """
    out = {}
    out["L_h"] = phys["L_h"] / (dx ** 2 / dt ** 2)
    out["Cp_L"] = phys["Cp_L"] / (dx ** 2 / (dt ** 2 * dT))
    out["Cp_S"] = phys["Cp_S"] / (dx ** 2 / (dt ** 2 * dT))
    out["kappa_L"] = phys["kappa_L"] / (dm * dx / (dt ** 3 * dT))
    out["kappa_S"] = phys["kappa_S"] / (dm * dx / (dt ** 3 * dT))
    out["alpha_L"] = phys["alpha_L"] / (dx ** 2 / dt)
    out["alpha_S"] = phys["alpha_S"] / (dx ** 2 / dt)
    out["D_L"] = phys["D_L"] / (dx ** 2 / dt)
    out["Gamma"] = phys["Gamma"] / (dT * dx)
    out["rho"] = phys.get("rho", 1000.0) * dx ** 3 / dm
    out["k"] = phys["k"]
    out["C_inf"] = phys["C_inf"]
    out["m_L"] = phys["m_L"] / dT
    out["eps_s"] = phys["eps_s"]
    out["d0"] = capillary_length(out["Gamma"], out["m_L"], out["k"], out["C_inf"])
    out["W0"] = phys["W0_over_dx"]
    out["lam"] = lambda_coupling(phys["a1"], out["W0"], out["d0"])
    out["Mc"] = solutal_coupling(out["m_L"], out["k"], out["C_inf"], out["L_h"], out["Cp_L"])
    return out


def table1_physical() -> dict:
    """Physical column of Table 1 (saline water), plus W0 = 2 dx (Section 4.4)
    and a1 = 0.8839."""
    return dict(
        L_h=3.34e5, Cp_L=4191.0, Cp_S=2090.0, kappa_L=0.5457, kappa_S=2.22,
        alpha_L=1.3e-7, alpha_S=1.06e-6, k=0.001, C_inf=0.03, m_L=-57.0,
        D_L=1.3e-9, Gamma=2.68e-8, eps_s=0.03, W0_over_dx=2.0, a1=0.8839,
        rho=1000.0,
    )


def min_tau(d: dict) -> dict:
    """Relaxation times at phi = +1 and phi = -1 for every carried field,
    used to reject parameter sets with tau <= 1/2."""
    out = {}
    # a_s spans [1 - eps, 1 + eps] in 2D and [1 - 5 eps/3, 1 + eps] in 3D
    a_min = 1.0 - (5.0 / 3.0) * d["eps_s"]
    out["phi"] = float(tau_phi(d, a_min ** 2))
    if d["has_U"]:
        out["U"] = float(min(tau_U(d, 1.0), tau_U(d, -1.0)))
    if d["has_T"]:
        out["T"] = float(min(tau_T(d, 1.0), tau_T(d, -1.0)))
    if d["has_flow"]:
        out["F"] = tau_F(d)
    return out


