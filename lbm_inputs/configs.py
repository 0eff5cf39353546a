"""The five synthetic workloads (2D thermal, 2D solutal, 2D thermosolutal with
forced flow, a batched ensemble of uneven 2D domains, 3D directional) and a
helper that shrinks any of them for quick tests.

Every value is either printed in the paper (cited beside it) or drawn from
``numpy.random.default_rng(25670)`` (PCG64).  Lattice units throughout:
delta_x = 1 and time in the unit in which ``dt_base`` is expressed.

A workload is a dict with keys
  ``name``      short label
  ``domains``   list of per-domain parameter dicts (one for single runs)
  ``steps``     base steps of the accuracy run
  ``steps_timed`` base steps of one timed window
  ``dtype``     compute precision, ``storage`` population storage format

Per-domain keys (all floats unless noted):
  dim, nx, ny, nz (int)         grid, x fastest
  q_scalar (int)                5 (D2Q5) / 7 (D3Q7) / 9 (D2Q9) scalar lattice
  has_U, has_T, has_flow (bool) which fields beside phi are carried
  N_phi, N_U, N_T, N_F (int)    update factors, dt_chi = N_chi * dt_base
  dt_base
  W0, tau0, eps_s, lam, Mc, k, theta_c       phase field (Eq. 1-5)
  D_L, D_S, C_inf                             solute (Eq. 5, 7)
  kappa_S, kappa_L, rhoCp_S, rhoCp_L          heat (Eq. 10-12)
  rho_L, L_h, T_m, m_L, Cp_L                  heat / maps (Eq. 5, 12)
  nu, s_e, s_eps, s_q, u_in, Fb (3-tuple)     flow (Eq. 13, 27-32)
  bc        per-axis scalar boundary: "periodic" | "wall"
  flow_bc   per-axis flow boundary: "periodic" | "wall" | "inlet_outflow"
  U0, T0    initial uniform values
  u0_liquid_only (bool)  initial velocity u_in * f_L along x
  seeds     list of (cx, cy[, cz], R)
  coupling  "instant" (Eq. 39) | "accum" (delayed coarse-step injection)
  T_mode    "transport" | "pulled" (3D: T advected at V_pull along z, no
            latent heat, walls of the last axis held at the moving profile
            T0 + T_grad (z - z_front - V_pull t)) | "dirichlet_low" (latent
            heat kept, low wall of the last axis held at T0)
  perturb   per-column front offset xi (nx values in 2D, ny x nx in 3D):
            phi = tanh[(z_front + xi - z)/(sqrt2 W0)] along the last axis
"""

from __future__ import annotations

import copy
import math

import numpy as np

SEED = 25670

# Common values
A1 = 0.8839  # a1 in lambda = a1 W0 / d0 (Section 4.1-4.3)


def _base_domain() -> dict:
    return dict(
        dim=2, nx=64, ny=64, nz=1, q_scalar=5,
        has_U=False, has_T=False, has_flow=False,
        N_phi=1, N_U=1, N_T=1, N_F=1, dt_base=1.0,
        W0=1.0, tau0=1.0, eps_s=0.0, lam=0.0, Mc=0.0, k=1.0, theta_c=0.0,
        D_L=0.0, D_S=0.0, C_inf=1.0,
        kappa_S=0.0, kappa_L=0.0, rhoCp_S=1.0, rhoCp_L=1.0,
        rho_L=1.0, L_h=1.0, T_m=0.0, m_L=0.0, Cp_L=1.0,
        nu=0.1, s_e=1.2, s_eps=1.4, s_q=1.2, u_in=0.0, Fb=(0.0, 0.0, 0.0),
        bc=("periodic", "periodic", "periodic"),
        flow_bc=("periodic", "periodic", "periodic"),
        U0=0.0, T0=0.0, u0_liquid_only=False,
        seeds=[], coupling="instant", T_mode="transport",
        T_grad=0.0, V_pull=0.0, z_front=0.0,
    )


def thermal_128() -> dict:
    """2D pure thermal dendrite, FP64, 128x128 periodic.

    Section 4.1 set with W0 = 1 and tau0 = 20 (keeps W0^2/tau0 = 0.05 and
    Pe = W0^2/(alpha tau0) = 0.25); alpha = 0.2, eps_s = 0.05,
    lambda = a1/(d0/W0) with d0 = 0.1385 W0, theta0 = -0.55, Mc = 0,
    L_h = 1 and rho*Cp = 1 so that theta = T.  Seed R0 = 5 at node (64, 64).
    """
    d = _base_domain()
    d.update(
        nx=128, ny=128, has_T=True,
        W0=1.0, tau0=20.0, eps_s=0.05, lam=A1 / 0.1385, Mc=0.0, k=1.0,
        kappa_S=0.2, kappa_L=0.2, rhoCp_S=1.0, rhoCp_L=1.0,
        rho_L=1.0, L_h=1.0, Cp_L=1.0, T_m=0.0, m_L=0.0,
        T0=-0.55, bc=("periodic", "periodic", "periodic"),
        seeds=[(64.0, 64.0, 5.0)],
    )
    return dict(name="thermal_128", domains=[d], steps=1000, steps_timed=1000,
                dtype="f64", storage="f64")


def solutal_512() -> dict:
    """2D isothermal solutal dendrite, FP32, 512x512 zero-flux box.

    Section 4.2 set: W0 = 2.5, tau0 = 50, eps_s = 0.02, d0 = 0.2762 W0,
    Mc = 1, k = 0.15, U0 = -0.55, D_L = 0.25, D_S = 1e-2 D_L, theta = 0.
    N_phi = 1, N_U = 4 with dt_base = 1/4 so that dt_U = 1 (the Section 4.2
    convention of a unit coarse step).  Seed R0 = 8 at the cell centre.
    """
    d = _base_domain()
    d.update(
        nx=512, ny=512, has_U=True, N_phi=1, N_U=4, dt_base=0.25,
        W0=2.5, tau0=50.0, eps_s=0.02, lam=A1 / 0.2762, Mc=1.0, k=0.15,
        D_L=0.25, D_S=0.0025, C_inf=1.0, U0=-0.55,
        bc=("wall", "wall", "wall"), seeds=[(255.5, 255.5, 8.0)],
    )
    return dict(name="solutal_512", domains=[d], steps=20000, steps_timed=2000,
                dtype="f32", storage="f32")


def thermosolutal_flow_1024() -> dict:
    """2D thermosolutal dendrite under forced convection, 1024x1024.

    Section 4.3 set (W0 = 2, tau0 = 1000, eps_s = 0.02, lambda = 1.5955,
    Mc = 0.1, k = 0.15, U0 = 0, theta0 = -0.55, D_L = 0.004, D_S = 4e-5)
    with Le = 100 (alpha = 0.4), rho*Cp = L_h = 1, nu = 0.1, u_in = 0.01 from
    the left, outflow on the right, periodic top/bottom; scalars zero-flux.
    Update factors 1:1:4:2, dt_base = 1.  Seed R = 30 at the centre, crystal
    orientation drawn uniformly in [0, 45) degrees.
    """
    rng = np.random.default_rng(SEED)
    theta = math.radians(float(rng.uniform(0.0, 45.0)))
    d = _base_domain()
    d.update(
        nx=1024, ny=1024, has_U=True, has_T=True, has_flow=True,
        N_phi=1, N_U=1, N_T=4, N_F=2, dt_base=1.0,
        W0=2.0, tau0=1000.0, eps_s=0.02, lam=1.5955, Mc=0.1, k=0.15,
        theta_c=theta, D_L=0.004, D_S=4.0e-5, C_inf=1.0,
        kappa_S=0.4, kappa_L=0.4, rhoCp_S=1.0, rhoCp_L=1.0,
        rho_L=1.0, L_h=1.0, Cp_L=1.0, T_m=0.0, m_L=0.0, T0=-0.55, U0=0.0,
        nu=0.1, u_in=0.01, u0_liquid_only=True,
        bc=("wall", "wall", "wall"),
        flow_bc=("inlet_outflow", "periodic", "periodic"),
        seeds=[(511.5, 511.5, 30.0)],
    )
    return dict(name="thermosolutal_flow_1024", domains=[d], steps=20000,
                steps_timed=2000, dtype="f32", storage="f16")


def thermosolutal_flow_4096() -> dict:
    """The forced-convection case enlarged to 4096 x 4096 (16.8 M sites, past
    the 256 MB last-level cache in every storage format), for the HBM-bound
    measurement of the four-field step.  The seed keeps its radius at the
    centre.  tau0 = 100, D_L = 0.04, D_S = 4e-4 (tau_phi ~ 0.62), where the
    scheme is stable: at the Section 4.3 scale it diverges within about 170
    steps on any grid.  The kernels and bytes per site are those of the
    1024 x 1024 case."""
    wl = thermosolutal_flow_1024()
    d = wl["domains"][0]
    d.update(nx=4096, ny=4096, seeds=[(2047.5, 2047.5, 30.0)], tau0=100.0, D_L=0.04, D_S=4.0e-4)
    return dict(wl, name="thermosolutal_flow_4096", domains=[d])


# Table 1 lattice values (saline water, Section 4.4)
TABLE1 = dict(
    L_h=133.6, Cp_L=1.676, Cp_S=0.836, kappa_L=0.0437, kappa_S=0.178,
    alpha_L=0.026, k=0.001, C_inf=0.03, m_L=-57.0, eps_s=0.03,
    lam=11.27, Mc=0.0214, W0=2.0, tau0=150.0, rho=1.0,
)


def ensemble_256(n_domains: int = 256, side_lo: int = 128, side_hi: int = 512) -> dict:
    """Batched ensemble of independent 2D thermosolutal domains (no flow).

    Table 1 lattice set; per domain: square side ~ U{side_lo..side_hi},
    eps_s ~ U(0.01, 0.05), undercooling Delta ~ U(0.3, 0.7) so
    theta0 = -Delta, Le ~ U{1, 10, 100, 1000} with D_L = alpha_L/Le,
    D_S = 1e-2 D_L and N_U = Le (the Section 4.4 rule that keeps the liquid
    concentration relaxation time fixed); 1-4 seeds, R ~ U(5, 10), centres by
    rejection at spacing >= 4 R_max.  Zero-flux walls, N_phi = N_T = 1.
    """
    rng = np.random.default_rng(SEED + 4)
    t = TABLE1
    doms = []
    for _ in range(n_domains):
        L = int(rng.integers(side_lo, side_hi + 1))
        eps = float(rng.uniform(0.01, 0.05))
        delta = float(rng.uniform(0.3, 0.7))
        Le = int(rng.choice([1, 10, 100, 1000]))
        nseed = int(rng.integers(1, 5))
        seeds = []
        tries = 0
        while len(seeds) < nseed and tries < 1000:
            tries += 1
            R = float(rng.uniform(5.0, 10.0))
            cx = float(rng.uniform(20.0, L - 21.0))
            cy = float(rng.uniform(20.0, L - 21.0))
            if all((cx - s[0]) ** 2 + (cy - s[1]) ** 2 >= 40.0 ** 2 for s in seeds):
                seeds.append((cx, cy, R))
        d = _base_domain()
        D_L = t["alpha_L"] / Le
        d.update(
            nx=L, ny=L, has_U=True, has_T=True, N_phi=1, N_U=Le, N_T=1,
            dt_base=1.0, W0=t["W0"], tau0=t["tau0"], eps_s=eps, lam=t["lam"],
            Mc=t["Mc"], k=t["k"], D_L=D_L, D_S=1.0e-2 * D_L, C_inf=t["C_inf"],
            kappa_S=t["kappa_S"], kappa_L=t["kappa_L"],
            rhoCp_S=t["rho"] * t["Cp_S"], rhoCp_L=t["rho"] * t["Cp_L"],
            rho_L=t["rho"], L_h=t["L_h"], Cp_L=t["Cp_L"], T_m=0.0, m_L=t["m_L"],
            U0=0.0, T0=t["m_L"] * t["C_inf"] - delta * t["L_h"] / t["Cp_L"],
            bc=("wall", "wall", "wall"), seeds=seeds,
        )
        d["Le"] = Le
        d["Delta"] = delta
        doms.append(d)
    return dict(name="ensemble_256", domains=doms, steps=10000, steps_timed=1000,
                dtype="f32", storage="f16")


def directional_3d(nx: int = 256, ny: int = 256, nz: int = 512) -> dict:
    """3D directional solidification with a frozen, pulled linear temperature.

    Table 1 set with k = 0.01 (lambda and Mc are the Table 1 definitions
    evaluated at that k), eps_s = 0.03, Le = 1000.
    Periodic in x, y; zero-flux for phi and U along z.  The planar front sits
    at z = 10 with a per-column random offset xi ~ U(-1, 1).  Update factors
    1:1:16:4.  T starts at T_L + G (z - 10) with T_L = m_L C_inf, G = 0.02, and
    is pulled at V = 2e-4 per base step (liquid thermal properties throughout,
    so the linear profile is exact).
    """
    rng = np.random.default_rng(SEED + 5)
    t = TABLE1
    k = 0.01
    # Table 1 definitions evaluated at k = 0.01 (Gamma = 0.268):
    # d0 = 0.158308, lambda = a1 W0 / d0, Mc = -m_L (1-k) C_inf / (L_h/Cp_L)
    lam = 11.16683
    Mc = 0.0212373
    xi = rng.uniform(-1.0, 1.0, size=(ny, nx))
    D_L = t["alpha_L"] / 1000.0
    d = _base_domain()
    d.update(
        dim=3, nx=nx, ny=ny, nz=nz, q_scalar=7, has_U=True, has_T=True,
        has_flow=True, N_phi=1, N_U=1, N_T=16, N_F=4, dt_base=1.0,
        W0=t["W0"], tau0=t["tau0"], eps_s=0.03, lam=lam, Mc=Mc, k=k,
        D_L=D_L, D_S=1.0e-2 * D_L, C_inf=t["C_inf"],
        kappa_S=t["kappa_L"], kappa_L=t["kappa_L"],
        rhoCp_S=t["Cp_L"], rhoCp_L=t["Cp_L"], rho_L=1.0, L_h=t["L_h"],
        Cp_L=t["Cp_L"], T_m=0.0, m_L=t["m_L"], U0=0.0,
        nu=0.025, bc=("periodic", "periodic", "wall"),
        flow_bc=("periodic", "periodic", "wall"),
        T_mode="pulled", T_grad=0.02, V_pull=2.0e-4, z_front=10.0,
        T0=t["m_L"] * t["C_inf"],
    )
    d["perturb"] = xi
    return dict(name="directional_3d", domains=[d], steps=5000, steps_timed=320,
                dtype="f32", storage="bf16")


def directional_2d(Le: int = 100, coupling: str = "instant", nx: int = 1000, ny: int = 1000) -> dict:
    """2D directional saline-water solidification of Section 4.4.

    Table 1 lattice set, W0 = 2, tau0 = 150, D_L = alpha_L / Le with
    N_U = Le and N_phi = N_T = 1 (Eq. 42), D_S = 1e-2 D_L, U0 = 0.  Eq. (41)
    front: phi = tanh[(10 + sin(10 pi x / L) - y)/(sqrt2 W0)].  T starts at
    T_b = -20 and the bottom wall is held there; T_m = 0; no flow.  Periodic
    in x (the perturbation has five whole wavelengths), zero-flux elsewhere.
    """
    t = TABLE1
    D_L = t["alpha_L"] / Le
    d = _base_domain()
    d.update(
        nx=nx, ny=ny, has_U=True, has_T=True, N_phi=1, N_U=int(Le), N_T=1, dt_base=1.0,
        W0=t["W0"], tau0=t["tau0"], eps_s=t["eps_s"], lam=t["lam"], Mc=t["Mc"], k=t["k"],
        D_L=D_L, D_S=1.0e-2 * D_L, C_inf=t["C_inf"],
        kappa_S=t["kappa_S"], kappa_L=t["kappa_L"],
        rhoCp_S=t["rho"] * t["Cp_S"], rhoCp_L=t["rho"] * t["Cp_L"],
        rho_L=t["rho"], L_h=t["L_h"], Cp_L=t["Cp_L"], T_m=0.0, m_L=t["m_L"],
        U0=0.0, T0=-20.0, bc=("periodic", "wall", "wall"),
        T_mode="dirichlet_low", z_front=10.0, coupling=coupling,
    )
    x = np.arange(nx, dtype=np.float64)
    d["perturb"] = np.sin(10.0 * math.pi * x / nx)
    d["Le"] = Le
    return dict(name=f"directional_2d_Le{Le}_{coupling}", domains=[d], steps=30000, steps_timed=1000,
                dtype="f64", storage="f64")


def thermal_forced_512(N_T: int = 15) -> dict:
    """Section 4.1 thermal dendrite under forced convection, 512 x 512.

    W0 = 2.5, tau0 = 125 (dt_phi = 1), alpha = 0.2, nu = 4.62, L_h = 1,
    eps_s = 0.05, lambda = 0.8839 / 0.1385, theta0 = -0.55, M_c = 0;
    seed R0 = 10 at the centre; u_in = W0 / tau0 from the left, outflow on the
    right, periodic top and bottom (flow), zero-flux scalars.  dt_base = 1/15
    with N_phi = 15, N_F = 1 (tau_F = 1.424) and N_T in {15, 30, 45} (the
    update-factor study of Fig. 4c).
    """
    d = _base_domain()
    W0, tau0 = 2.5, 125.0
    d.update(
        nx=512, ny=512, has_T=True, has_flow=True, N_phi=15, N_T=int(N_T), N_F=1, dt_base=1.0 / 15.0,
        W0=W0, tau0=tau0, eps_s=0.05, lam=0.8839 / 0.1385, Mc=0.0, k=0.15,
        kappa_S=0.2, kappa_L=0.2, rhoCp_S=1.0, rhoCp_L=1.0, rho_L=1.0, L_h=1.0, Cp_L=1.0,
        T_m=0.0, m_L=0.0, T0=-0.55, nu=4.62, u_in=W0 / tau0, u0_liquid_only=True,
        bc=("wall", "wall", "wall"), flow_bc=("inlet_outflow", "periodic", "periodic"),
        seeds=[(255.5, 255.5, 10.0)],
    )
    return dict(name=f"thermal_forced_512_NT{N_T}", domains=[d], steps=120000, steps_timed=15000,
                dtype="f32", storage="f32")


def solutal_forced_1000(N_U: int = 15) -> dict:
    """Section 4.2 solutal dendrite under forced convection, 1000 x 1000.

    W0 = 2.5, tau0 = 50 (dt_phi = 1), eps_s = 0.02, lambda = 0.8839 / 0.2762,
    M_c = 1, k = 0.15, U0 = -0.55, D_L = 0.25, D_S = 1e-2 D_L, u_in = W0/tau0;
    the viscosity is not given for this case, so the Section 4.1 value
    nu = 4.62 (tau_F = 1.424 at dt_F = 1/15) is used.  dt_base = 1/15 with
    N_phi = 15, N_F = 1 and N_U in {15, 30, 45} (Fig. 7c).
    """
    d = _base_domain()
    W0, tau0 = 2.5, 50.0
    d.update(
        nx=1000, ny=1000, has_U=True, has_flow=True, N_phi=15, N_U=int(N_U), N_F=1, dt_base=1.0 / 15.0,
        W0=W0, tau0=tau0, eps_s=0.02, lam=0.8839 / 0.2762, Mc=1.0, k=0.15,
        D_L=0.25, D_S=2.5e-3, U0=-0.55, nu=4.62, u_in=W0 / tau0, u0_liquid_only=True,
        bc=("wall", "wall", "wall"), flow_bc=("inlet_outflow", "periodic", "periodic"),
        seeds=[(499.5, 499.5, 10.0)],
    )
    return dict(name=f"solutal_forced_1000_NU{N_U}", domains=[d], steps=450000, steps_timed=15000,
                dtype="f32", storage="f32")


def thermosolutal_forced_1500(N_U: int = 30, tau0: float = 500.0) -> dict:
    """Section 4.3 thermosolutal dendrite under forced convection, 1500 x 1500.

    The printed set (W0 = 2, eps_s = 0.02, d0 = 0.554 W0, lambda = 1.5955,
    M_c = 0.1, k = 0.15, U0 = 0, theta0 = -0.55, Le = alpha_L / D_L = 50,
    D_S = 1e-2 D_L, Pr = nu / alpha_L = 23.1, u_in = W0 / (5 tau0), seed
    R_s = 45 at the centre, N_phi = N_T = N_F = 1) with tau0 = 500 instead of
    the printed 1000: at tau0 = 1000 the phase update of Eq. (26) has modes
    that grow at every reading (tau_phi = 0.512 < 1/(2 A) on diagonal
    normals), at 500 it has none (tau_phi = 0.523).  D_L follows from the
    printed D~_L = D_L tau0 / W0^2 = 1, so D_L = 0.008, alpha_L = 0.4,
    nu = 9.24; N_U in {30, 40, 50} (Fig. 10b, c).
    """
    d = _base_domain()
    W0 = 2.0
    D_L = W0 * W0 / tau0
    alpha = 50.0 * D_L
    d.update(
        nx=1500, ny=1500, has_U=True, has_T=True, has_flow=True,
        N_phi=1, N_U=int(N_U), N_T=1, N_F=1, dt_base=1.0,
        W0=W0, tau0=float(tau0), eps_s=0.02, lam=1.5955, Mc=0.1, k=0.15,
        D_L=D_L, D_S=1.0e-2 * D_L, C_inf=1.0,
        kappa_S=alpha, kappa_L=alpha, rhoCp_S=1.0, rhoCp_L=1.0,
        rho_L=1.0, L_h=1.0, Cp_L=1.0, T_m=0.0, m_L=0.0, T0=-0.55, U0=0.0,
        nu=23.1 * alpha, u_in=W0 / (5.0 * tau0), u0_liquid_only=True,
        bc=("wall", "wall", "wall"), flow_bc=("inlet_outflow", "periodic", "periodic"),
        seeds=[(749.5, 749.5, 45.0)],
    )
    return dict(name=f"thermosolutal_forced_1500_NU{N_U}", domains=[d], steps=540000, steps_timed=15000,
                dtype="f32", storage="f32")


WORKLOADS = {
    "thermal_128": thermal_128,
    "solutal_512": solutal_512,
    "thermosolutal_flow_1024": thermosolutal_flow_1024,
    "thermosolutal_flow_4096": thermosolutal_flow_4096,
    "ensemble_256": ensemble_256,
    "directional_3d": directional_3d,
    "directional_2d": directional_2d,
    "thermal_forced_512": thermal_forced_512,
    "solutal_forced_1000": solutal_forced_1000,
    "thermosolutal_forced_1500": thermosolutal_forced_1500,
}


def workload(name: str, **kw) -> dict:
    return WORKLOADS[name](**kw)


def reduced(wl: dict, nx: int, ny: int, nz: int | None = None, steps: int | None = None,
            domains: int | None = None) -> dict:
    """A copy of ``wl`` on a smaller grid.  Seeds keep their radius and their
    offset from the domain centre (clipped inside the grid)."""
    out = copy.deepcopy(wl)
    if domains is not None:
        out["domains"] = out["domains"][:domains]
    for d in out["domains"]:
        ocx, ocy = (d["nx"] - 1) / 2.0, (d["ny"] - 1) / 2.0
        ncx, ncy = (nx - 1) / 2.0, (ny - 1) / 2.0
        seeds = []
        for s in d["seeds"]:
            cx = min(max(s[0] - ocx + ncx, 0.0), nx - 1.0)
            cy = min(max(s[1] - ocy + ncy, 0.0), ny - 1.0)
            seeds.append((cx, cy) + tuple(s[2:]))
        d["seeds"] = seeds
        if "perturb" in d:
            xi = np.asarray(d["perturb"])
            d["perturb"] = xi[:ny, :nx] if xi.ndim == 2 else xi[:nx]
        d["nx"], d["ny"] = nx, ny
        if nz is not None:
            d["nz"] = nz
    if steps is not None:
        out["steps"] = steps
    out["name"] = wl["name"] + f"_reduced{nx}x{ny}"
    return out
