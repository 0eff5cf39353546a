"""The coupled multirate MRT lattice-Boltzmann scheme, one domain at a time.

Section 3 of the paper, in whole-grid passes:

* phase field:  Eq. (2)-(4), (14), (21)-(24), (26)            -> ``phase_step``
* transfer:     Eq. (36)-(39), compact divergence of J_at      -> ``transfer``
* U and T:      Eq. (6)-(8), (10)-(12), (14), (19), (23)-(25),
                (35), (40)                                    -> ``scalar_step``
* flow:         Eq. (27)-(33)                                  -> ``flow_step``
* schedule:     Eq. (34) and the procedure around Fig. 1        -> ``Domain.step``

Readings where the paper is silent (the same list is kept with the design
notes of the HIP library):
  * the source of the phase collision is dt_phi w_i Q_phi / tau0 (Eq. 1
    divided by tau0 is what the anisotropic streaming recovers);
  * a_s^2 of Eq. (26) is taken at the destination node, from the same
    collision step;
  * grad(phi) for n, a_s and N (and for grad(phi*) in the transport sources)
    is the isotropic finite difference; Eq. (40) is used for grad U and
    grad T only;
  * if |grad phi|^2 < 1e-16 (|grad phi| < 1e-8, far below interface
    gradients of order 1/W0) then n = 0, a_s = 1 and N = 0: below that
    level the direction of the gradient is not resolved in FP64 at a seed
    centre, yet it would steer the anti-trapping current there;
  * U*, theta* are the values before this phase step's injection; n and
    the denominators of Eq. (38) are taken at phi^{q+1};
  * base steps are k = 1..K, field chi runs iff k mod N_chi == 0, in the
    order phi(+transfer), U, T, flow;
  * the scalar source carries no (I - S/2) factor;
  * zero flux is half-way bounce-back with even-mirror stencil ghosts;
  * inlet: after streaming the x = 0 column is set to f_eq(1, (u_in, 0));
    outflow: the x = L-1 column copies x = L-2;
  * several seeds: phi = max over seeds; crystal orientation theta_c rotates
    the normal into the crystal frame for a_s and N and rotates N back;
  * accumulated coupling ("accum"): the phase-change increments are summed
    and injected right after the field's next transport update;
  * pulled temperature (3D directional case, T_mode "pulled"): T is carried
    by its lattice with the pulling velocity V z^ in its equilibrium, receives
    no latent heat, and the bottom and top walls hold the moving linear
    profile T_L + G (z - z_front - V t) by anti-bounce-back; the linear
    profile is then an exact solution of the T lattice;
  * cold bottom (2D directional case of Section 4.4, T_mode "dirichlet_low"):
    T keeps its latent-heat transfer and the low wall of the last axis is
    held at T0 by the same anti-bounce-back; the other walls stay zero-flux;
  * planar fronts (Eq. 41 and its 3D random form): phi = tanh[(z_front +
    xi - z)/(sqrt2 W0)] along the last axis with a per-column offset xi;
  * the variant grad_phi = "eq40" (2D) takes grad(phi) for n, a_s and N
    from the non-equilibrium phase populations by Eq. (40), with the
    equilibrium and tau_phi of the previous phase step at the site (v_n and
    A lagged one step; the first step sees v_n = 0 and A = 1, the initial
    equilibrium): grad phi = -(3 / tau_prev) (j - v_n,prev dt_phi), since
    sum_i e_i f_i^eq = v_n dt_phi.  The transfer's normal and the transport
    sources keep the isotropic stencil.
"""

from __future__ import annotations

import math

import numpy as np

from . import params as P
from .lattice import flow_lattice, scalar_lattice
from .stencils import div_iso, grad_iso, pull, source_outside, upstream  # noqa: F401

GRAD_EPS2 = 1.0e-16


def _mv(M: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Matrix times a population field: (M f)_k = sum_i M_ki f_i at every site."""
    return np.tensordot(M, f, axes=(1, 0))


def _edot(lat, vec: np.ndarray) -> np.ndarray:
    """e_i . v at every site for every i: returns [Q, ...]."""
    return np.tensordot(lat.e.astype(np.float64), vec, axes=(1, 0))


def _wq(lat, ndim):
    return lat.w.reshape((lat.Q,) + (1,) * ndim)


def mrt_collide(lat, f, feq, s_vec, G=None):
    """Eq. (14) without the scalar source: f - M^-1 S (m - m_eq)
    [+ M^-1 (I - S/2) G].  ``s_vec`` holds the diagonal of S per site
    ([Q, ...]) or per row ([Q])."""
    m = _mv(lat.M, f)
    meq = _mv(lat.M, feq)
    if s_vec.ndim == 1:
        s_vec = s_vec.reshape((lat.Q,) + (1,) * (f.ndim - 1))
    post = f - _mv(lat.Minv, s_vec * (m - meq))
    if G is not None:
        post = post + _mv(lat.Minv, (1.0 - s_vec / 2.0) * G)
    return post


def scalar_relaxation(lat, tau) -> np.ndarray:
    """Eq. (23): S = diag(1, .., 1/tau on the flux rows, .., 1) per site."""
    s = np.ones((lat.Q,) + np.shape(tau))
    for r in lat.flux_rows:
        s[r] = 1.0 / tau
    return s


def anisotropy(d: dict, g: np.ndarray):
    """Eq. (2)-(3) from the gradient g = grad(phi).

    n = -g/|g|; in the crystal frame n' = R(-theta_c) n,
    a_s = 1 - 3 eps + 4 eps sum_a n'_a^4 and
    N'_a = |g|^2 a_s d a_s / d g'_a = -16 eps a_s |g| n'_a (n'_a^2 - sum_b n'_b^4),
    rotated back N = R(theta_c) N'.  Degenerate gradient: n = 0, a_s = 1, N = 0.
    Returns (a_s, N, n)."""
    eps = d["eps_s"]
    dim = g.shape[0]
    gg = np.sum(g * g, axis=0)
    ok = gg >= GRAD_EPS2
    gn = np.sqrt(np.where(ok, gg, 1.0))
    n = np.where(ok, -g / gn, 0.0)
    th = d.get("theta_c", 0.0)
    if dim == 2 and th != 0.0:
        c, s = math.cos(th), math.sin(th)
        nc = np.stack([c * n[0] + s * n[1], -s * n[0] + c * n[1]])
    else:
        nc = n
    s4 = np.sum(nc ** 4, axis=0)
    a_s = np.where(ok, 1.0 - 3.0 * eps + 4.0 * eps * s4, 1.0)
    Nc = -16.0 * eps * a_s * np.where(ok, gn, 0.0) * nc * (nc * nc - s4)
    if dim == 2 and th != 0.0:
        N = np.stack([c * Nc[0] - s * Nc[1], s * Nc[0] + c * Nc[1]])
    else:
        N = Nc
    return a_s, N, n


def unit_normal(g: np.ndarray) -> np.ndarray:
    """n = -g/|g| (0 for a degenerate gradient)."""
    gg = np.sum(g * g, axis=0)
    ok = gg >= GRAD_EPS2
    gn = np.sqrt(np.where(ok, gg, 1.0))
    return np.where(ok, -g / gn, 0.0)


class Domain:
    """State of one domain: populations and macroscopic planes of every
    carried field, the base-step counter and the coupling diagnostics."""

    def __init__(self, d: dict):
        self.d = dict(d)
        self.dim = d["dim"]
        if self.dim == 2:
            self.shape = (d["ny"], d["nx"])
        else:
            self.shape = (d["nz"], d["ny"], d["nx"])
        self.bc = tuple(d["bc"][: self.dim])
        self.fbc = tuple(d["flow_bc"][: self.dim])
        self.ls = scalar_lattice(d["q_scalar"])
        self.lf = flow_lattice(self.dim) if d["has_flow"] else None
        self.inv_cs2 = 1.0 / self.ls.cs2
        self.k = 0
        self.S_phi = 0.0
        self.J_U = 0.0
        self.init()

    # ------------------------------------------------------------- init
    def coords(self):
        idx = np.indices(self.shape, dtype=np.float64)
        return idx[::-1]  # (x, y[, z])

    def init_phi(self) -> np.ndarray:
        """phi(x, 0) = tanh[(R0 - r)/(sqrt(2) W0)] (Section 4.1), max over
        seeds; the 3D directional case uses a planar front at z_front with
        per-column offsets xi(x, y) (random form of Eq. 41)."""
        d = self.d
        X = self.coords()
        s2w = math.sqrt(2.0) * d["W0"]
        if "perturb" in d:
            xi = np.asarray(d["perturb"], dtype=np.float64)
            if self.dim == 3:
                return np.tanh((d["z_front"] + xi[None, :, :] - X[2]) / s2w)
            return np.tanh((d["z_front"] + xi[None, :] - X[1]) / s2w)
        phi = np.full(self.shape, -1.0)
        for s in d["seeds"]:
            c = s[: self.dim]
            R = s[self.dim]
            r = np.sqrt(sum((X[a] - c[a]) ** 2 for a in range(self.dim)))
            phi = np.maximum(phi, np.tanh((R - r) / s2w))
        return phi

    def init(self):
        d = self.d
        ls = self.ls
        nd = self.dim
        self.phi = self.init_phi()
        # initial velocity (forced convection starts from u_in * f_L along x)
        self.u = np.zeros((nd,) + self.shape)
        if d["has_flow"] and d.get("u0_liquid_only", False):
            self.u[0] = d["u_in"] * (1.0 - self.phi) / 2.0
        self.rho = np.ones(self.shape)
        w = _wq(ls, nd)
        # phase populations at equilibrium with v_n = 0 (Eq. 21)
        self.f_phi = w * self.phi[None]
        self.U = np.full(self.shape, float(d["U0"]))
        self.T = np.full(self.shape, float(d["T0"]))
        if d.get("T_mode") == "pulled":
            self.T = self.pulled_T(self.coords()[nd - 1], 0.0)
        if d["has_U"]:
            self.f_U = self.scalar_eq(self.U, P.dt_field(d, "U"))
        if d["has_T"]:
            self.f_T = self.scalar_eq(self.T, P.dt_field(d, "T"), self.velocity_T())
        if d["has_flow"]:
            self.f_F = self.flow_eq(self.rho, self.u, P.dt_field(d, "F"))
        self.P_U = np.zeros(self.shape)
        self.P_T = np.zeros(self.shape)
        if d.get("grad_phi", "fd") == "eq40":
            self.vn_prev = np.zeros((nd,) + self.shape)   # v_n of the previous phase step
            self.A_prev = np.ones(self.shape)               # a_s^2 of the previous phase step

    # ------------------------------------------------------------- equilibria
    def scalar_eq(self, chi, dt, u=None):
        """Eq. (19): f_i^eq = w_i chi (1 + 3 e_i.u / c) with c = 1/dt (the
        factor 3 is 1/c_s^2 of the scalar lattice)."""
        w = _wq(self.ls, self.dim)
        u = self.u if u is None else u
        return w * chi[None] * (1.0 + self.inv_cs2 * _edot(self.ls, u) * dt)

    def velocity_T(self):
        """Advection velocity of T: the flow velocity, plus the pulling
        velocity V along the last axis for the pulled temperature."""
        if self.d.get("T_mode") != "pulled":
            return self.u
        u = self.u.copy()
        u[self.dim - 1] = u[self.dim - 1] + self.d["V_pull"]
        return u

    def pulled_T(self, z, t):
        """Moving linear profile T_L + G (z - z_front - V t), T_L = T0 (the
        cold bottom is the case G = V = 0)."""
        d = self.d
        if d.get("T_mode") == "dirichlet_low":
            return d["T0"] + 0.0 * z
        return d["T0"] + d["T_grad"] * (z - d["z_front"] - d["V_pull"] * t)

    def flow_eq(self, rho, u, dt):
        """Eq. (28) with c_F = 1/dt_F."""
        lf = self.lf
        w = _wq(lf, self.dim)
        eu = _edot(lf, u) * dt
        uu = np.sum(u * u, axis=0) * dt * dt
        return w * rho[None] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu[None])

    # ------------------------------------------------------------- phase
    def phase_step(self):
        """One phase update: Eq. (14) with Eq. (21)-(23) and the source
        dt_phi w_i Q_phi / tau0, then the anisotropic streaming of Eq. (26)
        in pull form with a_s^2 at the destination.  Returns (phi_q, phi_new)."""
        d = self.d
        ls = self.ls
        nd = self.dim
        dt = P.dt_field(d, "phi")
        f = self.f_phi
        phi_q = f.sum(axis=0)
        eq40 = d.get("grad_phi", "fd") == "eq40"
        if eq40:   # Eq. (40) with the previous step's equilibrium and tau_phi
            j = np.tensordot(ls.e.astype(np.float64).T, f, axes=(1, 0))
            g = -(self.inv_cs2 / P.tau_phi(d, self.A_prev))[None] * (j - self.vn_prev * dt)
        else:
            g = grad_iso(phi_q, self.bc)
        a_s, N, _ = anisotropy(d, g)
        A = a_s * a_s
        v_n = -d["W0"] ** 2 * N / d["tau0"]                  # Eq. (21)
        tau = P.tau_phi(d, A)                                  # Eq. (24)
        if eq40:
            self.A_prev, self.vn_prev = A, v_n
        Ustar = self.U if d["has_U"] else np.zeros(self.shape)
        theta = P.theta_of_T(d, self.T) if d["has_T"] else np.zeros(self.shape)
        om = 1.0 - phi_q * phi_q
        Q = phi_q * om - d["lam"] * (d["Mc"] * Ustar + theta) * om * om   # Eq. (4)
        w = _wq(ls, nd)
        feq = w * (phi_q[None] + self.inv_cs2 * _edot(ls, v_n) * dt)      # Eq. (21)
        post = mrt_collide(ls, f, feq, scalar_relaxation(ls, tau))
        post = post + dt * w * (Q / d["tau0"])[None]
        pulled = pull(post, ls, self.bc)
        f_new = (pulled - (1.0 - A)[None] * f) / A[None]                 # Eq. (26)
        self.f_phi = f_new
        phi_new = f_new.sum(axis=0)
        self.phi = phi_new
        return phi_q, phi_new

    # ------------------------------------------------------------- transfer
    def transfer(self, phi_q, phi_new):
        """Eq. (36)-(39): increments from the resolved phase change, with the
        time-integrated anti-trapping current and its compact divergence."""
        d = self.d
        nd = self.dim
        w = _wq(self.ls, nd)
        dphi = phi_new - phi_q                                            # Eq. (36)
        n1 = unit_normal(grad_iso(phi_new, self.bc))
        if d["has_U"]:
            coef = 1.0 + (1.0 - d["k"]) * self.U
            J = d["W0"] / (2.0 * math.sqrt(2.0)) * coef[None] * dphi[None] * n1   # Eq. (37)
            dU = (coef * dphi - 2.0 * div_iso(J, self.bc)) / P.kfac(d, phi_new)  # Eq. (38)
            self.S_phi = float(np.max(np.abs(dU)))
            if d["coupling"] == "instant":
                self.U = self.U + dU                                      # Eq. (39)
                self.f_U = self.f_U + w * dU[None]
                self.J_U = self.S_phi
            else:
                self.P_U = self.P_U + dU
        if d["has_T"] and d.get("T_mode", "transport") != "pulled":
            dT = d["rho_L"] * d["L_h"] * dphi / (2.0 * P.rhoCp_eff(d, phi_new))  # Eq. (38)
            if d["coupling"] == "instant":
                self.T = self.T + dT
                self.f_T = self.f_T + w * dT[None]
            else:
                self.P_T = self.P_T + dT

    # ------------------------------------------------------------- U and T
    def scalar_step(self, which: str):
        """One transport update of U or T: Eq. (14) with Eq. (19)-(20), (23),
        (24), the transport part of the source (first terms of Eq. 8 / 12, per
        Eq. 35) with grad chi from Eq. (40) and grad phi* by the isotropic
        stencil, then Eq. (25) and the reconstruction chi = sum f."""
        d = self.d
        ls = self.ls
        nd = self.dim
        dt = P.dt_field(d, which)
        f = self.f_U if which == "U" else self.f_T
        phis = self.phi
        chi = f.sum(axis=0)
        if which == "U":
            coeff = P.D_eff(d, phis)
        else:
            coeff = P.alpha_eff(d, phis)
        tau = self.inv_cs2 * dt * coeff + 0.5                            # Eq. (24)
        uadv = self.u if which == "U" else self.velocity_T()
        feq = self.scalar_eq(chi, dt, uadv)
        E = ls.e.astype(np.float64)
        neq = f - feq
        grad_chi = -(self.inv_cs2 / tau)[None] * np.tensordot(E[1:].T, neq[1:], axes=(1, 0))  # Eq. (40)
        gphi = grad_iso(phis, self.bc)
        gdot = np.sum(grad_chi * gphi, axis=0)
        if which == "U":
            Qtr = -(1.0 - d["k"]) * coeff * gdot / P.kfac(d, phis)      # Eq. (8), 1st term
        else:
            Qtr = ((d["rhoCp_S"] - d["rhoCp_L"]) / (2.0 * P.rhoCp_eff(d, phis))
                   * coeff * gdot)                                         # Eq. (12), 1st term
        w = _wq(ls, nd)
        post = mrt_collide(ls, f, feq, scalar_relaxation(ls, tau)) + dt * w * Qtr[None]
        f_new = pull(post, ls, self.bc)                                   # Eq. (25)
        if which == "T" and d.get("T_mode") in ("pulled", "dirichlet_low"):
            # anti-bounce-back on the walls of the last axis: populations whose
            # upstream node lies beyond the wall z_w = -1/2 or nz - 1/2 become
            # -f^+_ibar(y) + 2 w_i T(z_w) at the middle of the T step (the
            # cold bottom holds T0: only the low wall, G = V = 0)
            ax = nd - 1
            n = self.shape[0]
            t_mid = (self.k - 0.5 * d["N_T"]) * d["dt_base"]
            low_only = d.get("T_mode") == "dirichlet_low"
            for i in range(ls.Q):
                ez = int(ls.e[i, ax])
                if ez == 0 or (low_only and ez < 0):
                    continue
                zw = -0.5 if ez > 0 else n - 0.5
                src = np.arange(n) - ez
                m = ((src < 0) | (src >= n)).reshape((n,) + (1,) * (nd - 1))
                m = np.broadcast_to(m, self.shape)
                abb = -post[ls.opp[i]] + 2.0 * ls.w[i] * self.pulled_T(zw, t_mid)
                f_new[i] = np.where(m, abb, f_new[i])
        chi_new = f_new.sum(axis=0)
        if d["coupling"] != "instant":
            Pend = self.P_U if which == "U" else self.P_T
            f_new = f_new + w * Pend[None]
            chi_new = chi_new + Pend
            if which == "U":
                self.J_U = float(np.max(np.abs(Pend)))
                self.P_U = np.zeros(self.shape)
            else:
                self.P_T = np.zeros(self.shape)
        if which == "U":
            self.f_U, self.U = f_new, chi_new
        else:
            self.f_T, self.T = f_new, chi_new

    # ------------------------------------------------------------- flow
    def guo_moments(self, F, u, c):
        """Eq. (30): Guo forcing in moment space (D2Q9)."""
        Fx, Fy = F[0], F[1]
        ux, uy = u[0], u[1]
        Fu = Fx * ux + Fy * uy
        z = np.zeros_like(ux)
        return np.stack([
            z, 6.0 * Fu / c ** 2, -6.0 * Fu / c ** 2,
            Fx / c + z, -Fx / c + z, Fy / c + z, -Fy / c + z,
            2.0 * (Fx * ux - Fy * uy) / c ** 2, (Fy * ux + Fx * uy) / c ** 2,
        ])

    def flow_relaxation(self) -> np.ndarray:
        """Eq. (31): S^F = diag(0, s_e, s_eps, 0, s_q, 0, s_q, s_nu, s_nu)
        in 2D; in 3D the conserved rows relax at 0, the stress rows at s_nu,
        |e|^2 at s_e, |e|^4 at s_eps and all flux/ghost rows at s_q."""
        d = self.d
        snu = 1.0 / P.tau_F(d)
        if self.dim == 2:
            return np.array([0.0, d["s_e"], d["s_eps"], 0.0, d["s_q"], 0.0, d["s_q"], snu, snu])
        s = np.full(19, d["s_q"])
        s[0:4] = 0.0
        s[4] = d["s_e"]
        s[5] = d["s_eps"]
        s[6:11] = snu
        return s

    def flow_step(self):
        """One flow update: Eq. (27)-(32) collision, Eq. (33) partial
        bounce-back with f_L = (1 - phi*)/2, then inlet/outflow columns."""
        d = self.d
        lf = self.lf
        nd = self.dim
        dt = P.dt_field(d, "F")
        c = 1.0 / dt
        f = self.f_F
        F = np.zeros((nd,) + self.shape) + np.asarray(d["Fb"][:nd]).reshape((nd,) + (1,) * nd)
        rho = f.sum(axis=0)
        j = np.tensordot(lf.e.astype(np.float64).T, f, axes=(1, 0))
        u = (c * j + dt * F / 2.0) / rho[None]                          # Eq. (27)
        feq = self.flow_eq(rho, u, dt)                                   # Eq. (28)
        if nd == 2:
            G = self.guo_moments(F, u, c)                                # Eq. (30)
        else:
            G = _mv(lf.M, self.guo_velocity_space(F, u, c))
        post = mrt_collide(lf, f, feq, self.flow_relaxation(), G=G)     # Eq. (14)
        fL = (1.0 - self.phi) / 2.0
        fbc = tuple("periodic" if b == "periodic" else "wall" for b in self.fbc)
        out = np.empty_like(post)
        for i in range(lf.Q):
            m = 0.5 * (fL + upstream(fL, lf.e[i], fbc))                 # f_L at the link midpoint
            src = upstream(post[i], lf.e[i], fbc)                        # post_i(y - e_i)
            bounce = post[lf.opp[i]]
            val = m * src + (1.0 - m) * bounce                            # Eq. (33)
            outside = source_outside(self.shape, lf.e[i], fbc)
            val = np.where(outside, bounce, val)
            out[i] = val
        if self.fbc[0] == "inlet_outflow":
            uin = np.zeros((nd,) + self.shape[:-1] + (1,))
            uin[0] = d["u_in"]
            col = self.flow_eq(np.ones(self.shape[:-1] + (1,)), uin, dt)
            out[..., 0:1] = col
            out[..., -1:] = out[..., -2:-1]
        self.f_F = out
        rho = out.sum(axis=0)
        j = np.tensordot(lf.e.astype(np.float64).T, out, axes=(1, 0))
        self.rho = rho
        self.u = (c * j + dt * F / 2.0) / rho[None]

    def guo_velocity_space(self, F, u, c):
        """Guo's discrete force in velocity space,
        F_i = w_i [3 (e_i - u/c) . F + 9 (e_i . u/c)(e_i . F)] / c,
        whose D2Q9 moments are Eq. (30); used as M F_i on the 3D lattice."""
        lf = self.lf
        w = _wq(lf, self.dim)
        eu = _edot(lf, u) / c
        eF = _edot(lf, F)
        uF = np.sum(u * F, axis=0)
        return w * (3.0 * (eF - uF[None] / c) + 9.0 * eu * eF) / c

    # ------------------------------------------------------------- schedule
    def step(self):
        """One base step k -> k+1 of Eq. (34): each field runs iff
        k mod N_chi == 0, in the order phi (+transfer), U, T, flow."""
        d = self.d
        self.k += 1
        k = self.k
        if k % d["N_phi"] == 0:
            phi_q, phi_new = self.phase_step()
            self.transfer(phi_q, phi_new)
        if d["has_U"] and k % d["N_U"] == 0:
            self.scalar_step("U")
        if d["has_T"] and k % d["N_T"] == 0:
            self.scalar_step("T")
        if d["has_flow"] and k % d["N_F"] == 0:
            self.flow_step()

    # ------------------------------------------------------------- views
    def moments(self, which: str):
        """(chi, j) of a scalar field's populations: j = sum_i f_i e_i."""
        f = {"phi": self.f_phi, "U": getattr(self, "f_U", None), "T": getattr(self, "f_T", None)}[which]
        E = self.ls.e.astype(np.float64)
        return f.sum(axis=0), np.tensordot(E.T, f, axes=(1, 0))


def run(d: dict, steps: int) -> Domain:
    dom = Domain(d)
    for _ in range(steps):
        dom.step()
    return dom
