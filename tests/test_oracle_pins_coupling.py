"""Pins of the oracle's accumulated-coupling branch, its inlet/outflow
columns, and the stability margin of the anisotropic streaming (Eq. 26).

The accumulated coupling is the ablation of Section 4.4: the phase-change
increments of Eq. (38) are summed and injected after the field's next
transport update instead of at every phase step (Eq. 39).  Two properties
fix that branch independently of the oracle's own code:

* with k = 1 the transport source of Eq. (8) vanishes (its first term
  carries 1 - k) and the denominator (1 + k) - (1 - k) phi is 2, so the
  transfer adds sum(dphi)/2 to the total of U (the compact divergence of
  the anti-trapping current telescopes to zero in a closed box) and the U
  transport conserves sum U; hence sum(U + P_U) - sum(phi)/2 is invariant
  at every base step, and P_U is empty after every U update;
* the injection comes after the transport: a pending increment over a
  uniform U is added unchanged by one U update (a transport before the
  injection would diffuse it).

The inlet/outflow columns (Section 3.2.2 names the boundary kinds; the
schemes are a reading: equilibrium at the inlet, zero-gradient copy at the
outflow) are pinned by two facts of an empty channel: uniform flow at the
inlet velocity is a fixed point, and a channel started at rest relaxes to
it.

The last group is a frozen-coefficient linear stability analysis of the
phase update (Eq. 14 with Eq. 21-23 and Eq. 26): the amplification matrix
of a Fourier mode, and the closed form of the growth of a uniform flux
perturbation, g = [(1 - 1/tau_phi) - (1 - A)] / A, which the oracle must
reproduce.
"""

import math

import numpy as np
import pytest

import lbm_inputs as L
import oracle
from oracle import lattice as LT


def _dom(**kw):
    d = L.configs._base_domain()
    d.update(kw)
    return d


# ------------------------------------------------- accumulated coupling
def _closed_solutal(coupling, N_U, **kw):
    """A solutal seed in a walled box with k = 1 (Section 4.2 scales)."""
    d = _dom(nx=26, ny=22, has_U=True, N_U=N_U, dt_base=0.25, W0=2.5, tau0=50.0,
             eps_s=0.02, lam=0.8839 / 0.2762, Mc=1.0, k=1.0, D_L=0.25, D_S=0.0025,
             U0=-0.55, bc=("wall", "wall", "wall"), seeds=[(12.3, 10.6, 6.0)],
             coupling=coupling)
    d.update(kw)
    return d


@pytest.mark.parametrize("coupling", ["accum", "instant"])
def test_accumulated_coupling_conserves_pending_solute(coupling):
    """k = 1: sum(U + P_U) - sum(phi)/2 is invariant at every base step
    (Eq. 8 transport source zero, Eq. 38 with kfac = 2, compact divergence
    summing to zero with mirrored walls), and P_U = 0 right after every U
    update of the accumulated variant (Section 4.4)."""
    N_U = 4
    dom = oracle.Domain(_closed_solutal(coupling, N_U))
    inv0 = np.sum(dom.U + dom.P_U) - 0.5 * np.sum(dom.phi)
    scale = np.sum(np.abs(dom.U)) + np.sum(np.abs(dom.phi))
    grew = 0.0
    for k in range(1, 41):
        phi_before = dom.phi.copy()
        dom.step()
        grew = max(grew, float(np.max(np.abs(dom.phi - phi_before))))
        inv = np.sum(dom.U + dom.P_U) - 0.5 * np.sum(dom.phi)
        assert abs(inv - inv0) <= 1e-13 * scale, (k, inv - inv0)
        if coupling == "accum":
            if k % N_U == 0:
                assert np.all(dom.P_U == 0.0), k
            else:
                assert np.any(dom.P_U != 0.0), k
        else:
            assert np.all(dom.P_U == 0.0)
    assert grew > 1e-4   # the seed does grow: the invariant is not trivially met


def test_accumulated_thermal_coupling_conserves_pending_enthalpy():
    """Constant thermal properties: the T transport source of Eq. (12)
    vanishes and Eq. (38) adds rho_L L_h dphi / (2 rhoCp) to T, so
    sum(T + P_T) - rho_L L_h sum(phi) / (2 rhoCp) is invariant, and P_T = 0
    after every T update of the accumulated variant."""
    N_T = 3
    d = _dom(nx=24, ny=20, has_T=True, N_T=N_T, dt_base=0.5, W0=1.0, tau0=20.0, eps_s=0.05,
             lam=0.8839 / 0.1385, kappa_S=0.2, kappa_L=0.2, rhoCp_S=1.0, rhoCp_L=1.0,
             T0=-0.55, bc=("wall", "periodic", "wall"), seeds=[(11.5, 9.5, 5.0)],
             coupling="accum")
    dom = oracle.Domain(d)
    c = d["rho_L"] * d["L_h"] / (2.0 * d["rhoCp_L"])
    inv0 = np.sum(dom.T + dom.P_T) - c * np.sum(dom.phi)
    scale = np.sum(np.abs(dom.T)) + c * np.sum(np.abs(dom.phi))
    for k in range(1, 31):
        dom.step()
        inv = np.sum(dom.T + dom.P_T) - c * np.sum(dom.phi)
        assert abs(inv - inv0) <= 1e-13 * scale, (k, inv - inv0)
        if k % N_T == 0:
            assert np.all(dom.P_T == 0.0), k


def _gaussian(shape, c, sigma, amp):
    ny, nx = shape
    X, Y = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    return amp * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * sigma ** 2))


@pytest.mark.parametrize("q", [5, 9])
def test_pending_increment_is_injected_after_the_transport(q):
    """Section 4.4 accumulated variant: a pending increment P over a uniform
    U0 (phi = -1 everywhere, so no phase change and no transport source)
    leaves U = U0 + P after one U update, exactly: the transport acts on the
    uniform state (a fixed point) and the increment is added afterwards.
    The next U update then transports it: total solute kept, peak lowered."""
    d = _dom(nx=20, ny=18, has_U=True, N_U=4, dt_base=0.25, W0=2.5, tau0=50.0,
             eps_s=0.02, lam=3.2, Mc=1.0, k=0.15, D_L=0.25, D_S=0.0025, U0=-0.55,
             bc=("wall", "periodic", "wall"), coupling="accum", q_scalar=q)
    dom = oracle.Domain(d)
    P = _gaussian(dom.shape, (8.3, 9.1), 1.5, 0.02)
    dom.P_U = P.copy()
    for _ in range(4):        # phase steps 1-3 add nothing; step 4 runs U
        dom.step()
    assert np.max(np.abs(dom.U - (d["U0"] + P))) <= 1e-15
    assert np.all(dom.P_U == 0.0)
    w = dom.ls.w.reshape((dom.ls.Q, 1, 1))
    assert np.max(np.abs(dom.f_U - w * (d["U0"] + P)[None])) <= 1e-15
    peak = np.max(dom.U - d["U0"])
    for _ in range(4):
        dom.step()
    assert np.max(dom.U - d["U0"]) < 0.9 * peak
    assert abs(np.sum(dom.U - d["U0"]) - np.sum(P)) <= 1e-13


# ------------------------------------------------- inlet and outflow
def _channel(u0_liquid_only, nx=40, ny=6, nu=0.1):
    return _dom(nx=nx, ny=ny, has_flow=True, N_F=1, u_in=0.01, nu=nu,
                bc=("wall", "periodic", "wall"),
                flow_bc=("inlet_outflow", "periodic", "periodic"),
                u0_liquid_only=u0_liquid_only)


def test_uniform_inlet_flow_is_a_fixed_point():
    """An empty channel (phi = -1, f_L = 1) started at f_eq(1, (u_in, 0))
    stays there: the inlet column is that equilibrium, the outflow copies a
    column equal to it, and the interior streams a uniform state."""
    d = _channel(True)
    dom = oracle.Domain(d)
    f0 = dom.f_F.copy()
    assert np.allclose(dom.u[0], d["u_in"], atol=0, rtol=0)
    for _ in range(50):
        dom.step()
    assert np.max(np.abs(dom.f_F - f0)) <= 1e-16
    assert np.max(np.abs(dom.u[0] - d["u_in"])) <= 1e-15
    assert np.max(np.abs(dom.u[1])) <= 1e-16


def test_channel_at_rest_reaches_the_inlet_flux_balance():
    """The same channel started at rest (rho = 1, u = 0) reaches a uniform
    interior state (rho', u') whose mass flux balances the inlet link: the
    right-moving D2Q9 populations of f_eq(1, (u_in, 0)) at x = 0 minus the
    left-moving ones of f_eq(rho', (u', 0)) at x = 1 carry rho' u', i.e.
    rho' (1 + 3u' + 3u'^2) = 1 + 3u_in + 3u_in^2 (Eq. 28 summed over each
    half of the lattice).  The inlet fixes the flux, not the interior
    velocity: from rest the channel settles at u' = 0.75 u_in with a
    raised density (a wrong inlet velocity or sign, or an outflow column
    that reflects, breaks the balance or the uniformity)."""
    d = _channel(False, nx=24, ny=4, nu=0.5)
    dom = oracle.Domain(d)
    for _ in range(2000):
        dom.step()
    rho, u = dom.rho[:, 1:], dom.u[0][:, 1:]
    assert np.ptp(rho) <= 1e-13 and np.ptp(u) <= 1e-13
    assert np.max(np.abs(dom.u[1])) <= 1e-15
    r, v, ui = rho[0, 0], u[0, 0], d["u_in"]
    assert abs(r * (1 + 3 * v + 3 * v * v) - (1 + 3 * ui + 3 * ui * ui)) <= 1e-13
    assert 0.5 * ui < v < ui and r > 1.0


# ------------------------------------------------- stability of Eq. (26)
def _amplification(lat, A, tau, kx, ky, post_reading=False):
    """Frozen-coefficient amplification matrix of one phase update for the
    Fourier mode exp(i k.x): collision of Eq. (14) with S of Eq. (23) and
    f_eq = w_i phi (Eq. 21 without v_n), then Eq. (26):
    A f_i(y, t+1) = f_i^+(y - e_i) - (1 - A) f_i(y, t).  The alternative
    reading takes the post-collision value at y in the last term."""
    Q = lat.Q
    E = lat.e.astype(float)
    S = np.ones(Q)
    for r in lat.flux_rows:
        S[r] = 1.0 / tau
    proj = np.eye(Q) - np.outer(lat.w, np.ones(Q))        # f - f_eq(sum f)
    C = np.eye(Q) - lat.Minv @ np.diag(S) @ lat.M @ proj
    D = np.diag(np.exp(-1j * (E[:, 0] * kx + E[:, 1] * ky)))
    if post_reading:
        return (D - (1.0 - A) * np.eye(Q)) @ C / A
    return (D @ C - (1.0 - A) * np.eye(Q)) / A


def _spectral_radius(lat, A, tau, post_reading=False, n=17):
    r = 0.0
    for kx in np.linspace(0.0, math.pi, n):
        for ky in np.linspace(0.0, math.pi, n):
            r = max(r, float(np.max(np.abs(np.linalg.eigvals(
                _amplification(lat, A, tau, kx, ky, post_reading))))))
    return r


def _A_tau(W0, tau0, eps, s4):
    a = 1.0 - 3.0 * eps + 4.0 * eps * s4          # Eq. (2), s4 = n_x^4 + n_y^4
    A = a * a
    return A, 3.0 * A * W0 * W0 / tau0 + 0.5        # Eq. (24), dt_phi = 1


def test_section43_scale_is_linearly_unstable_under_every_reading():
    """At the Section 4.3 scale (W0 = 2, tau0 = 1000, eps = 0.02) the
    phase update has modes growing per step on both lattices and under both
    readings of the last term of Eq. (26), where the normal lies along a
    diagonal (A = (1 - eps)^2); the plain D2Q9 update with the relaxation
    of Eq. (23) is unstable there even at A = 1.  At the scales that are
    run (tau0 = 100 for the enlarged four-field case, 150 for the
    directional case of Section 4.4) no mode grows."""
    diag = _A_tau(2.0, 1000.0, 0.02, 0.5)
    for lat in (LT.D2Q5, LT.D2Q9):
        for post in (False, True):
            assert _spectral_radius(lat, *diag, post_reading=post) > 1.03
    assert _spectral_radius(LT.D2Q9, 1.0, 0.512) > 1.005
    assert _spectral_radius(LT.D2Q5, 1.0, 0.512) <= 1.0 + 1e-12
    for tau0 in (100.0, 150.0):
        for s4 in (0.5, 0.75, 1.0):
            A, tau = _A_tau(2.0, tau0, 0.02, s4)
            for lat in (LT.D2Q5, LT.D2Q9):
                assert _spectral_radius(lat, A, tau) <= 1.0 + 1e-12, (tau0, s4, lat)


@pytest.mark.parametrize("q", [5, 9])
@pytest.mark.parametrize("diagonal,tau0", [(True, 1000.0), (False, 1000.0), (True, 100.0)])
def test_oracle_flux_mode_grows_at_the_closed_form_rate(q, diagonal, tau0):
    """A uniform flux perturbation on a field whose normal is uniform (a
    small plane wave along a diagonal or an axis, so A is the same at every
    site and the correction vector N vanishes) is multiplied per phase step
    by g = [(1 - 1/tau_phi) - (1 - A)] / A.  On the diagonal at the
    Section 4.3 scale |g| = 1.036: the mode behind the divergence of that
    parameter set."""
    n, W0, eps = 30, 2.0, 0.02
    d = _dom(nx=n, ny=n, W0=W0, tau0=tau0, eps_s=eps, lam=1.5955, q_scalar=q)
    dom = oracle.Domain(d)
    X, Y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    s = X + Y if diagonal else X
    phi = -1.0 + 1e-3 * np.sin(2 * math.pi * s / n)
    w = dom.ls.w.reshape((dom.ls.Q, 1, 1))
    E = dom.ls.e.astype(float)
    j0 = np.array([1e-6, 0.5e-6])
    dom.f_phi = w * phi[None] + 3.0 * w * (E @ j0)[:, None, None]
    js = []
    for _ in range(11):
        dom.step()
        js.append(np.tensordot(E.T, dom.f_phi, axes=(1, 0)).mean(axis=(1, 2))[0])
    A, tau = _A_tau(W0, tau0, eps, 0.5 if diagonal else 1.0)
    g = ((1.0 - 1.0 / tau) - (1.0 - A)) / A
    assert abs(js[10] / js[9] - g) <= 1e-7 * abs(g), (js[10] / js[9], g)
    if diagonal and tau0 == 1000.0:
        assert abs(g) > 1.035
    else:
        assert abs(g) < 0.9


# ------------------------------------------------- Eq. (40) for the phase field
@pytest.mark.parametrize("q", [5, 9])
def test_eq40_phase_gradient_recovers_the_wave_gradient(q):
    """The grad_phi = "eq40" variant: grad phi = -(3/tau_prev)(j - v_n,prev
    dt_phi) from the phase populations (Eq. 40 with the previous step's
    equilibrium).  On a small oblique plane wave (wave vector 2pi(2, 1)/64,
    so the normal is off both axes and the correction vector N, hence v_n,
    does not vanish; amplitude 1e-3, so the wave stays a single mode) the
    recovered gradient equals the mode's analytic gradient to 1.5 % after
    40 steps, while leaving out the equilibrium flux v_n dt would be off by
    about 7 %."""
    n = 64
    d = _dom(nx=n, ny=n, W0=2.0, tau0=40.0, eps_s=0.05, lam=0.0, q_scalar=q, grad_phi="eq40")
    dom = oracle.Domain(d)
    X, Y = np.meshgrid(np.arange(float(n)), np.arange(float(n)))
    arg = 2 * math.pi * (2 * X + Y) / n
    w = dom.ls.w.reshape((dom.ls.Q, 1, 1))
    dom.f_phi = w * (1e-3 * np.sin(arg))[None]
    for _ in range(40):
        dom.step()
    phi = dom.f_phi.sum(axis=0)
    E = dom.ls.e.astype(float)
    j = np.tensordot(E.T, dom.f_phi, axes=(1, 0))
    tau = 3.0 * dom.A_prev * d["W0"] ** 2 / d["tau0"] + 0.5        # Eq. (24), dt_phi = 1
    g40 = -(3.0 / tau)[None] * (j - dom.vn_prev)                   # Eq. (40)
    s, c = np.sin(arg), np.cos(arg)
    a_s, a_c = np.sum(phi * s) / np.sum(s * s), np.sum(phi * c) / np.sum(c * c)
    kx, ky = 2 * math.pi * 2 / n, 2 * math.pi / n
    ga = np.stack([kx * (a_s * c - a_c * s), ky * (a_s * c - a_c * s)])
    scale = np.max(np.abs(ga))
    assert np.max(np.abs(g40 - ga)) <= 0.015 * scale
    assert np.max(np.abs(3.0 / tau[None] * dom.vn_prev)) >= 0.05 * scale   # the v_n term matters
    assert np.max(np.abs(-(3.0 / tau)[None] * j - ga)) >= 0.04 * scale
