"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the pin it implements and the passage it follows.  None of
them compares the oracle with itself: they use printed moment vectors,
closed-form solutions, invariants, special cases, an independent spectral
solution of the continuum equations, and printed parameter values.
"""

import json
import math
import os

import numpy as np
import pytest

import lbm_inputs as L
import oracle
from oracle import lattice as LT
from oracle import model
from oracle import params as P
from oracle.stencils import div_iso, grad_iso

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "printed_parameters.json")


def _dom(**kw):
    d = L.configs._base_domain()
    d.update(kw)
    return d


# --------------------------------------------------------------------- K1
def test_moment_bases_orthogonal():
    """Eq. (16): the D2Q9 rows are orthogonal with squared norms
    (9, 36, 36, 6, 12, 6, 12, 4, 4); the D2Q5 rows (5, 2, 2, 20, 4)."""
    for lat, norms in ((LT.D2Q9, (9, 36, 36, 6, 12, 6, 12, 4, 4)), (LT.D2Q5, (5, 2, 2, 20, 4))):
        G = lat.M @ lat.M.T
        assert np.allclose(G, np.diag(norms), atol=0, rtol=0)
    for lat in (LT.D3Q7, LT.D3Q19):
        G = lat.M @ lat.M.T
        assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12)
        assert np.all(np.diag(G) > 0.5)
    # lattice isotropy: sum w = 1, sum w e = 0, sum w e e = c_s^2 I
    for lat in (LT.D2Q9, LT.D2Q5, LT.D3Q7, LT.D3Q19):
        E = lat.e.astype(float)
        assert abs(lat.w.sum() - 1) < 1e-15
        assert np.allclose(lat.w @ E, 0)
        assert np.allclose(np.einsum("i,ia,ib->ab", lat.w, E, E), lat.cs2 * np.eye(lat.d))


def test_equilibrium_moments_match_printed_vectors():
    """K1: M f^eq equals the printed moment vectors of Eq. (20), (22), (29)."""
    rng = np.random.default_rng(1)
    d = _dom(nx=5, ny=4, has_U=True, has_flow=True, N_U=3, N_F=2, dt_base=0.5)
    dom = oracle.Domain(d)
    U = rng.uniform(-1, 1, dom.shape)
    u = rng.uniform(-0.05, 0.05, (2,) + dom.shape)
    dom.u = u
    M = LT.D2Q9.M
    # Eq. (20) on D2Q9 scalars
    dom9 = oracle.Domain(dict(d, q_scalar=9))
    dom9.u = u
    dtU = 3 * 0.5
    cU = 1 / dtU
    m = np.tensordot(M, dom9.scalar_eq(U, dtU), axes=(1, 0))
    ux, uy = u
    ref = np.stack([U, -2 * U, U, ux * U / cU, -ux * U / cU, uy * U / cU, -uy * U / cU, 0 * U, 0 * U])
    assert np.allclose(m, ref, atol=1e-15)
    # Eq. (22): phase equilibrium w_i (phi + 3 e_i.v_n / c)
    phi = rng.uniform(-1, 1, dom.shape)
    vn = rng.uniform(-0.1, 0.1, (2,) + dom.shape)
    c = 1 / 0.5
    feq = LT.D2Q9.w[:, None, None] * (phi[None] + 3 * np.tensordot(LT.D2Q9.e.astype(float), vn, axes=(1, 0)) / c)
    m = np.tensordot(M, feq, axes=(1, 0))
    ref = np.stack([phi, -2 * phi, phi, vn[0] / c, -vn[0] / c, vn[1] / c, -vn[1] / c, 0 * phi, 0 * phi])
    assert np.allclose(m, ref, atol=1e-15)
    # Eq. (29): flow equilibrium
    rho = rng.uniform(0.9, 1.1, dom.shape)
    dtF = 2 * 0.5
    cF = 1 / dtF
    m = np.tensordot(M, dom.flow_eq(rho, u, dtF), axes=(1, 0))
    u2 = ux ** 2 + uy ** 2
    ref = rho * np.stack([1 + 0 * rho, -2 + 3 * u2 / cF ** 2, 1 - 3 * u2 / cF ** 2, ux / cF, -ux / cF,
                          uy / cF, -uy / cF, (ux ** 2 - uy ** 2) / cF ** 2, ux * uy / cF ** 2])
    assert np.allclose(m, ref, atol=1e-14)
    # D2Q5 scalar equilibrium: zeroth moment chi, flux chi u / c, isotropic rest
    m5 = np.tensordot(LT.D2Q5.M, dom.scalar_eq(U, dtU), axes=(1, 0))
    assert np.allclose(m5[0], U) and np.allclose(m5[1], U * ux / cU) and np.allclose(m5[2], U * uy / cU)
    assert np.allclose(m5[3], -2 * U / 3) and np.allclose(m5[4], 0)


def test_guo_moments_equal_velocity_space_guo():
    """Eq. (30) equals the moments of Guo's velocity-space discrete force."""
    rng = np.random.default_rng(2)
    d = _dom(nx=4, ny=3, has_flow=True, N_F=3, dt_base=0.25)
    dom = oracle.Domain(d)
    F = rng.uniform(-1e-3, 1e-3, (2,) + dom.shape)
    u = rng.uniform(-0.05, 0.05, (2,) + dom.shape)
    c = 1 / 0.75
    G = dom.guo_moments(F, u, c)
    Fi = dom.guo_velocity_space(F, u, c)
    assert np.allclose(np.tensordot(LT.D2Q9.M, Fi, axes=(1, 0)), G, atol=1e-17)


# --------------------------------------------------------------------- K2, K3, K9
def _random_state(shape, Q, rng):
    return rng.uniform(0.01, 0.2, (Q,) + shape)


@pytest.mark.parametrize("lat", [LT.D2Q5, LT.D2Q9, LT.D3Q7])
def test_scalar_collision_closed_form_and_conservation(lat):
    """K2 + K3: the literal Eq. (14) collision with the relaxation of Eq. (23)
    conserves the zeroth moment and equals the closed form
    f_i^eq + (1 - 1/tau)(j - j^eq).e_i / (sum_k e_kx^2) + source."""
    rng = np.random.default_rng(3)
    shape = (3, 4) if lat.d == 2 else (2, 3, 4)
    f = _random_state(shape, lat.Q, rng)
    chi = f.sum(0)
    u = rng.uniform(-0.1, 0.1, (lat.d,) + shape)
    w = lat.w.reshape((lat.Q,) + (1,) * lat.d)
    E = lat.e.astype(float)
    feq = w * chi[None] * (1 + (1 / lat.cs2) * np.tensordot(E, u, axes=(1, 0)))
    tau = rng.uniform(0.6, 2.0, shape)
    post = model.mrt_collide(lat, f, feq, model.scalar_relaxation(lat, tau))
    assert np.allclose(post.sum(0), chi, atol=1e-15)
    j = np.tensordot(E.T, f, axes=(1, 0))
    jeq = np.tensordot(E.T, feq, axes=(1, 0))
    norm = float(np.sum(E[:, 0] ** 2))
    closed = feq + (1 - 1 / tau)[None] * np.tensordot(E, j - jeq, axes=(1, 0)) / norm
    assert np.allclose(post, closed, atol=1e-15)


def test_flow_collision_conserves_mass_and_momentum():
    """K2: with F_b = 0 the flow collision leaves rho and j unchanged."""
    rng = np.random.default_rng(4)
    lat = LT.D2Q9
    d = _dom(nx=4, ny=3, has_flow=True)
    dom = oracle.Domain(d)
    f = _random_state(dom.shape, 9, rng)
    rho = f.sum(0)
    E = lat.e.astype(float)
    j = np.tensordot(E.T, f, axes=(1, 0))
    feq = dom.flow_eq(rho, j / rho, 1.0)
    post = model.mrt_collide(lat, f, feq, dom.flow_relaxation())
    assert np.allclose(post.sum(0), rho, atol=1e-15)
    assert np.allclose(np.tensordot(E.T, post, axes=(1, 0)), j, atol=1e-15)


def test_injection_changes_zeroth_moment_only():
    """K9 / Eq. (39): the transfer adds w_i dU; the flux moment is unchanged
    and the zeroth moment moves by exactly the macroscopic increment."""
    wl = L.reduced(L.solutal_512(), 40, 36)
    dom = oracle.Domain(wl["domains"][0])
    for _ in range(8):
        dom.step()
    chi0, j0 = dom.moments("U")
    U0 = dom.U.copy()
    phi_q, phi_new = dom.phase_step()
    dom.transfer(phi_q, phi_new)
    chi1, j1 = dom.moments("U")
    assert np.allclose(j1, j0, atol=1e-15)
    assert np.allclose(chi1 - chi0, dom.U - U0, atol=1e-15)
    assert np.max(np.abs(dom.U - U0)) > 1e-6


# --------------------------------------------------------------------- K4
@pytest.mark.parametrize("N_U,dt_base,adv", [(1, 1.0, False), (4, 0.25, False), (2, 0.5, True)])
def test_gaussian_diffusion_closed_form(N_U, dt_base, adv):
    """K4: with phi = -1 everywhere (no interface) the U lattice solves
    dU/dt + u.grad U = D_L lap U, whose Gaussian solution is
    U0 + A s0^2/(s0^2 + 2Dt) exp(-|x - x0 - u t|^2 / (2 (s0^2 + 2Dt))).
    Exercises Eq. (19), (23)-(25) and the dt_U = N_U dt_base scaling."""
    n = 96
    D = 0.1
    d = _dom(nx=n, ny=n, has_U=True, N_U=N_U, dt_base=dt_base, k=0.15, D_L=D, D_S=D,
             bc=("periodic",) * 3, U0=0.0)
    dom = oracle.Domain(d)
    u = np.array([0.02, -0.01]) if adv else np.zeros(2)
    dom.u = np.zeros((2,) + dom.shape) + u.reshape(2, 1, 1)
    X, Y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    s0, A, x0 = 6.0, 0.5, 47.0
    U = A * np.exp(-((X - x0) ** 2 + (Y - x0) ** 2) / (2 * s0 ** 2))
    dtU = N_U * dt_base
    dom.U = U
    dom.f_U = dom.scalar_eq(U, dtU)
    n_upd = 60
    for _ in range(n_upd):
        dom.scalar_step("U")
    t = n_upd * dtU
    s2 = s0 ** 2 + 2 * D * t
    xc, yc = x0 + u[0] * t, x0 + u[1] * t
    ref = A * s0 ** 2 / s2 * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2 * s2))
    err = np.linalg.norm(dom.U - ref) / np.linalg.norm(ref)
    assert err < 5e-3, err
    # the same run with the base step in place of dt_U misses badly
    wrong = A * s0 ** 2 / (s0 ** 2 + 2 * D * n_upd * dt_base) * np.exp(
        -((X - x0 - u[0] * n_upd * dt_base) ** 2 + (Y - x0 - u[1] * n_upd * dt_base) ** 2)
        / (2 * (s0 ** 2 + 2 * D * n_upd * dt_base)))
    if N_U > 1:
        assert np.linalg.norm(dom.U - wrong) / np.linalg.norm(ref) > 10 * err


# --------------------------------------------------------------------- K5
def test_poiseuille_flow():
    """K5: body-force-driven channel between half-way bounce-back walls:
    u_x(y) = F/(2 nu) (y + 1/2)(H - 1/2 - y).  Pins Eq. (27)-(33) and Guo
    forcing (Eq. 30) with f_L = 1 everywhere."""
    H = 12
    nu = 0.1
    F = 1e-5
    d = _dom(nx=3, ny=H, has_flow=True, nu=nu, Fb=(F, 0.0, 0.0),
             flow_bc=("periodic", "wall", "periodic"), bc=("periodic", "wall", "periodic"))
    dom = oracle.Domain(d)
    for _ in range(4000):
        dom.flow_step()
    y = np.arange(H, dtype=float)
    ref = F / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    got = dom.u[0][:, 1]
    err = np.max(np.abs(got - ref)) / np.max(ref)
    assert err < 2e-2, err
    assert np.max(np.abs(dom.u[1])) < 1e-12


# --------------------------------------------------------------------- K6
def test_partial_bounce_back_conserves_mass():
    """K6: Eq. (33) only moves mass between links, so sum rho is invariant
    for any liquid-fraction field on a periodic box."""
    rng = np.random.default_rng(6)
    d = _dom(nx=9, ny=7, has_flow=True, flow_bc=("periodic",) * 3, bc=("periodic",) * 3)
    dom = oracle.Domain(d)
    dom.f_F = rng.uniform(0.05, 0.2, (9,) + dom.shape)
    dom.phi = rng.uniform(-1, 1, dom.shape)
    m0 = dom.f_F.sum()
    for _ in range(5):
        dom.flow_step()
    assert abs(dom.f_F.sum() - m0) / m0 < 1e-14


# --------------------------------------------------------------------- K7
def test_transfer_conserves_solute_exactly():
    """K7: the transfer changes C = C_inf kfac(phi)[1 + (1-k)U]/2 by
    -C_inf (1-k) div J, whose sum vanishes on a closed box (mirrored normal
    component at walls) and on a periodic box."""
    for bc in (("wall",) * 3, ("periodic",) * 3):
        wl = L.reduced(L.solutal_512(), 48, 40)
        d = dict(wl["domains"][0], bc=bc)
        dom = oracle.Domain(d)
        for _ in range(12):
            dom.step()
        C0 = P.concentration(d, dom.phi, dom.U)
        phi_q, phi_new = dom.phase_step()
        dom.transfer(phi_q, phi_new)
        C1 = P.concentration(d, dom.phi, dom.U)
        assert abs(C1.sum() - C0.sum()) / C0.sum() < 1e-14
        assert np.max(np.abs(C1 - C0)) > 1e-6


def _planar_transfer_error(W0, n=256):
    k, U0 = 0.15, -0.3
    d = _dom(nx=n, ny=4, has_U=True, W0=W0, k=k, U0=U0, D_L=0.1, D_S=0.001,
             bc=("wall", "periodic", "periodic"))
    dom = oracle.Domain(d)
    x = np.arange(n, dtype=float)
    s = math.sqrt(2) * W0
    x0, dx0 = n / 2 + 0.3, 0.05
    phi_q = np.tanh((x0 - x) / s)[None].repeat(4, 0)
    phi_n = np.tanh((x0 + dx0 - x) / s)[None].repeat(4, 0)
    dom.U = np.full(dom.shape, U0)
    dom.transfer(phi_q, phi_n)
    dU = dom.U - U0
    coef = 1 + (1 - k) * U0
    dphi = phi_n - phi_q
    sech2 = lambda z: 1 / np.cosh(z) ** 2  # noqa: E731
    ddphi = (-sech2((x0 + dx0 - x) / s) + sech2((x0 - x) / s)) / s   # exact d/dx of dphi
    dJ = W0 / (2 * math.sqrt(2)) * coef * ddphi[None]
    ref = (coef * dphi - 2 * dJ) / ((1 + k) - (1 - k) * phi_n)
    no_div = coef * dphi / ((1 + k) - (1 - k) * phi_n)
    scale = np.max(np.abs(ref))
    return np.max(np.abs(dU - ref)) / scale, np.max(np.abs(no_div - ref)) / scale


def test_transfer_matches_analytic_planar_front():
    """Eq. (36)-(38) against exact derivatives: a planar front
    phi = tanh((x0 - x)/(sqrt2 W0)) advanced by a small shift with uniform U.
    Expected dU = ([1 + (1-k)U] dphi - 2 d/dx J_x) / kfac(phi_new) with
    J_x = W0/(2 sqrt2) [1 + (1-k)U] dphi n_x and n_x = +1 (towards the
    liquid), differentiated analytically.  The compact stencil converges at
    second order in dx/W0, and the anti-trapping term is ~70 % of dU."""
    e4, d4 = _planar_transfer_error(4.0)
    e8, d8 = _planar_transfer_error(8.0)
    assert e8 < 5e-3, e8
    assert e4 / e8 > 3.5, (e4, e8)
    assert d8 > 50 * e8


# --------------------------------------------------------------------- K8
@pytest.mark.parametrize("bc", ["periodic", "wall"])
def test_enthalpy_invariant_constant_properties(bc):
    """K8: with constant properties, sum(T - rho_L L_h phi/(2 rhoCp)) is
    invariant through the coupled phase + transfer + T-transport run."""
    wl = L.reduced(L.thermal_128(), 48, 48)
    d = dict(wl["domains"][0], bc=(bc,) * 3)
    dom = oracle.Domain(d)
    h0 = oracle.diag.totals(dom)["enthalpy"]
    s0 = oracle.diag.totals(dom)["solid"]
    for _ in range(60):
        dom.step()
    t = oracle.diag.totals(dom)
    assert abs(t["enthalpy"] - h0) / abs(h0) < 1e-13
    assert t["solid"] > s0 + 1.0  # the seed grows


# --------------------------------------------------------------------- K10
@pytest.mark.parametrize("name", ["thermal", "solutal"])
def test_fourfold_symmetry_of_centred_seed(name):
    """K10: a seed centred on a symmetry point of the grid keeps the D4
    symmetry: phi(x, y) = phi(y, x) = phi(-x, y)."""
    if name == "thermal":
        d = L.reduced(L.thermal_128(), 64, 64)["domains"][0]
        d["seeds"] = [(32.0, 32.0, 5.0)]
        phi_sym = lambda p: (p[1:, 1:], p[1:, 1:].T, p[1:, 1:][:, ::-1])  # noqa: E731
    else:
        d = L.reduced(L.solutal_512(), 48, 48)["domains"][0]
        phi_sym = lambda p: (p, p.T, p[:, ::-1])  # noqa: E731
    dom = oracle.Domain(d)
    for _ in range(60):
        dom.step()
    a, b, c = phi_sym(dom.phi)
    assert np.max(np.abs(a - b)) < 1e-12
    assert np.max(np.abs(a - c)) < 1e-12
    if name == "solutal":
        a, b, c = phi_sym(dom.U)
        assert np.max(np.abs(a - b)) < 1e-12 and np.max(np.abs(a - c)) < 1e-12


# --------------------------------------------------------------------- K11
def test_uniform_states_are_fixed_points():
    """K11: uniform liquid or solid with uniform U, T and a uniform flow at
    rest stays exactly where it is."""
    for phi0 in (-1.0, 1.0):
        d = _dom(nx=12, ny=10, has_U=True, has_T=True, has_flow=True, k=0.15, D_L=0.1, D_S=0.01,
                 kappa_S=0.2, kappa_L=0.1, rhoCp_S=1.3, rhoCp_L=1.0, lam=2.0, Mc=0.5,
                 W0=2.0, tau0=10.0, eps_s=0.05, U0=-0.2, T0=-0.3,
                 bc=("wall", "periodic", "wall"), flow_bc=("periodic", "wall", "wall"))
        dom = oracle.Domain(d)
        dom.phi[:] = phi0
        dom.f_phi = dom.ls.w[:, None, None] * dom.phi[None]
        for _ in range(5):
            dom.step()
        assert np.allclose(dom.phi, phi0, atol=1e-15, rtol=0)
        assert np.allclose(dom.U, -0.2, atol=1e-15, rtol=0)
        assert np.allclose(dom.T, -0.3, atol=1e-15, rtol=0)
        assert np.allclose(dom.u, 0.0, atol=1e-15)


def test_no_anisotropy_reduces_to_standard_streaming():
    """K11: eps_s = 0 gives a_s = 1, so Eq. (26) is standard streaming."""
    d = L.reduced(L.thermal_128(), 32, 32)["domains"][0]
    d["eps_s"] = 0.0
    dom = oracle.Domain(d)
    for _ in range(3):
        dom.step()
    g = grad_iso(dom.phi, dom.bc)
    a_s, N, _ = model.anisotropy(d, g)
    assert np.all(a_s == 1.0) and np.all(N == 0.0)


def test_planar_front_is_stationary():
    """K11: with U = theta = 0 the front tanh(x/(sqrt2 W0 a_s)) solves
    W0^2 a_s^2 phi'' + phi (1 - phi^2) = 0 (N is tangential to a planar
    front, so div N = 0); it stays put up to O(dx^2/W^2)."""
    n = 96
    W0, eps = 4.0, 0.03
    d = _dom(nx=n, ny=3, W0=W0, tau0=60.0, eps_s=eps, lam=3.0, bc=("wall", "periodic", "periodic"))
    dom = oracle.Domain(d)
    a_s = 1 + eps  # normal along x
    x = np.arange(n, dtype=float)
    phi0 = np.tanh((47.3 - x) / (math.sqrt(2) * W0 * a_s))[None].repeat(3, 0)
    dom.phi = phi0.copy()
    dom.f_phi = dom.ls.w[:, None, None] * phi0[None]
    for _ in range(300):
        dom.step()
    drift = np.max(np.abs(dom.phi - phi0))
    assert drift < 2e-3, drift
    # a front with the wrong width (no a_s) is not stationary at this level
    dom2 = oracle.Domain(d)
    wrong = np.tanh((47.3 - x) / (math.sqrt(2) * W0 * 0.7))[None].repeat(3, 0)
    dom2.phi = wrong.copy()
    dom2.f_phi = dom2.ls.w[:, None, None] * wrong[None]
    for _ in range(300):
        dom2.step()
    assert np.max(np.abs(dom2.phi - wrong)) > 10 * drift


# --------------------------------------------------------------------- K12
def test_printed_parameter_values():
    """K12: every relaxation time, coupling constant and Table 1 lattice value
    the paper prints is reproduced by the parameter algebra."""
    g = json.load(open(GOLDEN))
    e = g["lambda_thermosolutal"]
    assert math.isclose(P.lambda_coupling(e["a1"], 1.0, e["d0_over_W0"]), e["value"], rel_tol=e["rtol"])
    e = g["tau_F_forced_thermal"]
    d = _dom(nu=e["nu"], dt_base=e["dt_base"], N_F=e["N_F"])
    assert math.isclose(P.tau_F(d), e["value"], rel_tol=e["rtol"])
    e = g["tau_U_thermosolutal"]
    d = _dom(N_U=e["N_U"], D_L=e["D_L"], D_S=e["D_S"], k=e["k"])
    assert abs(P.tau_U(d, 1.0) - e["solid"]) < e["atol"]
    assert abs(P.tau_U(d, -1.0) - e["liquid"]) < e["atol"]
    e = g["tau_T_thermosolutal"]
    d = _dom(N_T=e["N_T"], kappa_S=e["alpha"], kappa_L=e["alpha"])
    assert math.isclose(P.tau_T(d, 0.3), e["value"], rel_tol=e["rtol"])
    e = g["tau_U_liquid_lewis"]
    for Le in e["Le"]:
        d = _dom(N_U=Le, D_L=e["D_L_lattice_Le100"] * 100 / Le, D_S=0.0, k=0.001)
        assert abs(P.tau_U(d, -1.0) - e["value"]) < e["atol"]
    t = g["table1"]
    lat = P.lattice_from_physical(P.table1_physical(), t["dx"], t["dt"], t["dm"], t["dT"])
    for key, val in t["lattice"].items():
        assert math.isclose(lat[key], val, rel_tol=t["rtol"]), (key, lat[key], val)
    assert math.isclose(lat["d0"] * t["dx"], t["d0_physical_m"], rel_tol=t["rtol"])
    assert math.isclose(lat["rho"], 1.0, rel_tol=1e-12)
    e = g["ablation_blowup"]
    assert round(e["t_ms"] * 1e-3 / e["dt_base_s"]) == e["base_steps"]


def test_workload_parameters_follow_the_paper_definitions():
    """The synthetic workloads use Table 1 / Eq. (5) consistently: the
    ensemble's T0 maps to theta0 = -Delta, its tau_U,L = 0.578, and the 3D
    set's lambda and Mc are the Table 1 definitions at k = 0.01."""
    wl = L.ensemble_256(n_domains=8)
    for d in wl["domains"]:
        assert math.isclose(P.theta_of_T(d, d["T0"]), -d["Delta"], rel_tol=1e-12)
        assert abs(P.tau_U(d, -1.0) - 0.578) < 1e-12
        assert abs(P.tau_T(d, -1.0) - 0.578) < 5e-4
    d3 = L.directional_3d(nx=8, ny=8, nz=8)["domains"][0]
    phys = P.table1_physical()
    d0 = P.capillary_length(0.268, phys["m_L"], 0.01, phys["C_inf"])
    assert math.isclose(d3["lam"], P.lambda_coupling(0.8839, 2.0, d0), rel_tol=1e-6)
    assert math.isclose(d3["Mc"], P.solutal_coupling(-57.0, 0.01, 0.03, 133.6, 1.676), rel_tol=1e-5)
    # every workload keeps every relaxation time above 1/2
    for name in L.WORKLOADS:
        kw = dict(n_domains=4) if name == "ensemble_256" else {}
        if name == "directional_3d":
            kw = dict(nx=8, ny=8, nz=8)
        for d in L.workload(name, **kw)["domains"]:
            for f, tau in P.min_tau(d).items():
                assert tau > 0.5, (name, f, tau)


# --------------------------------------------------------------------- K13
@pytest.mark.parametrize("dim,theta", [(2, 0.0), (2, 0.37), (3, 0.0)])
def test_anisotropy_vector_equals_numerical_derivative(dim, theta):
    """K13: N = |g|^2 a_s d a_s/d g (Eq. 3) in closed form equals a central
    difference of a_s(n(g)) (Eq. 2) with respect to g."""
    rng = np.random.default_rng(13)
    d = dict(eps_s=0.05, theta_c=theta)
    g = rng.normal(size=(dim, 50)) * rng.uniform(0.01, 2.0, 50)
    a_s, N, _ = model.anisotropy(d, g)
    h = 1e-6
    Nn = np.zeros_like(g)
    for a in range(dim):
        gp, gm = g.copy(), g.copy()
        gp[a] += h
        gm[a] -= h
        da = (model.anisotropy(d, gp)[0] - model.anisotropy(d, gm)[0]) / (2 * h)
        Nn[a] = np.sum(g * g, axis=0) * a_s * da
    assert np.allclose(N, Nn, rtol=1e-6, atol=1e-9)
    # and a_s follows Eq. (2) in the crystal frame (range 1 +- eps in 2D)
    if dim == 2:
        assert np.all(a_s <= 1.05 + 1e-12) and np.all(a_s >= 0.95 - 1e-12)


# --------------------------------------------------------------------- K14
def test_schedule_counts():
    """K14 / Eq. (34): over K base steps field chi is updated floor(K/N_chi)
    times, in the order phi, U, T, flow."""
    d = _dom(nx=6, ny=5, has_U=True, has_T=True, has_flow=True, N_phi=1, N_U=4, N_T=3, N_F=2,
             D_L=0.1, D_S=0.1, kappa_S=0.1, kappa_L=0.1, k=0.5)
    dom = oracle.Domain(d)
    log = []
    dom.phase_step = lambda: (log.append("phi"), (dom.phi, dom.phi))[1]
    dom.transfer = lambda a, b: log.append("pc")
    dom.scalar_step = lambda w: log.append(w)
    dom.flow_step = lambda: log.append("F")
    K = 60
    for _ in range(K):
        dom.step()
    assert log.count("phi") == K and log.count("pc") == K
    assert log.count("U") == K // 4 and log.count("T") == K // 3 and log.count("F") == K // 2
    # at k = 12 all four run, phase first
    i12 = [i for i, x in enumerate(log) if x == "phi"][11]
    assert log[i12:i12 + 5] == ["phi", "pc", "U", "T", "F"]


# --------------------------------------------------------------------- continuum consistency
def _spectral(n):
    k = 2 * np.pi * np.fft.fftfreq(n)
    KX, KY = np.meshgrid(k, k)
    dx = lambda a: np.real(np.fft.ifft2(1j * KX * np.fft.fft2(a)))  # noqa: E731
    dy = lambda a: np.real(np.fft.ifft2(1j * KY * np.fft.fft2(a)))  # noqa: E731
    return dx, dy


def _rk4(f, y, dt, n):
    for _ in range(n):
        k1 = f(y)
        k2 = f(y + dt / 2 * k1)
        k3 = f(y + dt / 2 * k2)
        k4 = f(y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def test_phase_lattice_recovers_eq1():
    """The phase lattice (Eq. 14, 21-24, 26 with the tau0-scaled source)
    recovers Eq. (1): a_s^2 tau0 dphi/dt = W0^2 div(a_s^2 grad phi)
    + W0^2 div N + Q_phi, compared with a spectral RK4 solution on a smooth
    periodic field.  Flipping the sign of N changes the answer by ~20 %,
    ten times the tolerance."""
    n = 64
    d = _dom(nx=n, ny=n, W0=4.0, tau0=96.0, eps_s=0.05, lam=0.0, bc=("periodic",) * 3)
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    phi0 = (0.3 * np.sin(2 * np.pi * X / n) * np.cos(2 * np.pi * Y / n) + 0.2 * np.sin(4 * np.pi * Y / n)
            + 0.1 * np.cos(2 * np.pi * (X + Y) / n))
    dx, dy = _spectral(n)

    def rhs(phi):
        gx, gy = dx(phi), dy(phi)
        a_s, N, _ = model.anisotropy(d, np.stack([gx, gy]))
        A = a_s ** 2
        W2, t0 = d["W0"] ** 2, d["tau0"]
        return (W2 / t0 * (dx(A * gx) + dy(A * gy) + dx(N[0]) + dy(N[1])) + phi * (1 - phi ** 2) / t0) / A

    dom = oracle.Domain(d)
    dom.phi = phi0.copy()
    dom.f_phi = dom.ls.w[:, None, None] * phi0[None]
    S = 40
    for _ in range(S):
        dom.step()
    ref = _rk4(rhs, phi0, 0.25, 4 * S)
    err = np.linalg.norm((dom.phi - phi0) - (ref - phi0)) / np.linalg.norm(ref - phi0)
    assert err < 0.03, err


def test_concentration_lattice_recovers_conservative_form():
    """Eq. (6)-(8) transport part: with Q_U^tr = -(1-k) D_eff grad U . grad
    phi / kfac, the U lattice recovers dU/dt = div(q grad U)/kfac with
    q = kfac D_eff = (1+phi) D_S + (1-phi) D_L (the conservative form of the
    solute flux).  Static smooth phi, spectral RK4 reference."""
    n = 64
    d = _dom(nx=n, ny=n, has_U=True, k=0.15, D_L=0.15, D_S=0.0015, N_U=2, dt_base=0.5,
             bc=("periodic",) * 3)
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    phi = 0.8 * np.sin(2 * np.pi * X / n) * np.cos(2 * np.pi * Y / n)
    U0 = 0.3 * np.cos(2 * np.pi * X / n + 0.4) + 0.2 * np.sin(4 * np.pi * Y / n)
    dx, dy = _spectral(n)
    k = d["k"]
    kf = (1 + k) - (1 - k) * phi
    q = (1 + phi) * d["D_S"] + (1 - phi) * d["D_L"]
    rhs = lambda U: (dx(q * dx(U)) + dy(q * dy(U))) / kf  # noqa: E731
    dom = oracle.Domain(d)
    dom.phi = phi
    dom.U = U0.copy()
    dom.f_U = dom.scalar_eq(U0, 1.0)
    S = 40
    for _ in range(S):
        dom.scalar_step("U")
    ref = _rk4(rhs, U0, 0.25, 4 * S)
    err = np.linalg.norm((dom.U - U0) - (ref - U0)) / np.linalg.norm(ref - U0)
    assert err < 0.03, err
    # without the transport source the lattice would solve div(D_eff grad U)
    rhs2 = lambda U: dx(q / kf * dx(U)) + dy(q / kf * dy(U))  # noqa: E731
    ref2 = _rk4(rhs2, U0, 0.25, 4 * S)
    assert np.linalg.norm(ref2 - ref) / np.linalg.norm(ref - U0) > 5 * err


def test_temperature_lattice_recovers_conductive_form():
    """Eq. (10)-(12) transport part: the first term of Q_T makes the thermal
    operator div(kappa_eff grad T)/(rho Cp)_eff (Section 2.3).  Static smooth
    phi with strong property contrast, spectral RK4 reference."""
    n = 64
    d = _dom(nx=n, ny=n, has_T=True, kappa_S=0.3, kappa_L=0.08, rhoCp_S=0.6, rhoCp_L=1.4,
             bc=("periodic",) * 3)
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    phi = 0.8 * np.cos(2 * np.pi * X / n) * np.cos(2 * np.pi * Y / n)
    T0 = 0.5 * np.sin(2 * np.pi * X / n) + 0.3 * np.cos(2 * np.pi * (X - Y) / n)
    dx, dy = _spectral(n)
    kap = (1 + phi) / 2 * d["kappa_S"] + (1 - phi) / 2 * d["kappa_L"]
    rc = (1 + phi) / 2 * d["rhoCp_S"] + (1 - phi) / 2 * d["rhoCp_L"]
    rhs = lambda T: (dx(kap * dx(T)) + dy(kap * dy(T))) / rc  # noqa: E731
    dom = oracle.Domain(d)
    dom.phi = phi
    dom.T = T0.copy()
    dom.f_T = dom.scalar_eq(T0, 1.0)
    S = 40
    for _ in range(S):
        dom.scalar_step("T")
    ref = _rk4(rhs, T0, 0.25, 4 * S)
    err = np.linalg.norm((dom.T - T0) - (ref - T0)) / np.linalg.norm(ref - T0)
    assert err < 0.03, err
    alpha = kap / rc
    rhs2 = lambda T: dx(alpha * dx(T)) + dy(alpha * dy(T))  # noqa: E731
    ref2 = _rk4(rhs2, T0, 0.25, 4 * S)
    assert np.linalg.norm(ref2 - ref) / np.linalg.norm(ref - T0) > 5 * err


# --------------------------------------------------------------------- stencils
def test_isotropic_stencils_exact_on_quadratics():
    """The isotropic gradient and divergence are exact for quadratic fields
    in the interior and the divergence telescopes to zero with mirrored
    ghosts (the discrete form of the closed-box solute identity)."""
    n = 12
    X, Y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    f = 0.3 * X * X - 0.2 * X * Y + 0.1 * Y * Y + X - 2 * Y
    g = grad_iso(f, ("wall", "wall"))
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(g[0][inner], (0.6 * X - 0.2 * Y + 1)[inner])
    assert np.allclose(g[1][inner], (-0.2 * X + 0.2 * Y - 2)[inner])
    J = np.stack([X * Y, X - Y * Y])
    dv = div_iso(J, ("wall", "wall"))
    assert np.allclose(dv[inner], (Y - 2 * Y)[inner])
    rng = np.random.default_rng(0)
    J = rng.normal(size=(2, 9, 11))
    for bc in (("wall", "wall"), ("periodic", "wall"), ("periodic", "periodic")):
        assert abs(div_iso(J, bc).sum()) < 1e-12


# --------------------------------------------------------------------- diagnostics
def test_tip_position_of_a_circle():
    """Tip reading: a tanh circle of radius R centred off the lattice has
    its phi = 0 crossing at distance R along every axis (to the accuracy of
    linear interpolation over one spacing)."""
    d = _dom(nx=80, ny=70, W0=2.0, seeds=[(37.3, 33.6, 17.4)], theta_c=0.2)
    dom = oracle.Domain(d)
    t = oracle.diag.tips(dom)
    assert np.allclose(t, 17.4, atol=2e-2)


# --------------------------------------------------------------------- brute force
@pytest.mark.parametrize("case", ["walls", "mixed", "periodic_q9", "flow"])
def test_tiny_grid_brute_force(case):
    """The vectorised oracle equals a per-site loop implementation (closed
    form collisions, explicit neighbour indexing) for full base steps on
    7x6 grids with every boundary combination, including corners and the
    inlet/outflow columns."""
    from tests import brute

    d = _dom(nx=7, ny=6, has_U=True, has_T=True, W0=1.3, tau0=4.0, eps_s=0.05, lam=2.0,
             Mc=0.4, k=0.2, D_L=0.2, D_S=0.01, kappa_S=0.3, kappa_L=0.15, rhoCp_S=1.2,
             rhoCp_L=0.9, L_h=1.3, U0=-0.3, T0=-0.4, theta_c=0.3, N_U=2, N_T=1, N_F=1,
             seeds=[(2.6, 3.1, 2.2)])
    if case == "walls":
        d["bc"] = ("wall", "wall", "wall")
    elif case == "mixed":
        d["bc"] = ("periodic", "wall", "wall")
    elif case == "periodic_q9":
        d["bc"] = ("periodic", "periodic", "periodic")
        d["q_scalar"] = 9
    else:
        d.update(has_flow=True, bc=("wall", "wall", "wall"), u_in=0.02, u0_liquid_only=True,
                 flow_bc=("inlet_outflow", "periodic", "periodic"), nu=0.12, Fb=(1e-4, -2e-4, 0.0))
    dom = oracle.Domain(d)
    for _ in range(4):
        ref = brute.step(dom)
        dom.step()
        for key, val in ref.items():
            got = getattr(dom, key)
            assert np.allclose(got, val, atol=1e-14, rtol=0), (case, dom.k, key, np.max(np.abs(got - val)))


# --------------------------------------------------------------------- stability margin of Eq. (26)
def test_anisotropic_streaming_needs_a_relaxation_margin():
    """Eq. (26) divides the streamed populations by A = a_s^2 and subtracts
    (1 - A) f: for A < 1 a checkerboard mode that the collision flips with
    factor (1 - 1/tau_phi) grows unless |1 - 1/tau_phi| + (1 - A) <= A, i.e.
    tau_phi >= 1/(2A) roughly 0.52 at eps = 0.02.  A circle with pure
    Allen-Cahn dynamics (lambda = 0) stays within [-1, 1] at tau0 = 100
    (tau_phi ~ 0.62) and overshoots at tau0 = 1000 (tau_phi ~ 0.512, the
    Section 4.3 scale, where the thermosolutal case diverges)."""
    def run(tau0):
        d = _dom(nx=64, ny=64, W0=2.0, tau0=tau0, eps_s=0.02, lam=0.0, theta_c=0.5,
                 bc=("periodic",) * 3, seeds=[(31.5, 31.5, 14.0)])
        dom = oracle.Domain(d)
        peak = 0.0
        for _ in range(300):
            dom.step()
            peak = max(peak, float(np.max(np.abs(dom.phi))))
        return peak

    assert run(100.0) <= 1.0 + 1e-6
    assert run(1000.0) > 1.05


# --------------------------------------------------------------------- cold bottom (Section 4.4)
def test_cold_bottom_follows_the_erf_solution():
    """T held at T_b on the low wall y = -1/2 by anti-bounce-back, zero flux
    elsewhere, uniform T_i at t = 0 and no interface: the half-space
    solution T_b + (T_i - T_b) erf((y + 1/2) / (2 sqrt(alpha t))).  A wall at
    y = 0 instead of -1/2, or no Dirichlet wall at all, misses by far."""
    from scipy.special import erf

    alpha, n_steps, Tb = 0.1, 250, -1.0
    d = _dom(nx=3, ny=80, has_T=True, N_T=1, kappa_S=alpha, kappa_L=alpha, rhoCp_S=1.0, rhoCp_L=1.0,
             T0=Tb, bc=("periodic", "wall", "wall"), T_mode="dirichlet_low", L_h=1.0, Cp_L=1.0)
    dom = oracle.Domain(d)
    dom.T = np.zeros(dom.shape)
    dom.f_T = dom.scalar_eq(dom.T, 1.0)
    for _ in range(n_steps):
        dom.k += 1
        dom.scalar_step("T")
    y = np.arange(80, dtype=float)
    s = 2 * math.sqrt(alpha * n_steps)
    ref = Tb - Tb * erf((y + 0.5) / s)
    err = np.max(np.abs(dom.T[:, 1] - ref))
    assert err < 1e-3, err
    assert np.max(np.abs(Tb - Tb * erf(y / s) - ref)) > 20 * err


def test_eq41_front_initial_condition():
    """Eq. (41): phi(x, 0) = tanh[(10 + sin(10 pi x / L) - y)/(sqrt2 W0)],
    mean height 10, amplitude 1, wavelength L/5; T = T_b = -20, U = 0."""
    wl = L.directional_2d(Le=10, nx=100, ny=40)
    d = wl["domains"][0]
    dom = oracle.Domain(d)
    X, Y = np.meshgrid(np.arange(100.0), np.arange(40.0))
    ref = np.tanh((10 + np.sin(10 * math.pi * X / 100) - Y) / (math.sqrt(2) * d["W0"]))
    assert np.allclose(dom.phi, ref, atol=1e-15)
    assert np.all(dom.T == -20.0) and np.all(dom.U == 0.0)
    # the liquid concentration relaxation time is the printed 0.578 for every Le (Eq. 42)
    for Le in (1, 10, 100, 1000):
        dd = L.directional_2d(Le=Le, nx=8, ny=8)["domains"][0]
        assert abs(P.tau_U(dd, -1.0) - 0.578) < 1e-12
