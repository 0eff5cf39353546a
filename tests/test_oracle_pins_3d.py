"""Pins of the 3D oracle (D3Q7 scalars, D3Q19 flow, pulled temperature).

The 3D directional case extends the paper's 2D construction (Sections 2-3)
to cubic lattices.  As for the 2D pins, nothing here compares the oracle
with itself: closed forms, invariants, symmetries and exact solutions.
"""

import numpy as np
import pytest

import lbm_inputs as L
import oracle
from oracle import lattice as LT
from oracle import model
from oracle import params as P


def _dom3(**kw):
    d = L.configs._base_domain()
    d.update(dim=3, q_scalar=7, nz=kw.pop("nz", 8))
    d.update(kw)
    return d


def _stress(lat, f):
    E = lat.e.astype(float)
    return np.einsum("ia,ib,i...->ab...", E, E, f)


# ------------------------------------------------------------------ flow
def test_d3q19_collision_relaxes_each_moment_at_its_rate():
    """Eq. (14) on D3Q19 with F_b = 0: rho and j are conserved, the traceless
    stress of f - f^eq relaxes by (1 - s_nu), its trace part (energy) by
    (1 - s_e), each per collision (the 3D counterpart of Eq. 31)."""
    rng = np.random.default_rng(31)
    d = _dom3(nx=3, ny=2, nz=2, has_flow=True, nu=0.07, s_e=1.3)
    dom = oracle.Domain(d)
    lat = LT.D3Q19
    f = rng.uniform(0.02, 0.08, (19,) + dom.shape)
    rho = f.sum(0)
    E = lat.e.astype(float)
    j = np.tensordot(E.T, f, axes=(1, 0))
    feq = dom.flow_eq(rho, j / rho, 1.0)
    post = model.mrt_collide(lat, f, feq, dom.flow_relaxation())
    assert np.allclose(post.sum(0), rho, atol=1e-15)
    assert np.allclose(np.tensordot(E.T, post, axes=(1, 0)), j, atol=1e-15)
    S0 = _stress(lat, f - feq)
    S1 = _stress(lat, post - feq)
    tr0 = np.trace(S0)
    tr1 = np.trace(S1)
    dev0 = S0 - np.eye(3)[:, :, None, None, None] * tr0 / 3
    dev1 = S1 - np.eye(3)[:, :, None, None, None] * tr1 / 3
    snu = 1.0 / P.tau_F(d)
    assert np.allclose(dev1, (1 - snu) * dev0, atol=1e-15)
    assert np.allclose(tr1, (1 - d["s_e"]) * tr0, atol=1e-15)


def test_d3q19_poiseuille_between_z_walls():
    """Body-force channel between half-way bounce-back walls normal to z:
    u_x(z) = F/(2 nu) (z + 1/2)(H - 1/2 - z), u_y = u_z = 0 (Eq. 27-33 on
    D3Q19 with Guo forcing)."""
    H, nu, F = 12, 0.1, 1e-5
    d = _dom3(nx=3, ny=3, nz=H, has_flow=True, nu=nu, Fb=(F, 0.0, 0.0),
              flow_bc=("periodic", "periodic", "wall"), bc=("periodic", "periodic", "wall"))
    dom = oracle.Domain(d)
    for _ in range(4000):
        dom.flow_step()
    z = np.arange(H, dtype=float)
    ref = F / (2 * nu) * (z + 0.5) * (H - 0.5 - z)
    got = dom.u[0][:, 1, 1]
    assert np.max(np.abs(got - ref)) / np.max(ref) < 2e-2
    assert np.max(np.abs(dom.u[1:])) < 1e-12
    # the same force along y between the same walls gives the same profile in u_y
    d2 = dict(d, Fb=(0.0, F, 0.0))
    dom2 = oracle.Domain(d2)
    for _ in range(4000):
        dom2.flow_step()
    assert np.allclose(dom2.u[1], dom.u[0], atol=1e-15)


def test_d3q19_partial_bounce_back_conserves_mass():
    """Eq. (33) on D3Q19 moves mass between links only: sum rho is invariant
    for any liquid fraction on a periodic box."""
    rng = np.random.default_rng(33)
    d = _dom3(nx=5, ny=4, nz=3, has_flow=True, flow_bc=("periodic",) * 3, bc=("periodic",) * 3)
    dom = oracle.Domain(d)
    dom.f_F = rng.uniform(0.02, 0.1, (19,) + dom.shape)
    dom.phi = rng.uniform(-1, 1, dom.shape)
    m0 = dom.f_F.sum()
    for _ in range(5):
        dom.flow_step()
    assert abs(dom.f_F.sum() - m0) / m0 < 1e-14


# ------------------------------------------------------------------ scalars
def test_d3q7_gaussian_diffusion_closed_form():
    """phi = -1 (no interface): the D3Q7 U lattice with tau = 4 dt D + 1/2
    (c_s^2 = 1/4) solves dU/dt + u.grad U = D lap U; the Gaussian keeps its
    closed form A (s0^2/s^2)^{3/2} exp(-|x - x0 - u t|^2 / (2 s^2)),
    s^2 = s0^2 + 2 D t."""
    n, D = 32, 0.08
    d = _dom3(nx=n, ny=n, nz=n, has_U=True, N_U=2, dt_base=0.5, k=0.15, D_L=D, D_S=D,
              bc=("periodic",) * 3, U0=0.0)
    dom = oracle.Domain(d)
    u = np.array([0.03, -0.02, 0.01])
    dom.u = np.zeros((3,) + dom.shape) + u.reshape(3, 1, 1, 1)
    Z, Y, X = np.indices(dom.shape, dtype=float)
    s0, A, x0 = 4.0, 0.5, 15.0
    dom.U = A * np.exp(-((X - x0) ** 2 + (Y - x0) ** 2 + (Z - x0) ** 2) / (2 * s0 ** 2))
    dtU = 1.0
    dom.f_U = dom.scalar_eq(dom.U, dtU)
    n_upd = 40
    for _ in range(n_upd):
        dom.scalar_step("U")
    t = n_upd * dtU
    s2 = s0 ** 2 + 2 * D * t
    c = x0 + u * t
    ref = A * (s0 ** 2 / s2) ** 1.5 * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s2))
    err = np.linalg.norm(dom.U - ref) / np.linalg.norm(ref)
    assert err < 1e-2, err
    # the D2Q5 factor 3 in place of 4 would give a diffusivity off by 4/3
    s2w = s0 ** 2 + 2 * D * 0.75 * t
    wrong = A * (s0 ** 2 / s2w) ** 1.5 * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s2w))
    assert np.linalg.norm(dom.U - wrong) / np.linalg.norm(ref) > 3 * err


def _pulled(nz, V, nx=4, ny=3):
    wl = L.reduced(L.directional_3d(), nx, ny, nz)
    d = wl["domains"][0]
    d["perturb"] = np.zeros((ny, nx))
    d["z_front"] = -60.0            # all liquid: the phase field plays no part
    d["V_pull"] = V
    return d


def test_pulled_temperature_static_profile_is_exact():
    """V = 0: the linear profile T0 + G (z - z_front) solves the diffusion
    equation and anti-bounce-back imposes it at z_w = -1/2 and nz - 1/2
    exactly; T stays on it to rounding."""
    d = _pulled(24, 0.0)
    dom = oracle.Domain(d)
    z = dom.coords()[2]
    for _ in range(30):
        dom.k += d["N_T"]
        dom.scalar_step("T")
    ref = dom.pulled_T(z, 0.0)
    assert np.max(np.abs(dom.T - ref)) < 1e-14


def test_pulled_temperature_follows_the_moving_profile():
    """V > 0: T0 + G (z - z_front - V t) is an exact solution of
    T_t + V T_z = alpha T_zz.  In the interior the lattice follows it to
    advection rounding; at the walls the anti-bounce-back condition leaves
    an error far below one cell of gradient (G dz)."""
    d = _pulled(48, 2e-4)
    dom = oracle.Domain(d)
    z = dom.coords()[2]
    for _ in range(100):
        dom.k += d["N_T"]
        dom.scalar_step("T")
    ref = dom.pulled_T(z, dom.k * d["dt_base"])
    err = np.abs(dom.T - ref)[:, 0, 0]
    G = d["T_grad"]
    assert err.max() < 0.01 * G
    assert err[20:28].max() < 2e-4 * G
    # the profile has moved by V t: the static profile is far off at the centre
    static = dom.pulled_T(z, 0.0)[:, 0, 0]
    assert abs(static[24] - dom.T[24, 0, 0]) > 50 * err[20:28].max()
    # columns stay identical (x, y play no part)
    assert np.max(np.abs(dom.T - dom.T[:, :1, :1])) < 1e-15


# ------------------------------------------------------------------ phase + coupling
def test_cubic_symmetry_of_centred_sphere():
    """A sphere centred in a periodic cube with fourfold-cubic anisotropy
    (a_s = 1 - 3 eps + 4 eps sum n_a^4) keeps the symmetry of the cube: phi
    and U are invariant under axis permutations and reflections."""
    n = 17
    d = _dom3(nx=n, ny=n, nz=n, has_U=True, U0=-0.55, k=0.15, eps_s=0.05, lam=3.19, Mc=0.05,
              D_L=1.0, D_S=1e-4, bc=("periodic",) * 3, seeds=[(8.0, 8.0, 8.0, 4.0)])
    dom = oracle.Domain(d)
    for _ in range(12):
        dom.step()
    for f in (dom.phi, dom.U):
        assert np.max(np.abs(f - f.transpose(1, 0, 2))) < 1e-13
        assert np.max(np.abs(f - f.transpose(2, 1, 0))) < 1e-13
        assert np.max(np.abs(f - f.transpose(0, 2, 1))) < 1e-13
        for ax in range(3):
            assert np.max(np.abs(f - np.flip(f, axis=ax))) < 1e-13
    # the interface moved (the test is not vacuous)
    assert np.max(np.abs(dom.phi - oracle.Domain(d).phi)) > 1e-3


def test_anisotropy_values_on_cube_directions():
    """Eq. (2) in 3D: a_s = 1 + eps along <100>, 1 - eps along <110>,
    1 - 5 eps / 3 along <111>; N vanishes on these symmetry directions."""
    eps = 0.04
    g = np.array([[1.0, 1.0, 1.0], [0.0, 1.0, 1.0], [0.0, 0.0, 1.0]])   # columns: <100>, <110>, <111>
    a_s, N, _ = model.anisotropy(dict(eps_s=eps), g)
    assert np.allclose(a_s, [1 + eps, 1 - eps, 1 - 5 * eps / 3], atol=1e-15)
    assert np.allclose(N, 0.0, atol=1e-15)


def test_directional_3d_transfer_conserves_solute_exactly():
    """The transfer (Eq. 36-39) changes C = C_inf kfac(phi)[1 + (1-k)U]/2 by
    -C_inf (1-k) div J on D3Q19 stencils; the compact divergence sums to zero
    on a box with periodic sides and zero-flux z walls (mirrored normal
    component), so one phase step plus transfer keeps sum C to rounding."""
    wl = L.reduced(L.directional_3d(), 12, 10, 24)
    d = wl["domains"][0]
    d["Fb"] = (2e-5, 1e-5, 0.0)
    dom = oracle.Domain(d)
    for _ in range(24):
        dom.step()
    C0 = P.concentration(d, dom.phi, dom.U)
    phi_q, phi_new = dom.phase_step()
    dom.transfer(phi_q, phi_new)
    C1 = P.concentration(d, dom.phi, dom.U)
    assert abs(C1.sum() - C0.sum()) / C0.sum() < 1e-14
    assert np.max(np.abs(C1 - C0)) > 1e-6
    assert np.max(np.abs(dom.u)) > 1e-7                      # the flow is driven


def test_unperturbed_front_stays_laterally_uniform():
    """With xi = 0 the initial state and every update are invariant under
    x, y translations (periodic sides): every column is identical."""
    wl = L.reduced(L.directional_3d(), 6, 5, 24)
    d = wl["domains"][0]
    d["perturb"] = np.zeros((5, 6))
    dom = oracle.Domain(d)
    for _ in range(20):
        dom.step()
    for f in (dom.phi, dom.U, dom.T):
        assert np.max(np.abs(f - f[:, :1, :1])) < 1e-14
