"""The paper's own scalar lattice, D2Q9 (Eq. 15-16), for the phase, U and T
fields on the GPU, against the FP64 oracle's literal D2Q9 moment-space
collision, and compared with the D2Q5 default on the thermal and solutal
benchmarks."""

import sys

import numpy as np
import pytest

import lbm_inputs as L
import oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 1e-300 else 1.0)


def _q9(wl):
    for d in wl["domains"]:
        d["q_scalar"] = 9
    return wl


def _ref(dom, names):
    m = dict(phi=dom.phi, U=getattr(dom, "U", None), T=getattr(dom, "T", None), rho=dom.rho, vel=dom.u,
             f_phi=dom.f_phi, P_U=dom.P_U)
    if "jU" in names:
        m["jU"] = dom.moments("U")[1]
    if "jT" in names:
        m["jT"] = dom.moments("T")[1]
    return {n: m[n] for n in names}


def _parity(case, wl, steps, names, storage="f64", tol=TOL64):
    from paper_2609_25670_amd import simulation_for

    _say(f"case d2q9 {case} {storage} {steps} steps")
    sim = simulation_for(wl, storage=storage)
    diag = sim.step(steps, diag=True)
    got = [sim.read(i, names) for i in range(sim.n)]
    sim.close()
    for i, d in enumerate(wl["domains"]):
        dom = oracle.run(d, steps)
        refs = _ref(dom, names)
        for n, r in refs.items():
            e = _rel(got[i][n], r)
            bar = tol
            if n in ("jU", "jT"):
                # a first moment is a difference of populations of the size of
                # the zeroth moment, so any FP64 evaluation loses the digits of
                # that cancellation: its relative bar is the field's scaled by
                # |zeroth| / |first| (1 where the first moment is the larger);
                # the error on the zeroth moment's scale is printed beside
                z = dom.U if n == "jU" else dom.T
                ratio = np.linalg.norm(z) / max(np.linalg.norm(r), 1e-300)
                bar = tol * max(1.0, ratio)
                ez = np.linalg.norm(got[i][n] - r) / np.linalg.norm(z)
                _say(f"  {case} domain {i}: {n} rel L2 = {e:.3e} (bar {bar:.1e}; on the scale of the zeroth "
                     f"moment {ez:.3e})")
            else:
                _say(f"  {case} domain {i}: {n} rel L2 = {e:.3e}")
            assert e <= bar, (case, i, n, e, bar)
    return diag


def test_d2q9_thermal_fp64():
    """Thermal dendrite (phi + T, periodic) with D2Q9 scalars, 400 steps."""
    _parity("thermal_128", _q9(L.thermal_128()), 400, ("phi", "T", "f_phi", "jT"))


def test_d2q9_solutal_walls_fp64():
    """Solutal dendrite (phi + U, zero-flux walls: diagonal bounce-back in the
    corners) on 150 x 70, N_U = 4, 400 steps; then accumulated coupling."""
    wl = _q9(L.reduced(L.solutal_512(), 150, 70))
    _parity("solutal", wl, 400, ("phi", "U", "f_phi", "jU"))
    wl["domains"][0]["coupling"] = "accum"
    _parity("solutal accum", wl, 402, ("phi", "U", "jU", "P_U"))


def test_d2q9_thermosolutal_flow_fp64():
    """All four fields, inlet/outflow flow, rotated seed, 150 x 90."""
    wl = _q9(L.reduced(L.thermosolutal_flow_1024(), 150, 90))
    d = wl["domains"][0]
    d["seeds"] = [(75.0, 44.0, 12.0)]
    d["tau0"] = 40.0
    d["u_in"] = 0.02
    _parity("thermosolutal_flow", wl, 300, ("phi", "U", "T", "rho", "vel", "f_phi", "jU", "jT"))


def test_d2q9_cold_bottom_fp64():
    """The Section 4.4 directional case (anti-bounce-back on the cold bottom
    for the three upward directions), Le = 10, 130 x 90."""
    wl = _q9(L.directional_2d(Le=10, nx=130, ny=90))
    _parity("directional_2d", wl, 240, ("phi", "U", "T", "jU", "jT"))


def test_d2q9_batched_uneven_fp32():
    """Three uneven domains with different update factors in one FP32
    context (FP32 tolerance)."""
    wl = _q9(L.ensemble_256(n_domains=3, side_lo=40, side_hi=90))
    for i, d in enumerate(wl["domains"]):
        d["tau0"] = 30.0
        d["N_U"] = [1, 10, 2][i]
        d["D_L"] = 0.026 / d["N_U"]
        d["D_S"] = 1e-2 * d["D_L"]
    _parity("batched", wl, 120, ("phi", "U", "T"), storage="f32", tol=2e-6)


def test_d2q9_against_d2q5_tip_lengths():
    """The two scalar lattices solve the same equations.  Where the
    interface is resolved as in the paper (W0 = 2.5: the Section 4.2
    solutal dendrite on 256^2 over 16k steps, and the Section 4.1 thermal
    dendrite without flow on 512^2 to t = 32 tau0) the mean tip lengths
    agree to within 1 %.  The 128^2 thermal workload uses W0 = 1, where the
    interface spans two nodes and the lattices' own anisotropy separates the
    tips by about 8 % at 1000 steps; that difference is printed, not bounded."""
    from paper_2609_25670_amd import simulation_for

    def tips(wl, steps, every):
        sim = simulation_for(wl, storage="f32")
        out = []
        for _ in range(steps // every):
            dd = sim.step(every, diag=True)[0]
            assert dd["nonfinite"] == 0
            out.append(float(np.mean(dd["tip"][:4])))
        sim.close()
        return np.array(out)

    def thermal_diffusion_512():
        wl = L.thermal_forced_512(15)
        d = wl["domains"][0]
        d.update(has_flow=False, u_in=0.0, u0_liquid_only=False)
        return wl

    cases = (("solutal_256", lambda: L.reduced(L.solutal_512(), 256, 256), 16000, 1000, 0.01),
             ("thermal_512 (Sec. 4.1, W0 = 2.5)", thermal_diffusion_512, 60000, 3000, 0.01),
             ("thermal_128 (W0 = 1)", L.thermal_128, 1000, 250, None))
    for name, make, steps, every, tol in cases:
        t5 = tips(make(), steps, every)
        t9 = tips(_q9(make()), steps, every)
        rel = np.abs(t9 - t5) / t5
        _say(f"  {name}: tip length D2Q5 {t5[-1]:.3f}, D2Q9 {t9[-1]:.3f}; largest relative difference "
             f"over the run {rel.max():.3e}")
        if tol is not None:
            assert rel.max() <= tol, (name, rel.max())
