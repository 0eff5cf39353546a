"""Full-size parity of the 2D workloads with the FP64 oracle.

The 1024 x 1024 forced-convection case is compared on the whole grid; the
256-domain ensemble runs whole in one context (every domain stepped by the
same launches) and a spread of its domains, smallest and largest included,
is compared with the oracle domain by domain.
"""

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


def _c3_full(wl, steps, case):
    from paper_2609_25670_amd import simulation_for

    names = ("phi", "U", "T", "rho", "vel")
    _say(f"case {case} full size fp64 {steps} steps")
    sim = simulation_for(wl, storage="f64")
    diag = sim.step(steps, diag=True)[0]
    got = sim.read(0, names)
    sim.close()
    assert diag["nonfinite"] == 0
    dom = oracle.run(wl["domains"][0], steps)
    ref = dict(phi=dom.phi, U=dom.U, T=dom.T, rho=dom.rho, vel=dom.u)
    for n in names:
        e = _rel(got[n], ref[n])
        _say(f"  {case}: {n} rel L2 = {e:.3e}")
        assert e <= TOL64, (n, e)


def test_thermosolutal_flow_1024_full_fp64():
    """All four fields on 1024 x 1024 (inlet/outflow flow, rotated seed),
    N = 1:1:4:2, FP64 against the oracle on every site.  At this scale
    (tau0 = 1000, so tau_phi ~ 0.512) the anisotropic streaming amplifies
    a checkerboard mode by about 1.4 per step, rounding differences
    included, so the window is 12 base steps."""
    _c3_full(L.thermosolutal_flow_1024(), 12, "thermosolutal_flow_1024")


def test_thermosolutal_flow_1024_stable_scale_full_fp64():
    """The same 1024 x 1024 case at tau0 = 100 (tau_phi ~ 0.62), D_L = 0.04,
    D_S = 4e-4, where the scheme is stable: 60 base steps on every site."""
    wl = L.thermosolutal_flow_1024()
    wl["domains"][0].update(tau0=100.0, D_L=0.04, D_S=4e-4)
    _c3_full(wl, 60, "thermosolutal_flow_1024 tau0=100")


def test_thermosolutal_flow_1024_as_specified_loses_stability():
    """At the Section 4.3 scale tau_phi ~ 0.512 lies below the margin the
    anisotropic streaming needs (about 0.52 at eps = 0.02), and the solid
    concentration relaxation time is 0.5008: the scheme diverges within
    about 170 base steps, as the oracle does on the same parameters.  The
    library reports it as LBM_EUNSTABLE with the non-finite count, and the
    state stays readable."""
    from paper_2609_25670_amd import lbm, simulation_for

    wl = L.thermosolutal_flow_1024()
    _say("case thermosolutal_flow_1024 fp32 divergence detection")
    sim = simulation_for(wl, storage="f32")
    with pytest.raises(lbm.LBMError) as ei:
        sim.step(400, diag=True)
    assert ei.value.status == lbm.LBM_EUNSTABLE
    assert ei.value.diag[0]["nonfinite"] > 0
    phi = sim.read(0, ("phi",))["phi"]
    assert phi.shape == (1024, 1024)
    sim.close()


def test_ensemble_256_full_fp64_sampled_domains():
    """All 256 domains (29.7 M sites, N_U = Le in {1, 10, 100, 1000}) in one
    FP64 context for 24 base steps; domains 0, 85, 170, 255 and the
    smallest and largest domain are each equal to their own oracle run."""
    from paper_2609_25670_amd import simulation_for

    wl = L.ensemble_256()
    doms = wl["domains"]
    sides = [d["nx"] for d in doms]
    pick = sorted({0, 85, 170, 255, int(np.argmin(sides)), int(np.argmax(sides))})
    names = ("phi", "U", "T")
    _say(f"case ensemble_256 full fp64 24 steps, compared domains {pick}")
    sim = simulation_for(wl, storage="f64")
    diag = sim.step(24, diag=True)
    got = {i: sim.read(i, names) for i in pick}
    sim.close()
    assert all(dd["nonfinite"] == 0 for dd in diag)
    for i in pick:
        dom = oracle.run(doms[i], 24)
        for n in names:
            e = _rel(got[i][n], getattr(dom, n))
            _say(f"  domain {i} ({sides[i]}^2, Le {doms[i]['Le']}): {n} rel L2 = {e:.3e}")
            assert e <= TOL64, (i, n, e)
