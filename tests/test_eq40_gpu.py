"""The Eq. (40) phase-gradient variant (scope f4): grad phi for the
normal, a_s and N of the phase collision from the non-equilibrium phase
populations, with the previous phase step's v_n and tau_phi at the site,
instead of the isotropic stencil.  FP64 parity with the oracle's variant,
and its effect on the tip velocity against the stencil reading."""

import sys

import numpy as np
import pytest

import lbm_inputs as L
import oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TIP_BAR = 0.02


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(name, q):
    if name == "thermal":
        wl = L.thermal_128()
    else:
        wl = L.reduced(L.solutal_512(), 150, 90)
    for d in wl["domains"]:
        d["q_scalar"] = q
        d["grad_phi"] = "eq40"
    return wl


@pytest.mark.parametrize("q", [5, 9])
@pytest.mark.parametrize("name,steps", [("thermal", 120), ("solutal", 64)])
def test_eq40_variant_fp64_parity(name, steps, q):
    from paper_2609_25670_amd import simulation_for

    wl = _case(name, q)
    field = "T" if name == "thermal" else "U"
    _say(f"case eq40 {name} D2Q{q} fp64 {steps} steps")
    sim = simulation_for(wl, storage="f64")
    sim.configure(8, True)
    sim.step(steps)
    got = sim.read(0, ("phi", field))
    sim.close()
    dom = oracle.run(wl["domains"][0], steps)
    for n, ref in (("phi", dom.phi), (field, getattr(dom, field))):
        e = _rel(got[n], ref)
        _say(f"  {n} rel L2 = {e:.3e}")
        assert e <= TOL64, (n, e)


def _thermal_diffusion_512():
    """The Section 4.1 thermal dendrite (W0 = 2.5) on 512^2 without flow."""
    wl = L.thermal_forced_512(15)
    wl["domains"][0].update(has_flow=False, u_in=0.0, u0_liquid_only=False)
    return wl


# (name, workload, steps, diagnostic interval, bar on the largest relative
# difference of the mean tip length over the run, or None: printed only)
TIP_CASES = (
    ("solutal_256 (Sec. 4.2, W0 = 2.5)", lambda: L.reduced(L.solutal_512(), 256, 256), 16000, 1000, TIP_BAR),
    ("thermal_512 (Sec. 4.1, W0 = 2.5)", _thermal_diffusion_512, 60000, 3000, TIP_BAR),
    ("thermal_128 (W0 = 1)", L.thermal_128, 1600, 200, None),
)


@pytest.mark.parametrize("case", range(len(TIP_CASES)), ids=[c[0].split()[0] for c in TIP_CASES])
def test_eq40_against_stencil_tip_length(case):
    """grad phi from Eq. (40) (lagged one phase step) and from the isotropic
    stencil reconstruct the same gradient to second order in the interface
    resolution.  Where the interface is resolved as in the paper (W0 = 2.5)
    the mean tip lengths of the two readings stay within TIP_BAR of each
    other over the run.  At W0 = 1 (thermal 128^2, an interface of about
    three cells) the two differ by several per cent; printed, not bounded."""
    from paper_2609_25670_amd import simulation_for

    name, make, steps, every, bar = TIP_CASES[case]
    tips = {}
    for mode in ("fd", "eq40"):
        wl = make()
        wl["domains"][0]["grad_phi"] = mode
        _say(f"case eq40 tip {name} {mode} {steps} steps")
        sim = simulation_for(wl, storage="f64")
        out = []
        for _ in range(steps // every):
            dd = sim.step(every, diag=True)[0]
            assert dd["nonfinite"] == 0
            out.append(float(np.mean(dd["tip"][:4])))
        sim.close()
        tips[mode] = np.array(out)
    rel = np.abs(tips["eq40"] - tips["fd"]) / tips["fd"]
    _say(f"  {name}: tip length stencil {tips['fd'][-1]:.3f}, Eq. (40) {tips['eq40'][-1]:.3f}; "
         f"largest relative difference over the run {rel.max():.3e}")
    assert tips["eq40"][-1] > tips["eq40"][0]
    if bar is not None:
        assert rel.max() <= bar, (name, rel.max())
