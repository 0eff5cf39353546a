"""The allocation-free stepping entry point (lbm_step_multirate_static)
against lbm_step_multirate: the same state bit for bit and the same
diagnostics, on two calls in a row (a larger context, then a smaller one,
so that the second call starts from the first call's leftovers in the
shared static scratch), and a clear error for a context whose scratch
exceeds the static array."""

import sys

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(wl, storage, steps, static, names, rows):
    from paper_2609_25670_amd import simulation_for

    sim = simulation_for(wl, storage=storage)
    if rows:
        sim.configure(rows, True)
    sim.step(steps[0], static=static)
    diag = sim.step(steps[1], diag=True, static=static)
    got = [sim.read(i, names) for i in range(sim.n)]
    sim.close()
    return got, diag


CASES = [
    # (label, workload, storage, (steps, steps with diagnostics), fields, tile rows), from the largest
    # reduction scratch (3D: one partial per 256 sites) to the smallest
    ("3D directional 64x32x40 bf16", lambda: L.reduced(L.directional_3d(), 64, 32, 40), "bf16", (32, 35),
     ("phi", "U", "T", "rho", "vel"), 0),
    ("batched 3 domains fp32", lambda: L.ensemble_256(n_domains=3, side_lo=40, side_hi=70), "f32", (30, 12),
     ("phi", "U", "T"), 16),
    ("thermosolutal flow 150x90 fp64", lambda: _flow(150, 90), "f64", (20, 13),
     ("phi", "U", "T", "rho", "vel", "f_phi", "jU", "jT", "f_F"), 8),
    ("solutal 70x52 fp32", lambda: L.reduced(L.solutal_512(), 70, 52), "f32", (9, 7),
     ("phi", "U", "jU"), 4),
]


def _flow(nx, ny):
    wl = L.reduced(L.thermosolutal_flow_1024(), nx, ny)
    wl["domains"][0]["tau0"] = 40.0
    return wl


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_static_entry_point_equals_the_allocating_one(case):
    """Bitwise-identical state and diagnostics.  The cases run in order
    from the largest scratch to the smallest."""
    import torch

    label, make, storage, steps, names, rows = case
    wl = make()
    _say(f"case no-alloc {label}: allocating entry point")
    ref, dref = _run(wl, storage, steps, False, names, rows)
    _say(f"case no-alloc {label}: static entry point")
    free0 = torch.cuda.mem_get_info()[0]
    got, dgot = _run(wl, storage, steps, True, names, rows)
    free1 = torch.cuda.mem_get_info()[0]
    for i in range(len(ref)):
        for n in names:
            assert np.array_equal(got[i][n], ref[i][n]), (label, i, n)
        for key in ("step", "solid", "M_C", "enthalpy", "mass", "S_phi", "J_U", "nonfinite", "t", "R_M",
                    "first_nonfinite_step", "tip"):
            assert dgot[i][key] == dref[i][key], (label, i, key, dgot[i][key], dref[i][key])
    _say(f"  equal; S_phi {dgot[0]['S_phi']:.3e}, R_M {dgot[0]['R_M']:.3e}; free memory {free0} -> {free1}")
    assert free1 >= free0 - (2 << 20)


def test_static_entry_point_rejects_an_oversized_context():
    """A 2D context of 8192 x 8192 (262,144 partial slots of 80 bytes at
    the smallest tile height) needs more reduction scratch than the 16 MiB
    static array: LBM_EINVAL with the sizes in the message."""
    from paper_2609_25670_amd import lbm

    d = L.configs._base_domain()
    d.update(nx=8192, ny=8192, W0=1.0, tau0=1.0)
    _say("case no-alloc oversized context")
    sim = lbm.Simulation([d], storage="f32")
    with pytest.raises(lbm.LBMError) as ei:
        sim.step(1, static=True)
    sim.close()
    assert ei.value.status == lbm.LBM_EINVAL
    assert "static scratch holds 16777216" in str(ei.value)
