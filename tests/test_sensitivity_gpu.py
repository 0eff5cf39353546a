"""Update-factor sensitivity under forced convection (Sections 4.1, 4.2).

The thermal case (Fig. 4c) is run with N_T = 15, 30, 45 and the solutal
case (Fig. 7c) with N_U = 15, 30, 45, all other parameters fixed
(dt_base = 1/15, N_phi = 15, N_F = 1).  The paper reports directional tip
velocities that are nearly indistinguishable across the update factors and
the ordering v_west > v_normal > v_east (inlet on the west side).  Here:
the tip lengths at the end keep that ordering (and north = south), and
across update factors the tip-length histories over the second half of the
run differ by at most 2 % and their mean velocities by at most 5 %, in FP32
(the runs are 120k and 150k base steps).
"""

import sys

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tip_history(wl, t_end, every_t):
    """Directional tip lengths (east, north, west, south) from the seed
    centre, sampled every ``every_t`` units of dt_phi."""
    from paper_2609_25670_amd import simulation_for

    d = wl["domains"][0]
    per_t = d["N_phi"]                      # base steps per unit time (dt_phi = 1)
    sim = simulation_for(wl, storage="f32")
    ts, tips = [], []
    for _ in range(int(t_end / every_t)):
        dd = sim.step(int(every_t * per_t), diag=True)[0]
        assert dd["nonfinite"] == 0
        ts.append(dd["step"] / per_t)
        tips.append(dd["tip"][:4])
    sim.close()
    return np.array(ts), np.array(tips)


def _check(name, runs, tol_pos, tol_vel):
    t, base = runs[0][1], runs[0][2]
    half = len(t) // 2
    for N, _, tips in runs:
        e, n, w, s = tips[-1]
        v = (tips[-1] - tips[half]) / (t[-1] - t[half])
        _say(f"  {name} N={N}: tips at the end E {e:.2f} N {n:.2f} W {w:.2f} S {s:.2f}; "
             f"mean velocity over the second half E {v[0]:.3e} N {v[1]:.3e} W {v[2]:.3e}")
        assert w > n > e, (N, tips[-1])              # upstream tip longest, downstream shortest
        assert abs(n - s) <= 1e-3 * n, (N, n, s)     # symmetric about the flow axis
    vb = (base[-1] - base[half]) / (t[-1] - t[half])
    for N, _, tips in runs[1:]:
        dpos = np.max(np.abs(tips[half:, :3] - base[half:, :3]) / base[half:, :3], axis=0)
        v = (tips[-1] - tips[half]) / (t[-1] - t[half])
        dvel = np.abs(v[:3] - vb[:3]) / vb[:3]
        _say(f"  {name} N={N} vs N={runs[0][0]}: max relative tip-length difference (E, N, W) "
             f"{np.round(dpos, 4)}, velocity difference {np.round(dvel, 4)}")
        assert np.all(dpos <= tol_pos), (N, dpos)
        assert np.all(dvel <= tol_vel), (N, dvel)


def test_thermal_forced_convection_update_factor_sensitivity():
    runs = []
    for N_T in (15, 30, 45):
        _say(f"case thermal forced convection N_T={N_T}, t/tau0 = 64")
        runs.append((N_T,) + _tip_history(L.thermal_forced_512(N_T), t_end=8000.0, every_t=100.0))
    _check("thermal", runs, tol_pos=0.02, tol_vel=0.05)


def test_solutal_forced_convection_update_factor_sensitivity():
    runs = []
    for N_U in (15, 30, 45):
        _say(f"case solutal forced convection N_U={N_U}, t/tau0 = 200")
        runs.append((N_U,) + _tip_history(L.solutal_forced_1000(N_U), t_end=10000.0, every_t=100.0))
    _check("solutal", runs, tol_pos=0.02, tol_vel=0.05)


def test_thermosolutal_forced_convection_update_factor_sensitivity():
    """Section 4.3 (Fig. 10b, c): N_U = 30, 40, 50 with N_phi = N_T = N_F = 1,
    Le = 50, at tau0 = 500 (the printed 1000 is linearly unstable under
    Eq. 26), to t D_L / d0^2 = 1000 (about 150k base steps)."""
    runs = []
    for N_U in (30, 40, 50):
        wl = L.thermosolutal_forced_1500(N_U)
        d = wl["domains"][0]
        d0 = 0.554 * d["W0"]
        t_end = 1000.0 * d0 * d0 / d["D_L"]
        _say(f"case thermosolutal forced convection N_U={N_U}, t D_L/d0^2 = 1000 ({t_end:.0f} steps)")
        runs.append((N_U,) + _tip_history(wl, t_end=round(t_end, -3), every_t=2000.0))
    _check("thermosolutal", runs, tol_pos=0.02, tol_vel=0.05)
