"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 storage/compute is compared element by element with the oracle at
1e-12 relative L2 per field (the bar the method's FP64 path is held to).
Grids are chosen to span several 64 x TY tiles with ragged tails in x and y.
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


def _gpu(wl, steps, storage="f64", names=("phi",), tile_rows=None, use_graph=True, domains=None, fuse=False,
         march=None):
    from paper_2609_25670_amd import simulation_for

    sim = simulation_for(wl, storage=storage)
    if tile_rows is not None:
        sim.configure(tile_rows, use_graph, fuse, march)
    diag = sim.step(steps, diag=True)
    outs = [sim.read(i, names) for i in (domains if domains is not None else range(sim.n))]
    sim.close()
    return outs, diag


def _oracle_fields(dom, names):
    out = {}
    for n in names:
        if n == "phi":
            out[n] = dom.phi
        elif n == "U":
            out[n] = dom.U
        elif n == "T":
            out[n] = dom.T
        elif n == "rho":
            out[n] = dom.rho
        elif n == "vel":
            out[n] = dom.u
        elif n == "f_phi":
            out[n] = dom.f_phi
        elif n == "jU":
            out[n] = dom.moments("U")[1]
        elif n == "jT":
            out[n] = dom.moments("T")[1]
        elif n == "f_F":
            out[n] = dom.f_F
        elif n == "P_U":
            out[n] = dom.P_U
    return out


def _compare(case, got, ref, tol):
    for name, r in ref.items():
        e = _rel(got[name], r)
        _say(f"  {case}: {name} rel L2 = {e:.3e}")
        assert e <= tol, (case, name, e)


def test_thermal_128_full_run_fp64():
    """2D thermal dendrite 128^2 periodic, phi + T, 1000 steps."""
    wl = L.thermal_128()
    names = ("phi", "T", "f_phi", "jT")
    _say("case thermal_128 fp64 1000 steps")
    (got,), diag = _gpu(wl, 1000, names=names)
    dom = oracle.run(wl["domains"][0], 1000)
    _compare("thermal_128", got, _oracle_fields(dom, names), TOL64)
    t = oracle.diag.totals(dom)
    assert abs(diag[0]["enthalpy"] - t["enthalpy"]) < 1e-9 * abs(t["enthalpy"])
    assert abs(diag[0]["solid"] - t["solid"]) < 1e-9 * abs(t["solid"])
    tips = oracle.diag.tips(dom)[0]
    assert np.allclose(diag[0]["tip"][:4], tips, atol=1e-9)


def test_solutal_reduced_fp64_ragged_tiles():
    """2D solutal dendrite (N_U = 4, zero-flux) on 150 x 70, with the
    default configuration (3 of every 4 transfers deferred into the next
    phase kernel)."""
    wl = L.reduced(L.solutal_512(), 150, 70)
    names = ("phi", "U", "f_phi", "jU")
    _say("case solutal 150x70 fp64 600 steps")
    (got,), diag = _gpu(wl, 600, names=names)
    dom = oracle.run(wl["domains"][0], 600)
    _compare("solutal", got, _oracle_fields(dom, names), TOL64)
    t = oracle.diag.totals(dom)
    assert abs(diag[0]["M_C"] - t["M_C"]) < 1e-10 * t["M_C"]
    assert abs(diag[0]["S_phi"] - t["S_phi"]) < 1e-10 * t["S_phi"]


def test_thermosolutal_flow_reduced_fp64():
    """All four fields, N = 1:1:4:2, rotated seed, inlet/outflow flow."""
    wl = L.reduced(L.thermosolutal_flow_1024(), 150, 90)
    d = wl["domains"][0]
    d["seeds"] = [(75.0, 44.0, 12.0)]
    d["tau0"] = 40.0          # faster phase dynamics so 300 steps exercise the coupling
    d["u_in"] = 0.02
    names = ("phi", "U", "T", "rho", "vel", "f_phi", "jU", "jT", "f_F")
    _say("case thermosolutal_flow 150x90 fp64 300 steps")
    (got,), diag = _gpu(wl, 300, names=names)
    dom = oracle.run(d, 300)
    _compare("thermosolutal_flow", got, _oracle_fields(dom, names), TOL64)


def test_accumulated_coupling_fp64():
    """The delayed coarse-step injection variant (pending planes)."""
    wl = L.reduced(L.solutal_512(), 100, 80)
    wl["domains"][0]["coupling"] = "accum"
    names = ("phi", "U", "jU", "P_U")
    _say("case accumulated coupling 100x80 fp64 402 steps")
    (got,), diag = _gpu(wl, 402, names=names)
    dom = oracle.run(wl["domains"][0], 402)
    _compare("accum", got, _oracle_fields(dom, ("phi", "U", "jU")), TOL64)
    assert _rel(got["P_U"], dom.P_U) < 1e-11
    assert abs(diag[0]["J_U"] - dom.J_U) <= 1e-10 * dom.J_U


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_uneven_domains_fp64(use_graph):
    """Five independent domains of uneven sizes with different update factors
    (Le = N_U in {1, 10, 100, 1000}) and variable thermal properties, in one
    context; each equals its own oracle run."""
    wl = L.ensemble_256(n_domains=5, side_lo=40, side_hi=100)
    for i, d in enumerate(wl["domains"]):
        d["tau0"] = 30.0
        Le = [1, 10, 1, 10, 2][i]
        d["N_U"] = Le
        d["D_L"] = 0.026 / Le
        d["D_S"] = 1e-2 * d["D_L"]
    names = ("phi", "U", "T")
    steps = 420
    _say(f"case batched 5 domains fp64 {steps} steps graph={use_graph}")
    gots, diag = _gpu(wl, steps, names=names, tile_rows=16, use_graph=use_graph)
    for i, d in enumerate(wl["domains"]):
        dom = oracle.run(d, steps)
        _compare(f"domain{i}", gots[i], _oracle_fields(dom, names), TOL64)


SMALLEST_2D = {
    "solutal_3x3_walls": (L.solutal_512, 3, 3, ("wall", "wall", "wall"), None),
    "solutal_5x4_wall_periodic": (L.solutal_512, 5, 4, ("wall", "periodic", "wall"), None),
    "four_field_4x3_inlet": (L.thermosolutal_flow_1024, 4, 3, ("wall", "wall", "wall"), None),
    "four_field_5x4_periodic": (L.thermosolutal_flow_1024, 5, 4, ("periodic", "periodic", "wall"),
                                ("periodic", "periodic", "periodic")),
}


@pytest.mark.parametrize("case", sorted(SMALLEST_2D))
def test_smallest_2d_grids_fp64(case):
    """Domains smaller than one tile, down to the smallest side accepted (3),
    with a seed of radius 1.2 in the middle: the tiles' rings and the
    phase window wrap across the whole periodic domain or fold onto the
    walls, and the inlet and outflow columns of the four-field case are
    neighbours."""
    make, nx, ny, bc, fbc = SMALLEST_2D[case]
    wl = L.reduced(make(), nx, ny)
    d = wl["domains"][0]
    d.update(bc=bc, seeds=[(nx / 2 - 0.5, ny / 2 - 0.5, 1.2)])
    if fbc:
        d.update(flow_bc=fbc)
    names = ("phi", "U", "T", "rho", "vel") if d.get("has_flow") else ("phi", "U")
    _say(f"case smallest 2d {case} fp64 24 steps")
    gots, diag = _gpu(wl, 24, names=names)
    dom = oracle.run(d, 24)
    ref = _oracle_fields(dom, names)
    for n, r in ref.items():
        e = _rel(gots[0][n], r)
        bar = TOL64
        if n == "vel":
            # the velocity is a first moment of populations the size of rho:
            # its relative bar is scaled by |rho| / |rho u| (the cancellation
            # any FP64 evaluation goes through); printed with its error on
            # the scale of rho
            z = np.linalg.norm(dom.rho)
            bar = TOL64 * max(1.0, z / max(np.linalg.norm(r * dom.rho), 1e-300))
            _say(f"  {case}: vel rel L2 = {e:.3e} (bar {bar:.1e}; on the scale of rho "
                 f"{np.linalg.norm(gots[0][n] - r) / z:.3e})")
        else:
            _say(f"  {case}: {n} rel L2 = {e:.3e}")
        assert e <= bar, (case, n, e, bar)
    assert diag[0]["nonfinite"] == 0


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_batched_domains_are_bitwise_equal_to_each_domain_alone(storage):
    """Each domain of a batched context (uneven sizes and update factors)
    ends bit for bit where the same domain ends in a context of its own:
    the batch shares launches, never arithmetic or rounding streams."""
    wl = L.ensemble_256(n_domains=4, side_lo=40, side_hi=100)
    for i, d in enumerate(wl["domains"]):
        d["tau0"] = 30.0
        Le = [1, 10, 2, 10][i]
        d["N_U"] = Le
        d["D_L"] = 0.026 / Le
        d["D_S"] = 1e-2 * d["D_L"]
    names = ("phi", "U", "T", "jU", "jT")
    steps = 200
    _say(f"case batched vs alone {storage} {steps} steps")
    batch, _ = _gpu(wl, steps, storage=storage, names=names)
    for i, d in enumerate(wl["domains"]):
        alone, _ = _gpu(dict(wl, domains=[d]), steps, storage=storage, names=names)
        for n in names:
            same = np.array_equal(batch[i][n], alone[0][n])
            _say(f"  domain {i} ({d['nx']} x {d['ny']}, N_U = {d['N_U']}): {n} bitwise equal = {same}")
            assert same, (storage, i, n)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_tile_shapes_graph_and_fusion_are_bitwise_identical(storage):
    """Race detector: every tile height, graph replay versus eager launches,
    the phase + transfer kernel versus the two separate kernels, and the
    marching phase kernel versus the tiled one give bitwise-identical
    state."""
    wl = L.reduced(L.thermosolutal_flow_1024(), 130, 75)
    wl["domains"][0]["tau0"] = 40.0
    names = ("phi", "U", "T", "rho", "vel", "f_phi", "jU", "jT", "f_F")
    ref = None
    runs = [(r, g, f, False) for r in (4, 8, 16, 32) for g in (True, False) for f in (True, False)]
    runs += [(r, g, False, True) for r in (4, 32) for g in (True, False)]
    runs += [(r, g, True, True) for r in (8, 16) for g in (True, False)]   # fused transfer, marching transports
    for rows, g, fuse, march in runs:
        _say(f"case determinism {storage} rows={rows} graph={g} fused={fuse} march={march}")
        (got,), _ = _gpu(wl, 64, storage=storage, names=names, tile_rows=rows, use_graph=g, fuse=fuse, march=march)
        if ref is None:
            ref = got
        else:
            for n in names:
                assert np.array_equal(got[n], ref[n]), (rows, g, fuse, march, n)


@pytest.mark.parametrize("storage,case", [("f64", "solutal"), ("f32", "solutal"), ("f64", "thermosolutal"),
                                          ("f32", "flow")])
def test_deferred_transfer_is_bitwise_identical(storage, case):
    """The transfer of a phase step with no transport after it (3 of 4 in
    the solutal case, N_U = 4; 2 of 3 with U and T at N = 3 and latent
    heat) runs inside the next phase kernel, and the transfer of a step at
    which U is due inside that U transport (every step with flow, N_U = 1,
    where the transport takes the velocity).  Against the separate kernels:
    the same state bit for bit and the same S_phi and J_U, over tile
    heights, graph replay or direct launches, and calls that end inside a
    multirate cycle (5 + 3 + 59 steps)."""
    from paper_2609_25670_amd import simulation_for

    if case == "solutal":
        wl = L.reduced(L.solutal_512(), 130, 75)
        names = ("phi", "U", "f_phi", "jU")
    elif case == "thermosolutal":
        wl = L.reduced(L.thermosolutal_flow_1024(), 130, 75)
        wl["domains"][0].update(has_flow=False, N_U=3, N_T=3, tau0=40.0)
        names = ("phi", "U", "T", "f_phi", "jU", "jT")
    else:
        wl = L.reduced(L.thermosolutal_flow_1024(), 130, 75)
        wl["domains"][0].update(tau0=40.0)
        names = ("phi", "U", "T", "vel", "f_phi", "jU", "jT")
    ref = None
    for rows, g, defer in [(r, g, d) for r in (4, 16) for g in (True, False) for d in (False, True)]:
        _say(f"case deferred transfer {storage} rows={rows} graph={g} defer={defer}")
        sim = simulation_for(wl, storage=storage)
        sim.configure(rows, g, False, False, defer)
        sim.step(5)
        sim.step(3)
        diag = sim.step(59, diag=True)[0]
        got = sim.read(0, names)
        sim.close()
        if ref is None:
            ref = (got, diag)
        else:
            for n in names:
                assert np.array_equal(got[n], ref[0][n]), (rows, g, defer, n)
            assert diag["S_phi"] == ref[1]["S_phi"] and diag["J_U"] == ref[1]["J_U"]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_deferred_transfer_more_blocks_than_fit_on_the_chip(storage):
    """The deferred transfer reads the transfer's old phase field on rings
    that neighbouring blocks own, while those blocks write the next phase
    field.  On 1024 x 1024 with four seeds (long interfaces across many
    tile edges) and 64 x 4 tiles, 4096 blocks, more than are resident at
    once, so late blocks run after their neighbours have finished: the
    state equals that of the separate kernels bit for bit, and FP64 equals
    the oracle."""
    from paper_2609_25670_amd import simulation_for

    wl = L.reduced(L.solutal_512(), 1024, 1024)
    d = wl["domains"][0]
    d["seeds"] = [(300.5, 300.5, 120.0), (720.5, 310.5, 110.0), (310.5, 730.5, 100.0), (715.5, 715.5, 130.0)]
    names = ("phi", "U", "f_phi", "jU")
    steps = 27
    res = {}
    for defer in (False, True):
        _say(f"case deferred transfer 1024x1024 {storage} rows=4 defer={defer}")
        sim = simulation_for(wl, storage=storage)
        sim.configure(4, True, False, False, defer)
        diag = sim.step(steps, diag=True)[0]
        res[defer] = sim.read(0, names)
        sim.close()
        assert diag["nonfinite"] == 0
    for n in names:
        assert np.array_equal(res[True][n], res[False][n]), n
    if storage == "f64":
        dom = oracle.run(d, steps)
        for n, ref in (("phi", dom.phi), ("U", dom.U)):
            e = _rel(res[True][n], ref)
            _say(f"  deferred 1024x1024: {n} rel L2 = {e:.3e}")
            assert e <= TOL64, (n, e)


@pytest.mark.parametrize("q", [5, 9])
def test_marching_kernels_fp64(q):
    """The marching phase, transfer and T-transport kernels on the 2D
    directional case (cold bottom, walls, Le = 10) on 150 x 70 (a second
    run of 6 rows, 150 = 2 x 64 + 22 columns), in D2Q5 and D2Q9: FP64
    parity with the oracle, and the same S_phi and J_U diagnostics as the
    tiled kernels."""
    wl = L.directional_2d(Le=10, coupling="instant", nx=150, ny=70)
    wl["domains"][0]["q_scalar"] = q
    names = ("phi", "U", "T", "f_phi", "jU", "jT")
    _say(f"case marching kernels D2Q{q} fp64 150x70 120 steps")
    (got,), diag = _gpu(wl, 120, names=names, tile_rows=8, march=True)
    _, diag_t = _gpu(wl, 120, names=names, tile_rows=8, march=False)
    assert diag[0]["S_phi"] == diag_t[0]["S_phi"] and diag[0]["J_U"] == diag_t[0]["J_U"]
    dom = oracle.run(wl["domains"][0], 120)
    _compare(f"marching D2Q{q}", got, _oracle_fields(dom, names), TOL64)


@pytest.mark.parametrize("storage,case", [("f64", "directional"), ("f16", "directional"), ("f32", "flow")])
def test_marching_transfer_in_T_transport_is_bitwise_identical(storage, case):
    """On the marching path the transfer of a step at which T is due runs
    inside the T transport (every step in the directional case, N_T = 1;
    every fourth with flow, N_T = 4, where the transport takes the
    velocity).  Against the separate marching kernels: the same state bit
    for bit and the same S_phi and J_U, over tile heights (partial slots),
    graph replay or direct launches and calls that end inside a cycle."""
    from paper_2609_25670_amd import simulation_for

    if case == "directional":
        wl = L.directional_2d(Le=10, coupling="instant", nx=150, ny=70)
        names = ("phi", "U", "T", "f_phi", "jU", "jT")
    else:
        wl = L.reduced(L.thermosolutal_flow_1024(), 130, 75)
        wl["domains"][0].update(tau0=40.0)
        names = ("phi", "U", "T", "vel", "f_phi", "jU", "jT")
    ref = None
    for rows, g, defer in [(r, g, d) for r in (4, 16) for g in (True, False) for d in (False, True)]:
        _say(f"case marching transfer in T {case} {storage} rows={rows} graph={g} defer={defer}")
        sim = simulation_for(wl, storage=storage)
        sim.configure(rows, g, False, True, defer)
        sim.step(5)
        sim.step(3)
        diag = sim.step(41, diag=True)[0]
        got = sim.read(0, names)
        sim.close()
        assert diag["nonfinite"] == 0
        if ref is None:
            ref = (got, diag)
        else:
            for n in names:
                assert np.array_equal(got[n], ref[0][n]), (rows, g, defer, n)
            assert diag["S_phi"] == ref[1]["S_phi"] and diag["J_U"] == ref[1]["J_U"]


@pytest.mark.parametrize("fuse", [False, True])
@pytest.mark.parametrize("coupling", ["accum", "instant"])
def test_marching_U_transport_is_bitwise_identical(coupling, fuse):
    """The U transport marches with the phase field (62-column runs): the
    solutal case on 150 x 70 (walls, a 26-column last run, a 6-row last
    run) with accumulated or instantaneous coupling, N_U = 4, equals the
    tiled kernels bit for bit, with the same S_phi and J_U (with
    accumulated coupling J_U is the largest injected U, from the U
    transport).  With the transfer fused into the (tiled) phase kernel
    the transports still march: S_phi then comes from the tiles and the
    accumulated J_U from the marching U transport."""
    from paper_2609_25670_amd import simulation_for

    wl = L.reduced(L.solutal_512(), 150, 70)
    wl["domains"][0]["coupling"] = coupling
    names = ("phi", "U", "f_phi", "jU") + (("P_U",) if coupling == "accum" else ())
    res = []
    for march in (False, True):
        _say(f"case marching U transport {coupling} fuse={fuse} march={march}")
        sim = simulation_for(wl, storage="f64")
        sim.configure(8, True, fuse, march)
        sim.step(6)
        diag = sim.step(33, diag=True)[0]
        res.append((sim.read(0, names), diag))
        sim.close()
    for n in names:
        assert np.array_equal(res[0][0][n], res[1][0][n]), n
    assert res[0][1]["S_phi"] == res[1][1]["S_phi"] and res[0][1]["J_U"] == res[1][1]["J_U"]
    assert res[1][1]["J_U"] > 0


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_work_queue_launches_are_bitwise_identical(storage):
    """The marching kernels launched as persistent blocks that take their
    runs from the eight per-XCD work queues equal the static one-block-per-
    run grids bit for bit: twelve uneven domains of the ensemble (every
    Lewis number, so every update group of U), with graph replay and with
    direct launches, the same state and the same S_phi and J_U; and the
    FP64 form equals the oracle on two of the domains."""
    from paper_2609_25670_amd import simulation_for

    wl = L.ensemble_256(n_domains=12, side_lo=48, side_hi=190)
    names = ("phi", "U", "T", "jU", "jT")
    res = {}
    for queue in (False, True):
        for g in (True, False):
            _say(f"case work queue {storage} queue={queue} graph={g}")
            sim = simulation_for(wl, storage=storage)
            sim.configure(16, g, False, True, True, queue)
            sim.step(7)
            diag = sim.step(26, diag=True)
            got = [sim.read(i, names) for i in range(sim.n)]
            sim.close()
            res[(queue, g)] = (got, diag)
    ref = res[(False, True)]
    for key, (got, diag) in res.items():
        for i in range(len(got)):
            for n in names:
                assert np.array_equal(got[i][n], ref[0][i][n]), (key, i, n)
            assert diag[i]["S_phi"] == ref[1][i]["S_phi"] and diag[i]["J_U"] == ref[1][i]["J_U"], key
    if storage == "f64":
        for i in (0, 7):
            dom = oracle.run(wl["domains"][i], 33)
            _compare(f"work queue domain {i}", res[(True, True)][0][i], _oracle_fields(dom, ("phi", "U", "T")),
                     TOL64)


@pytest.mark.parametrize("bcx", ["periodic", "wall"])
def test_marching_one_column_last_run_fp64(bcx):
    """Marching on 125 x 67: the 62-column runs leave a last run one column
    wide (125 = 2 x 62 + 1), the 64-column phase runs one of 61, and the
    row runs a last run of 3 rows; x periodic (wrapping across the narrow
    run) or walled.  Thermosolutal (U every step, T every second step,
    latent heat): FP64 parity with the oracle and the same state as the
    tiled kernels."""
    wl = L.reduced(L.thermosolutal_flow_1024(), 125, 67)
    d = wl["domains"][0]
    d.update(has_flow=False, N_U=1, N_T=2, tau0=40.0, bc=(bcx, "wall", "wall"))
    names = ("phi", "U", "T", "f_phi", "jU", "jT")
    _say(f"case marching one-column last run 125x67 x={bcx} fp64 40 steps")
    (got,), diag = _gpu(wl, 40, names=names, tile_rows=8, march=True)
    (ref_t,), diag_t = _gpu(wl, 40, names=names, tile_rows=8, march=False)
    for n in names:
        assert np.array_equal(got[n], ref_t[n]), n
    assert diag[0]["S_phi"] == diag_t[0]["S_phi"] and diag[0]["J_U"] == diag_t[0]["J_U"]
    dom = oracle.run(d, 40)
    _compare(f"one-column run x={bcx}", got, _oracle_fields(dom, names), TOL64)


def test_checkpoint_restore_is_bitwise():
    """Read the full state, write it into a fresh context, continue: equal
    to the uninterrupted run, bit for bit."""
    from paper_2609_25670_amd import simulation_for

    wl = L.reduced(L.thermosolutal_flow_1024(), 100, 70)
    wl["domains"][0]["tau0"] = 40.0
    _say("case checkpoint")
    a = simulation_for(wl, storage="f64")
    a.configure(16, True)
    a.step(40)
    snap = a.read(0, a.state_names())
    a.step(24)
    ref = a.read(0, ("phi", "U", "T", "rho", "vel"))
    a.close()
    b = simulation_for(wl, storage="f64")
    b.configure(16, True)
    b.step(40)                       # same step counter (same buffer parity)
    b.write(0, {k: v for k, v in snap.items()})
    b.step(24)
    got = b.read(0, ("phi", "U", "T", "rho", "vel"))
    b.close()
    for n in ref:
        assert np.array_equal(got[n], ref[n]), n


def test_tile_rows_and_marching_queries():
    """lbm_tile_rows reports the fixed tile height, 0 before the autotuner
    has run and its pick afterwards; lbm_marching follows lbm_configure."""
    from paper_2609_25670_amd import simulation_for

    wl = L.reduced(L.solutal_512(), 130, 75)
    _say("case tile-rows and marching queries")
    sim = simulation_for(wl, storage="f32")
    assert sim.tile_rows == 0
    sim.step(4)
    assert sim.tile_rows in (4, 8, 16, 32)
    for rows in (4, 8, 16, 32):
        sim.configure(rows, True)
        assert sim.tile_rows == rows
    sim.configure(8, True, False, True)
    assert sim.marching
    sim.configure(8, True, False, False)
    assert not sim.marching
    sim.close()


def test_nonfinite_state_is_reported():
    """A NaN written into U is caught by the diagnostics: the step call
    returns LBM_EUNSTABLE and the count is reported."""
    from paper_2609_25670_amd import lbm, simulation_for

    wl = L.reduced(L.solutal_512(), 80, 70)
    _say("case nonfinite detection")
    sim = simulation_for(wl, storage="f32")
    sim.step(4)
    U = sim.read(0, ("U",))["U"].copy()
    U[30, 40] = np.nan
    sim.write(0, {"U": U})
    with pytest.raises(lbm.LBMError) as ei:
        sim.step(4, diag=True)
    assert ei.value.status == lbm.LBM_EUNSTABLE
    assert ei.value.diag[0]["nonfinite"] > 0
    assert ei.value.diag[0]["first_nonfinite_step"] == 8
    sim.close()


@pytest.mark.parametrize("case", ["direct", "graph", "batched", "3d"])
def test_nonfinite_state_is_reported_without_diagnostics(case):
    """Stepping without diagnostics still fails with LBM_EUNSTABLE: the
    device screens phi, U, T and rho after every replayed cycle and after
    the call's last step.  A NaN written into U after 8 steps is found at
    the first screen after it (the end of the call for direct steps, the
    end of the first replayed cycle otherwise), the right domain of a batch
    is named, and the first failing step stays reported afterwards."""
    from paper_2609_25670_amd import lbm, simulation_for

    if case == "3d":
        wl = L.reduced(L.directional_3d(), 64, 32, 48)
    elif case == "batched":
        wl = L.ensemble_256(n_domains=3, side_lo=40, side_hi=90)
    else:
        wl = L.reduced(L.solutal_512(), 80, 70)
    _say(f"case nonfinite detection without diagnostics: {case}")
    sim = simulation_for(wl, storage="f32")
    sim.configure(0 if case == "3d" else 8, case != "direct")
    sim.step(8)
    bad = sim.n - 1
    U = sim.read(bad, ("U",))["U"].copy()
    U[(slice(None),) * (U.ndim - 2) + (5, 7)] = np.nan
    sim.write(bad, {"U": U})
    n = 3 if case == "direct" else 4000
    with pytest.raises(lbm.LBMError) as ei:
        sim.step(n)
    assert ei.value.status == lbm.LBM_EUNSTABLE
    assert f"domain {bad}" in str(ei.value)
    with pytest.raises(lbm.LBMError) as ei2:
        sim.step(1, diag=True)
    first = ei2.value.diag[bad]["first_nonfinite_step"]
    _say(f"  first non-finite step {first}; message: {ei.value}")
    assert 8 < first <= 8 + n
    if case == "direct":
        assert first == 11
    for i in range(sim.n):
        if i != bad:
            assert ei2.value.diag[i]["first_nonfinite_step"] == -1
    sim.close()


def test_time_and_solute_drift_match_the_oracle():
    """t = k dt_base and R_M = [M_C(t) - M_C(0)]/M_C(0) (Section 4.4), with
    M_C(0) taken at the first step, against the oracle's total solute."""
    wl = L.reduced(L.solutal_512(), 96, 80)
    d = wl["domains"][0]
    _say("case t and R_M fp64 60 steps")
    (got,), diag = _gpu(wl, 60, names=("phi", "U"), tile_rows=8)
    dom0 = oracle.Domain(d)
    dom = oracle.run(d, 60)

    def total_C(o):
        kf = (1 + d["k"]) - (1 - d["k"]) * o.phi
        return float(np.sum(d["C_inf"] * kf * (1 + (1 - d["k"]) * o.U) / 2))

    m0, m1 = total_C(dom0), total_C(dom)
    r = (m1 - m0) / m0
    _say(f"  R_M gpu {diag[0]['R_M']:.6e} oracle {r:.6e}; t = {diag[0]['t']}")
    assert diag[0]["t"] == 60 * d["dt_base"]
    assert abs(diag[0]["R_M"] - r) <= 1e-12 * max(1.0, abs(r)) + 1e-15
    assert diag[0]["first_nonfinite_step"] == -1


@pytest.mark.parametrize("steps,tol", [(8, 1e-7), (40, 1e-7)])
def test_solutal_full_size_bench_configuration_fp32(steps, tol):
    """512 x 512 solutal case exactly as the benchmark launches it (FP32,
    autotuned tiles, deferred transfers, graph replay of the 16-step cycle)
    against the oracle on the full grid: 8 steps (direct launches) and 40
    (two graph replays, then 8 direct steps).  FP32 arithmetic and storage
    (unit roundoff 6e-8) keep the relative L2 near 1e-8 over these windows
    (3e-9 and 9e-9 measured for phi); the bar leaves a tenfold margin."""
    wl = L.solutal_512()
    names = ("phi", "U")
    _say(f"case solutal_512 full size fp32 {steps} steps")
    (got,), _ = _gpu(wl, steps, storage="f32", names=names)
    dom = oracle.run(wl["domains"][0], steps)
    for n in names:
        e = _rel(got[n], getattr(dom, n))
        _say(f"  solutal_512: {n} rel L2 = {e:.3e}")
        assert e < tol, (n, e)
