#!/usr/bin/env python
"""Throughput of the multirate coupled-field step on one MI355X.

A bench "step" is one multirate cycle: lcm(N_chi) base steps, in which every
kernel of the hot path (phase collision + anisotropic streaming, phase-step
transfer, each scalar transport, flow) runs at least once.  The default
workload is the largest single-GPU configuration: 3D directional
solidification on 256 x 256 x 512 (33.5 M sites; D3Q7 phase, U, T and D3Q19
flow, N_phi : N_U : N_T : N_F = 1 : 1 : 16 : 4), FP32 arithmetic with BF16
population storage.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  Each of the K steps is timed on its own (wall clock
between device synchronisations); ``value`` is coupled-field MLUPS
(sites x base steps / time) of the median step, ``ms_per_step`` that
median.  With ``--window W`` the library is called once per W steps and
each step's time is its call's over W (for workloads whose step is as short
as the synchronisation at the end of every call).  ``roofline`` describes the kernel with the largest share of device
time per base step: its algorithmic bytes per launch divided by its average
launch time, measured with HIP events on the stream the library issues its
work on; ``step_roofline`` does the same for the whole step (algorithmic
bytes of every kernel of the cycle over the median step time).
``cpu_baseline`` times the FP64 oracle on a bounded sample of the same
workload: one process, then one process per host core in parallel (each on
its own copy of the sample).  The line also carries
``batched_workload``: the same measurement on the 256-domain ensemble
(29.7 M sites of uneven 2D domains, FP16 storage).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("coupled-field MLUPS + % HBM peak; FP32/FP16-store vs FP64 at stated tip-velocity error")
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "directional_3d"
SIDE_WORKLOAD = "ensemble_256"
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2609_25670_amd", "csrc", f)
                  for f in ("lbm_kernels.hip", "lbm_dev.h")]
KERNEL_NAMES = {"phase": "k_phase", "phase_tr": "k_phase_tr", "transfer": "k_transfer", "U": "k_scalar<..., 0>",
                "T": "k_scalar<..., 1>", "flow": "k_flow", "phase_dtr": "k_dtr_phase", "U_dtr": "k_dtr_scalar"}
KERNEL_NAMES_MARCH = dict(KERNEL_NAMES, phase="k_phase_ym", transfer="k_transfer_ym", U="k_scalar_ym<..., 0>",
                          T="k_scalar_ym<..., 1>", T_tr="k_tr_scalar_ym")
KERNEL_NAMES_3D = {"phase": "k3z_phase", "transfer": "k3z_transfer", "U": "k3z_scalar<..., 0>",
                   "T": "k3z_scalar<..., 1>", "flow": "k3z_flow"}


def sites_of(d: dict) -> int:
    return d["nx"] * d["ny"] * (d["nz"] if d["dim"] == 3 else 1)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kind: str, d: dict, storage: str) -> int:
    """Compulsory HBM bytes per site of one launch of a kernel kind: every
    plane the kernel must read once and write once for the representation
    it keeps (stencil and halo re-reads excluded)."""
    s = STORAGE_BYTES[storage]
    r = 8 if storage == "f64" else 4
    U, T, F = int(d["has_U"]), int(d["has_T"]), int(d["has_flow"])
    acc = d.get("coupling", "instant") == "accum"
    dim = d["dim"]
    qs = d.get("q_scalar", 5) if dim == 2 else 7   # scalar lattice
    qf = 9 if dim == 2 else 19           # flow lattice
    if kind == "phase":      # s_1..s_{Q-1} in/out, phi in/out, U*, T*
        return 2 * (qs - 1) * s + (2 + U + T) * r
    if kind == "phase_tr":   # phase with its transfer in one kernel: the phase
        # kernel's bytes plus the new U and T planes (or the pending planes)
        return 2 * (qs - 1) * s + (2 + U + T) * r + (2 if acc else 1) * (U + T) * r
    if kind == "phase_dtr":  # phase kernel carrying the previous step's transfer: phi^{q-1}, phi^q, U, T,
        # s in; U, T, phi^{q+1}, s out
        return 2 * (qs - 1) * s + (3 + 2 * U + 2 * T) * r
    if kind == "U_dtr":      # U transport carrying its step's transfer: phi^q, phi^{q+1}, U, j_U, [u],
        # T in; U, j_U, T out (the transferred U stays on chip; j_U is stored at the compute precision)
        Tl = T if d.get("T_mode", "transport") != "pulled" else 0
        return (4 + dim * F + 2 * Tl) * r + 2 * dim * r
    if kind == "T_tr":       # T transport carrying its step's transfer: phi^q, phi^{q+1}, U, T, j_T, [u] in;
        # U*, T, j_T out (the transferred T stays on chip)
        return (4 + 2 * U + dim * F) * r + 2 * dim * s
    if kind == "transfer":   # phi^q, phi^{q+1}; U in, U out (or pending), T in, T out (not a pulled T)
        Tl = T if d.get("T_mode", "transport") != "pulled" else 0
        return (2 + 2 * U + 2 * Tl) * r
    if kind == "U":          # U, j_U, phi*, [u]; U, j_U out; [pending] (j_U at the compute precision)
        return (3 + dim * F + 2 * acc) * r + 2 * dim * r
    if kind == "T":          # as U; phi* only with phi-dependent properties
        tvar = d["kappa_S"] != d["kappa_L"] or d["rhoCp_S"] != d["rhoCp_L"]
        return (2 + int(tvar) + dim * F + 2 * acc) * r + 2 * dim * s
    if kind == "flow":       # rho, s_1..s_{QF-1}, phi* in; rho, s_1..s_{QF-1}, u out
        return (3 + dim) * r + 2 * (qf - 1) * s
    raise ValueError(kind)


def cycle_of(wl: dict) -> int:
    L = 1
    for d in wl["domains"]:
        for key, flag in (("N_phi", True), ("N_U", d["has_U"]), ("N_T", d["has_T"]), ("N_F", d["has_flow"])):
            if flag:
                L = L * d[key] // math.gcd(L, d[key])
    return L


def counters_key(kernel: str) -> str:
    """File key of a kernel's counter summary: its name, and for the scalar
    transports the field (template argument 0: U, 1: T), whether given in
    full (``lbm::k3z_scalar<float, float, 0, 8>``) or short
    (``k3z_scalar<..., 0>``)."""
    base = kernel.split("<")[0].split("::")[-1]
    if base in ("k_scalar", "k_scalar_ym", "k_scalar_ym_q", "k3z_scalar") and "<" in kernel:
        args = [a.strip() for a in kernel.split("<", 1)[1].rstrip(">").split(",")]
        field = args[2] if len(args) >= 3 and args[1] != "..." else args[-1]
        base += "_U" if field == "0" else "_T"
    return base


def traffic_from_profiles(workload: str, kernel: str, sha: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"counters_{counters_key(kernel)}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != sha:
        return None
    return rec.get("hbm_bytes_per_dispatch")


def host_cpus() -> int:
    """Cores this process may run on (its affinity set)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(workload: str, steps: int, procs: int) -> dict:
    """Time the FP64 oracle for ``steps`` base steps of the workload's
    bounded sample in ``procs`` child processes at once, each pinned to one
    BLAS/OpenMP thread and running its own copy; returns the aggregate
    MLUPS and the slowest child's record."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--workload", workload,
           "--cpu-steps", str(steps)]
    kids = [subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, text=True) for _ in range(procs)]
    recs = []
    for p in kids:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle child failed with status {p.returncode}")
        recs.append(json.loads(out.strip().splitlines()[-1]))
    slow = max(recs, key=lambda r: r["seconds"])
    return dict(slow, mlups=sum(r["sites"] * r["steps"] for r in recs) / slow["seconds"] / 1e6, procs=procs)


def cpu_child(workload: str, steps: int) -> None:
    import lbm_inputs as L
    import oracle

    wl = L.workload(workload)
    d0 = wl["domains"][0]
    if d0["dim"] == 3:       # bounded sample: the reduced 3D grid
        d0 = L.reduced(wl, 64, 64, 128)["domains"][0]
    elif d0["nx"] * d0["ny"] > 512 * 512:   # bounded sample: a 512 x 512 grid
        d0 = L.reduced(wl, 512, 512)["domains"][0]
    sites = sites_of(d0)
    dom = oracle.Domain(d0)
    t0 = time.perf_counter()
    for _ in range(steps):
        dom.step()
    dt = time.perf_counter() - t0
    grid = "x".join(str(d0[k]) for k in (("nx", "ny", "nz") if d0["dim"] == 3 else ("nx", "ny")))
    print(json.dumps(dict(seconds=dt, steps=steps, sites=sites, grid=grid, mlups=sites * steps / dt / 1e6)))


def measure(sim, wl: dict, storage: str, steps: int, warmup: int, window: int = 1) -> dict:
    """Time ``steps`` multirate cycles after ``warmup`` cycles, ``window``
    cycles per library call (wall clock between device synchronisations,
    and HIP events on the library's stream; every call synchronises at its
    end, which on small workloads costs as much as a cycle), then time each
    kernel kind with HIP events.  Closes ``sim``."""
    import torch

    cyc = cycle_of(wl)
    sites = sum(sites_of(d) for d in wl["domains"])
    # warm-up: autotune, graph capture, clocks
    sim.step(warmup * cyc)
    torch.cuda.synchronize()
    walls, evs = [], []
    t_all = time.perf_counter()
    for _ in range(max(1, steps // window)):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        sim.step(window * cyc)   # synchronises at its end (non-finite screen)
        ev1.record()
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) / window)
        evs.append(ev0.elapsed_time(ev1) / window)
    total = time.perf_counter() - t_all
    diag = sim.step(0, diag=True)
    finite = all(dd["nonfinite"] == 0 and dd["first_nonfinite_step"] < 0 for dd in diag)
    med = sorted(walls)[len(walls) // 2]
    mlups = sites * cyc / med / 1e6

    # per-kernel launch times (HIP events on the library's stream)
    marching = sim.marching
    kt = sim.kernel_times(reps=200)
    rows = sim.tile_rows
    sim.close()
    d0 = wl["domains"][0]
    if d0["dim"] == 2 and "phase" in kt and "transfer" not in kt:   # the transfer runs inside the phase kernel
        kt = {("phase_tr" if k == "phase" else k): v for k, v in kt.items()}
    per_kind = {}
    for kind, (ms, per) in kt.items():
        nbytes = sum(algorithmic_bytes(kind, d, storage) * sites_of(d) for d in wl["domains"])
        per_kind[kind] = dict(ms_per_launch=ms, launches_per_base_step=per,
                              alg_bytes_per_launch=nbytes,
                              alg_GBs=nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None,
                              share_ms_per_base_step=ms * per)
    dom_kind = max(per_kind, key=lambda k: per_kind[k]["share_ms_per_base_step"])
    names = KERNEL_NAMES_3D if d0["dim"] == 3 else KERNEL_NAMES_MARCH if marching else KERNEL_NAMES
    step_bytes = sum(v["alg_bytes_per_launch"] * v["launches_per_base_step"] for v in per_kind.values()) * cyc
    return dict(mlups=mlups, med_s=med, mean_s=total / (len(walls) * window), walls_ms=[round(w * 1e3, 4) for w in walls],
                event_ms=[round(e, 4) for e in evs], finite=finite, kernels=per_kind, dominant=dom_kind,
                names=names, tile_rows=rows, step_bytes=step_bytes)


def roofline_of(m: dict, workload: str, sha: str) -> dict:
    dk = m["kernels"][m["dominant"]]
    name = m["names"][m["dominant"]]
    return {"bound": "hbm", "kernel": name, "achieved": round(dk["alg_GBs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(dk["alg_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(workload, name, sha)}


def step_roofline_of(m: dict) -> dict:
    gbs = m["step_bytes"] / m["med_s"] / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_step": m["step_bytes"]}


def directional_run(args) -> int:
    """The long runs of Section 4.4 (2D directional saline solidification,
    1000 x 1000, Table 1 set, N_U = Le): every Lewis number of ``--le``
    (comma-separated) is one domain of a single batched context.  Steps to
    ``--t-end-ms`` (dt_base = 2e-9 s, so 20 ms = 1e7 base steps) and prints
    one JSON line per domain every ``--every-ms`` with the time, S_phi, J_U,
    R_M, the range of phi and of U (read back), then a summary line per
    domain.
    A domain whose state turns non-finite is reported with the step at which
    the device screen found it, and the run stops there."""
    import lbm_inputs as L
    from paper_2609_25670_amd import lbm, simulation_for

    les = [int(v) for v in str(args.le).split(",")]
    doms = []
    for le in les:
        d = L.directional_2d(Le=le, coupling=args.coupling)["domains"][0]
        d["q_scalar"] = args.q_scalar
        doms.append(d)
    storage = args.storage or "f32"
    steps_per_ms = int(round(1e-3 / 2e-9))
    every = max(1, int(round(args.every_ms * steps_per_ms)))
    total = int(round(args.t_end_ms * steps_per_ms))
    sim = simulation_for(dict(domains=doms), storage=storage)
    head = dict(run="directional_2d", Le=les, coupling=args.coupling, q_scalar=args.q_scalar,
                storage=storage, t_end_ms=args.t_end_ms, every_steps=every)
    print(json.dumps(head), flush=True)
    done, t0 = 0, time.perf_counter()
    first_bad = [-1] * len(les)
    peak = [dict(S_phi=0.0, J_U=0.0, phi=-1.0) for _ in les]
    last = [None] * len(les)
    stop = False
    while done < total and not stop:
        n = min(every, total - done)
        try:
            dd = sim.step(n, diag=True)
        except lbm.LBMError as e:
            if e.status != lbm.LBM_EUNSTABLE:
                raise
            dd = e.diag
            stop = True
        done += n
        for i, le in enumerate(les):
            x = dd[i]
            fld = sim.read(i, ("phi", "U"))
            phimax = float(np.max(fld["phi"]))
            first_bad[i] = x["first_nonfinite_step"]
            pk = peak[i]
            pk["S_phi"], pk["J_U"] = max(pk["S_phi"], x["S_phi"]), max(pk["J_U"], x["J_U"])
            pk["phi"] = max(pk["phi"], phimax) if np.isfinite(phimax) else phimax
            last[i] = dict(Le=le, step=x["step"], t_ms=x["step"] / steps_per_ms, S_phi=x["S_phi"], J_U=x["J_U"],
                           R_M=x["R_M"], phi_max=phimax, phi_min=float(np.min(fld["phi"])),
                           U_min=float(np.min(fld["U"])), U_max=float(np.max(fld["U"])), nonfinite=x["nonfinite"],
                           wall_s=round(time.perf_counter() - t0, 1))
            print(json.dumps(last[i]), flush=True)
    sim.close()
    for i, le in enumerate(les):
        fb = first_bad[i]
        print(json.dumps(dict(head, Le=le, summary=True, steps=done, final=last[i], max_S_phi=peak[i]["S_phi"],
                              max_J_U=peak[i]["J_U"], max_phi=peak[i]["phi"], first_nonfinite_step=fb,
                              first_nonfinite_ms=(fb / steps_per_ms if fb >= 0 else None))), flush=True)
    return 0


def directional3d_run(args) -> int:
    """A long run of the 3D directional workload (256 x 256 x 512, the
    storage of ``--storage``, BF16 by default) for ``--run-steps`` base
    steps: one JSON line every ``--every-steps`` with R_M, the largest and
    the mean front height, S_phi and the wall time, then a summary line."""
    import lbm_inputs as L
    from paper_2609_25670_amd import lbm, simulation_for

    wl = L.directional_3d()
    storage = args.storage or wl["storage"]
    sim = simulation_for(wl, storage=storage)
    head = dict(run="directional_3d", storage=storage, steps=args.run_steps, every_steps=args.every_steps)
    print(json.dumps(head), flush=True)
    done, t0, last, bad = 0, time.perf_counter(), None, -1
    while done < args.run_steps:
        n = min(args.every_steps, args.run_steps - done)
        try:
            x = sim.step(n, diag=True)[0]
        except lbm.LBMError as e:
            if e.status != lbm.LBM_EUNSTABLE:
                raise
            x = e.diag[0]
            bad = x["first_nonfinite_step"]
            done += n
            break
        done += n
        last = dict(step=x["step"], R_M=x["R_M"], front_max=x["tip"][0], front_mean=x["tip"][1],
                    S_phi=x["S_phi"], nonfinite=x["nonfinite"], wall_s=round(time.perf_counter() - t0, 1))
        print(json.dumps(last), flush=True)
    sim.close()
    print(json.dumps(dict(head, summary=True, final=last, first_nonfinite_step=bad)), flush=True)
    return 0 if bad < 0 else 1


def _progress(msg: str) -> None:
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-side-line", action="store_true",
                    help="skip the measurement of the batched ensemble beside the default workload")
    ap.add_argument("--storage", default=None, help="override the workload's population storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=32)
    ap.add_argument("--cpu-procs", type=int, default=16, help="at most this many oracle processes at once")
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    ap.add_argument("--profile-steps", type=int, default=0, metavar="N",
                    help="only run N warm-up and N measured base steps (for profiler runs); no JSON")
    ap.add_argument("--tile-rows", type=int, default=0, help="fix the tile height (0 = autotune)")
    ap.add_argument("--window", type=int, default=1, metavar="W",
                    help="steps per library call in the timed region (each call synchronises at its end); "
                         "the per-step times are the call times over W")
    ap.add_argument("--run", choices=["directional_2d", "directional_3d"], default=None,
                    help="instead of the benchmark: a long run of the Section 4.4 case (see directional_run) "
                         "or of the 3D directional workload (see directional3d_run)")
    ap.add_argument("--run-steps", type=int, default=20000, help="base steps of --run directional_3d")
    ap.add_argument("--every-steps", type=int, default=2000, help="report interval of --run directional_3d")
    ap.add_argument("--le", default="1", help="Lewis numbers of --run, comma-separated (N_U = Le)")
    ap.add_argument("--coupling", choices=["instant", "accum"], default="instant")
    ap.add_argument("--q-scalar", type=int, default=5, help="scalar lattice of --run: 5 (D2Q5) or 9 (D2Q9)")
    ap.add_argument("--t-end-ms", type=float, default=20.0)
    ap.add_argument("--every-ms", type=float, default=0.5)
    args = ap.parse_args()
    if args.run == "directional_3d":
        return directional3d_run(args)
    if args.run:
        return directional_run(args)

    if args.cpu_child:
        cpu_child(args.workload, args.cpu_steps)
        return 0
    if args.copy_probe:
        import torch

        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps(dict(copy_probe_bytes=n * 4, reps=13, ms_per_copy=ms,
                              read_plus_write_GBs=2 * n * 4 / (ms * 1e-3) / 1e9)), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "a multi-GPU run is not part of it", file=sys.stderr)
        return 2
    rank = int(os.environ.get("RANK", "0"))

    import torch

    import lbm_inputs as L
    from paper_2609_25670_amd import simulation_for

    wl = L.workload(args.workload)
    storage = args.storage or wl["storage"]
    cyc = cycle_of(wl)
    sites = sum(sites_of(d) for d in wl["domains"])
    sim = simulation_for(wl, storage=storage)
    if args.tile_rows:
        sim.configure(args.tile_rows, True)
    if args.profile_steps:
        sim.step(args.profile_steps)
        torch.cuda.synchronize()
        sim.step(args.profile_steps)
        torch.cuda.synchronize()
        sim.close()
        print(json.dumps(dict(profile_steps=args.profile_steps, workload=wl["name"], storage=storage)), flush=True)
        return 0
    m = measure(sim, wl, storage, args.steps, args.warmup, args.window)
    _progress(f"measured {wl['name']}: {m['mlups']:.0f} MLUPS")
    finite = m["finite"]
    d0 = wl["domains"][0]
    sha = kernel_source_sha()
    bytes_per_base_step = m["step_bytes"] / cyc / sites   # per site

    result = {
        "metric": METRIC,
        "value": round(m["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": len(m["walls_ms"]) * args.window,
        "warmup": args.warmup,
        "ms_per_step": m["med_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if storage == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": wl["name"],
            "grid": ([d0["nx"], d0["ny"]] + ([d0["nz"]] if d0["dim"] == 3 else [])
                     if len(wl["domains"]) == 1 else f"{len(wl['domains'])} domains"),
            "sites": sites,
            "fields": "+".join(["phi"] + [f for f, k in (("U", "has_U"), ("T", "has_T"), ("flow", "has_flow"))
                                          if d0[k]]),
            "update_factors": {k: d0[k] for k in ("N_phi", "N_U", "N_T", "N_F")},
            "storage": storage,
            "base_steps_per_step": cyc,
            "tile_rows": m["tile_rows"],
            "parallelism": "single_gpu",
        },
        "roofline": roofline_of(m, args.workload, sha),
        "step_roofline": step_roofline_of(m),
        "timing": {"median_of": len(m["walls_ms"]), "steps_per_call": args.window,
                   "ms_per_step_mean": round(m["mean_s"] * 1e3, 4),
                   "wall_ms": m["walls_ms"], "event_ms": m["event_ms"]},
        "kernels": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in m["kernels"].items()},
        "alg_bytes_per_site_per_base_step": round(bytes_per_base_step, 3),
        "finite": finite,
    }
    if args.workload == DEFAULT_WORKLOAD and not args.no_side_line:
        # the batched ensemble of uneven 2D domains, measured the same way
        hw = L.workload(SIDE_WORKLOAD)
        hsim = simulation_for(hw, storage=hw["storage"])
        hm = measure(hsim, hw, hw["storage"], 3, 1)
        _progress(f"measured {hw['name']}: {hm['mlups']:.0f} MLUPS")
        finite = finite and hm["finite"]
        result["batched_workload"] = {
            "workload": hw["name"],
            "sites": sum(sites_of(d) for d in hw["domains"]),
            "storage": hw["storage"],
            "value": round(hm["mlups"], 2),
            "unit": "MLUPS",
            "steps": 3,
            "ms_per_step": round(hm["med_s"] * 1e3, 4),
            "base_steps_per_step": cycle_of(hw),
            "tile_rows": hm["tile_rows"],
            "roofline": roofline_of(hm, SIDE_WORKLOAD, sha),
            "step_roofline": step_roofline_of(hm),
            "kernels": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k, v in hm["kernels"].items()},
        }
        result["finite"] = finite
    if rank == 0 and not args.no_cpu_baseline:
        ncpu = host_cpus()
        procs = max(1, min(ncpu, args.cpu_procs))
        one = cpu_baseline(args.workload, args.cpu_steps, 1)
        _progress(f"cpu baseline, one process: {one['mlups']:.2f} MLUPS")
        allc = cpu_baseline(args.workload, args.cpu_steps, procs)
        _progress(f"cpu baseline, {procs} processes: {allc['mlups']:.2f} MLUPS")
        result["cpu_baseline"] = {
            "value": round(allc["mlups"], 4),
            "unit": "MLUPS",
            "cores": procs,
            "kind": "oracle",
            "sample": (f"FP64 NumPy oracle on the bounded sample {allc['grid']} of {wl['name']} "
                       f"({allc['sites']} sites), {allc['steps']} base steps per process, {procs} processes at "
                       f"once, one thread each ({allc['seconds']:.1f} s); CPU {cpu_model()}, "
                       f"{ncpu} cores available"),
            "single_core": {"value": round(one["mlups"], 4), "unit": "MLUPS", "cores": 1,
                            "seconds": round(one["seconds"], 2)},
            "cpu_model": cpu_model(),
            "nproc": ncpu,
        }
    if rank == 0:
        print(json.dumps(result), flush=True)
    return 0 if finite else 1


if __name__ == "__main__":
    sys.exit(main())
