"""Thin ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies the device workspace and the HIP stream.
The binding refuses to run if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_EUNSTABLE",
          -5: "LBM_ESTATE"}

(F_PHI, F_U, F_T, F_RHO, F_VEL, F_POP_PHI, F_JU, F_JT, F_POP_F, F_PEND_U, F_PEND_T, F_SPHI,
 F_SF, F_SU, F_ST) = (1 << i for i in range(15))
BC = {"periodic": 0, "wall": 1, "inlet_outflow": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
COUPLING = {"instant": 0, "accum": 1}
T_MODE = {"transport": 0, "pulled": 1, "dirichlet_low": 2}
GRAD_PHI = {"fd": 0, "eq40": 1}

# names, plane counts per field bit (2D)
FIELD_BITS = [("phi", F_PHI, 1), ("U", F_U, 1), ("T", F_T, 1), ("rho", F_RHO, 1), ("vel", F_VEL, 2),
              ("f_phi", F_POP_PHI, 5), ("jU", F_JU, 2), ("jT", F_JT, 2), ("f_F", F_POP_F, 9),
              ("P_U", F_PEND_U, 1), ("P_T", F_PEND_T, 1), ("s_phi", F_SPHI, 4), ("s_F", F_SF, 8),
              ("s_U", F_SU, 1), ("s_T", F_ST, 1)]

EXPORTS = ["lbm_workspace_bytes", "lbm_create", "lbm_init_seeds", "lbm_init_front", "lbm_step_multirate",
           "lbm_step_multirate_static", "lbm_read_fields",
           "lbm_write_fields", "lbm_configure", "lbm_kernel_times", "lbm_steps_done", "lbm_marching",
           "lbm_tile_rows", "lbm_last_error", "lbm_destroy"]
KERNEL_KINDS = ("phase", "transfer", "U", "T", "flow", "phase_dtr", "U_dtr", "T_tr")


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("q_scalar", ctypes.c_int32), ("has_U", ctypes.c_int32), ("has_T", ctypes.c_int32),
        ("has_flow", ctypes.c_int32), ("N_phi", ctypes.c_int32), ("N_U", ctypes.c_int32),
        ("N_T", ctypes.c_int32), ("N_F", ctypes.c_int32), ("dt_base", ctypes.c_double),
        ("W0", ctypes.c_double), ("tau0", ctypes.c_double), ("eps_s", ctypes.c_double),
        ("lam", ctypes.c_double), ("Mc", ctypes.c_double), ("k", ctypes.c_double),
        ("theta_c", ctypes.c_double), ("D_L", ctypes.c_double), ("D_S", ctypes.c_double),
        ("C_inf", ctypes.c_double), ("kappa_S", ctypes.c_double), ("kappa_L", ctypes.c_double),
        ("rhoCp_S", ctypes.c_double), ("rhoCp_L", ctypes.c_double), ("rho_L", ctypes.c_double),
        ("L_h", ctypes.c_double), ("T_m", ctypes.c_double), ("m_L", ctypes.c_double),
        ("Cp_L", ctypes.c_double), ("nu", ctypes.c_double), ("s_e", ctypes.c_double),
        ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double), ("u_in", ctypes.c_double),
        ("Fb", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 3), ("flow_bc", ctypes.c_int32 * 3),
        ("U0", ctypes.c_double), ("T0", ctypes.c_double), ("u0_liquid_only", ctypes.c_int32),
        ("coupling", ctypes.c_int32), ("T_mode", ctypes.c_int32), ("grad_phi", ctypes.c_int32),
        ("T_grad", ctypes.c_double), ("V_pull", ctypes.c_double), ("z_front", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("solid", ctypes.c_double), ("M_C", ctypes.c_double),
        ("enthalpy", ctypes.c_double), ("mass", ctypes.c_double), ("S_phi", ctypes.c_double),
        ("J_U", ctypes.c_double), ("tip", ctypes.c_double * 16), ("nonfinite", ctypes.c_int64),
        ("t", ctypes.c_double), ("R_M", ctypes.c_double), ("first_nonfinite_step", ctypes.c_int64),
    ]


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load liblbm.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_25670_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.lbm_workspace_bytes.restype = ctypes.c_size_t
    lib.lbm_workspace_bytes.argtypes = [P(Params), ctypes.c_int32, ctypes.c_int32]
    lib.lbm_create.restype = ctypes.c_int
    lib.lbm_create.argtypes = [P(Params), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_size_t, P(ctypes.c_void_p)]
    lib.lbm_init_seeds.restype = ctypes.c_int
    lib.lbm_init_seeds.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double),
                                   P(ctypes.c_double)]
    lib.lbm_init_front.restype = ctypes.c_int
    lib.lbm_init_front.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_double)]
    lib.lbm_step_multirate.restype = ctypes.c_int
    lib.lbm_step_multirate.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.lbm_step_multirate_static.restype = ctypes.c_int
    lib.lbm_step_multirate_static.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.lbm_read_fields.restype = ctypes.c_int
    lib.lbm_read_fields.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_void_p]
    lib.lbm_write_fields.restype = ctypes.c_int
    lib.lbm_write_fields.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32,
                                     ctypes.c_void_p]
    lib.lbm_configure.restype = ctypes.c_int
    lib.lbm_configure.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    lib.lbm_kernel_times.restype = ctypes.c_int
    lib.lbm_kernel_times.argtypes = [ctypes.c_void_p, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double)]
    lib.lbm_steps_done.restype = ctypes.c_int64
    lib.lbm_steps_done.argtypes = [ctypes.c_void_p]
    lib.lbm_marching.restype = ctypes.c_int32
    lib.lbm_marching.argtypes = [ctypes.c_void_p]
    lib.lbm_tile_rows.restype = ctypes.c_int32
    lib.lbm_tile_rows.argtypes = [ctypes.c_void_p]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = [ctypes.c_void_p]
    lib.lbm_destroy.restype = None
    lib.lbm_destroy.argtypes = [ctypes.c_void_p]
    _lib = lib
    return lib


def to_params(d: dict) -> Params:
    """Marshal one domain dict of ``lbm_inputs`` into the C struct."""
    p = Params()
    p.dim = int(d["dim"])
    p.nx, p.ny, p.nz = int(d["nx"]), int(d["ny"]), int(d.get("nz", 1))
    p.q_scalar = int(d["q_scalar"])
    p.has_U, p.has_T, p.has_flow = int(d["has_U"]), int(d["has_T"]), int(d["has_flow"])
    p.N_phi, p.N_U, p.N_T, p.N_F = int(d["N_phi"]), int(d["N_U"]), int(d["N_T"]), int(d["N_F"])
    for key in ("dt_base", "W0", "tau0", "eps_s", "lam", "Mc", "k", "theta_c", "D_L", "D_S", "C_inf",
                "kappa_S", "kappa_L", "rhoCp_S", "rhoCp_L", "rho_L", "L_h", "T_m", "m_L", "Cp_L", "nu",
                "s_e", "s_eps", "s_q", "u_in", "U0", "T0"):
        setattr(p, key, float(d[key]))
    for a in range(3):
        p.Fb[a] = float(d["Fb"][a])
        p.bc[a] = BC[d["bc"][a]]
        p.flow_bc[a] = BC[d["flow_bc"][a]]
    p.u0_liquid_only = int(bool(d.get("u0_liquid_only", False)))
    p.coupling = COUPLING[d.get("coupling", "instant")]
    p.T_mode = T_MODE[d.get("T_mode", "transport")]
    p.grad_phi = GRAD_PHI[d.get("grad_phi", "fd")]
    p.T_grad = float(d.get("T_grad", 0.0))
    p.V_pull = float(d.get("V_pull", 0.0))
    p.z_front = float(d.get("z_front", 0.0))
    return p


def _check(lib, ctx, status):
    if status != LBM_OK:
        msg = lib.lbm_last_error(ctx)
        raise LBMError(status, msg.decode() if msg else "")


class Simulation:
    """One context of ``n`` domains stepped together.

    ``domains``  list of domain dicts (``lbm_inputs`` format)
    ``storage``  "f64" (FP64 everywhere) | "f32" | "f16" | "bf16" population storage
    ``workspace``  "torch" (a torch uint8 CUDA tensor) or "library" (hipMalloc)
    """

    def __init__(self, domains, storage="f64", device=0, workspace="torch", stream=None):
        import torch  # device memory and streams only

        self.lib = load()
        self.domains = [dict(d) for d in domains]
        self.n = len(self.domains)
        arr = (Params * self.n)(*[to_params(d) for d in self.domains])
        self._params = arr
        st = STORAGE[storage]
        self.storage = storage
        self.device = device
        nbytes = self.lib.lbm_workspace_bytes(arr, self.n, st)
        if nbytes == 0:
            raise LBMError(LBM_EINVAL, "invalid parameters (lbm_workspace_bytes returned 0)")
        self.workspace_bytes = nbytes
        self._ws = None
        ws_ptr = None
        if workspace == "torch":
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
            ws_ptr = self._ws.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        ctx = ctypes.c_void_p()
        s = self.lib.lbm_create(arr, self.n, st, device, ctypes.c_void_p(stream.cuda_stream),
                                ctypes.c_void_p(ws_ptr) if ws_ptr else None, nbytes, ctypes.byref(ctx))
        _check(self.lib, None, s)
        self.ctx = ctx

    # ----------------------------------------------------------------- calls
    def init(self):
        for i, d in enumerate(self.domains):
            if d["dim"] == 3 or "perturb" in d:
                xi = d.get("perturb")
                buf = None
                if xi is not None:
                    xi = np.asarray(xi, dtype=np.float64)
                    a = np.ascontiguousarray(xi[: d["ny"], : d["nx"]] if d["dim"] == 3 else xi[: d["nx"]])
                    buf = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                    self._xi = a
                _check(self.lib, self.ctx, self.lib.lbm_init_front(self.ctx, i, buf))
                continue
            seeds = d.get("seeds", [])
            c = (ctypes.c_double * max(1, 2 * len(seeds)))(*[v for s in seeds for v in s[:2]])
            r = (ctypes.c_double * max(1, len(seeds)))(*[s[2] for s in seeds])
            _check(self.lib, self.ctx, self.lib.lbm_init_seeds(self.ctx, i, len(seeds), c, r))

    def configure(self, tile_rows=0, use_graph=True, fuse_transfer=False, march=None, defer=True, queue=None):
        """Tile height (0 = autotune), HIP-graph replay of whole cycles,
        whether the 2D transfer runs inside the phase kernel, whether the 2D
        phase, transfer and T-transport kernels march up 64-wide columns
        (True), tile (False) or choose by size (None), whether a transfer
        may be deferred into the next phase kernel, and whether the marching
        kernels take their runs from per-XCD work queues (True), run one
        block per run (False) or let the autotuner pick (None)."""
        flags = (1 if use_graph else 0) | (2 if fuse_transfer else 0) | (0 if defer else 16)
        flags |= {None: 0, True: 4, False: 8}[march]
        flags |= {None: 0, True: 32, False: 64}[queue]
        _check(self.lib, self.ctx, self.lib.lbm_configure(self.ctx, int(tile_rows), flags))

    def step(self, n, diag=False, static=False):
        """Advance every domain by n base steps (synchronises).  With
        ``diag`` returns a list of per-domain diagnostic dicts.  Raises
        LBMError with status LBM_EUNSTABLE once non-finite values are
        found, with or without ``diag``.  ``static`` calls the entry point
        that allocates nothing (lbm_step_multirate_static)."""
        fn = self.lib.lbm_step_multirate_static if static else self.lib.lbm_step_multirate
        if not diag:
            _check(self.lib, self.ctx, fn(self.ctx, int(n), None))
            return None
        out = (Diag * self.n)()
        s = fn(self.ctx, int(n), out)
        res = [dict(step=o.step, solid=o.solid, M_C=o.M_C, enthalpy=o.enthalpy, mass=o.mass, S_phi=o.S_phi,
                    J_U=o.J_U, tip=list(o.tip), nonfinite=o.nonfinite, t=o.t, R_M=o.R_M,
                    first_nonfinite_step=o.first_nonfinite_step) for o in out]
        if s == LBM_EUNSTABLE:
            err = LBMError(s, self.lib.lbm_last_error(self.ctx).decode())
            err.diag = res
            raise err
        _check(self.lib, self.ctx, s)
        return res

    def kernel_times(self, reps=200):
        """Per-kind average launch time (ms) and launches per base step.
        Leaves the state undefined (call ``init`` before stepping again)."""
        ms = (ctypes.c_double * 8)()
        per = (ctypes.c_double * 8)()
        _check(self.lib, self.ctx, self.lib.lbm_kernel_times(self.ctx, int(reps), ms, per))
        return {k: (ms[i], per[i]) for i, k in enumerate(KERNEL_KINDS) if ms[i] >= 0}

    @property
    def steps_done(self) -> int:
        return int(self.lib.lbm_steps_done(self.ctx))

    @property
    def marching(self) -> bool:
        """Whether the 2D phase, transfer and T-transport kernels march."""
        return self.lib.lbm_marching(self.ctx) == 1

    @property
    def tile_rows(self) -> int:
        """Tile height of the 2D tiled kernels in use (0 before the
        autotuner has run); in 3D the rows fixed by ``configure`` (0: the
        per-kernel defaults)."""
        return int(self.lib.lbm_tile_rows(self.ctx))

    def _layout(self, names, domain=0):
        d = self.domains[domain]
        dim = d["dim"]
        cnts = dict(vel=dim, jU=dim, jT=dim, f_phi=d["q_scalar"], s_phi=d["q_scalar"] - 1,
                    f_F=9 if dim == 2 else 19, s_F=8 if dim == 2 else 18)
        mask = 0
        order = []
        for name, bit, cnt in FIELD_BITS:
            if name in names:
                mask |= bit
                order.append((name, cnts.get(name, cnt)))
        return mask, order

    def _shape(self, domain):
        d = self.domains[domain]
        return (d["ny"], d["nx"]) if d["dim"] == 2 else (d["nz"], d["ny"], d["nx"])

    def read(self, domain=0, names=("phi",), fp64=True, device=False):
        """Dict name -> array [planes..., ny, nx] (planes squeezed when 1).
        Host numpy arrays by default; torch CUDA tensors with ``device``."""
        import torch

        shape = self._shape(domain)
        mask, order = self._layout(names, domain)
        nplanes = sum(c for _, c in order)
        if device:
            buf = torch.empty((nplanes,) + shape, dtype=torch.float64 if fp64 else torch.float32,
                              device=f"cuda:{self.device}")
            _check(self.lib, self.ctx, self.lib.lbm_read_fields(self.ctx, domain, mask, 1, int(fp64),
                                                                ctypes.c_void_p(buf.data_ptr())))
        else:
            buf = np.empty((nplanes,) + shape, dtype=np.float64 if fp64 else np.float32)
            _check(self.lib, self.ctx, self.lib.lbm_read_fields(self.ctx, domain, mask, 0, int(fp64),
                                                                buf.ctypes.data_as(ctypes.c_void_p)))
        out = {}
        i = 0
        for name, cnt in order:
            out[name] = buf[i] if cnt == 1 else buf[i:i + cnt]
            i += cnt
        return out

    def write(self, domain, arrays: dict):
        """Overwrite planes from host FP64 arrays (same names as ``read``)."""
        mask, order = self._layout(list(arrays), domain)
        shape = self._shape(domain)
        parts = []
        for name, cnt in order:
            a = np.asarray(arrays[name], dtype=np.float64).reshape((cnt,) + shape)
            parts.append(a)
        buf = np.ascontiguousarray(np.concatenate(parts, axis=0))
        _check(self.lib, self.ctx, self.lib.lbm_write_fields(self.ctx, domain, mask, 0,
                                                             buf.ctypes.data_as(ctypes.c_void_p)))

    def state_names(self, domain=0):
        """Planes that restore a domain bit for bit (checkpoint set)."""
        d = self.domains[domain]
        names = ["phi", "s_phi"]
        if d["has_U"]:
            names += ["s_U", "jU", "P_U"]
        if d["has_T"]:
            names += ["s_T", "jT", "P_T"]
        if d["has_flow"]:
            names += ["rho", "vel", "s_F"]
        return tuple(names)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def simulation_for(wl: dict, storage=None, **kw) -> Simulation:
    """Create and initialise a Simulation for an ``lbm_inputs`` workload."""
    sim = Simulation(wl["domains"], storage=storage or wl["storage"], **kw)
    sim.init()
    return sim
