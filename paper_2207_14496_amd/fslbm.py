"""ctypes binding of the FSLBM C ABI (``include/fslbm.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libfslbm.so``.  PyTorch provides device memory (the workspace and the
canonical field tensors) and the stream.  Importing this module raises if the
library has not been built (``python -m paper_2207_14496_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfslbm.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
F64, F32, F16, BF16 = 0, 1, 2, 3
SRT, TRT = 0, 1
REFILL_EQ, REFILL_EQ_NEQ, REFILL_GEQ, REFILL_EXT, REFILL_AVG = 0, 1, 2, 3, 4
LIQUID, INTERFACE, GAS = 1, 2, 4
FIELD_FLAGS, FIELD_PDF, FIELD_MASS, FIELD_PHI, FIELD_RHO, FIELD_VEL = (1 << k for k in range(6))
FIELD_NAMES = ["flags", "pdf", "mass", "phi", "rho", "vel", "bubble_pressure"]
STORAGE_NAMES = {F64: "f64", F32: "f32", F16: "f16", BF16: "bf16"}
STORAGE_BYTES = {F64: 8, F32: 4, F16: 2, BF16: 2}
STATIC_WORKSPACE_BYTES = 64 << 20   # the static workspace of fslbm_init_static

# Exported symbols, in the order include/fslbm.h declares them.
SYMBOLS = ["fslbm_workspace_bytes", "fslbm_init", "fslbm_init_static", "fslbm_step",
           "fslbm_step_timed",
           "fslbm_refill_scheme",
           "fslbm_use_graphs", "fslbm_set_stream", "fslbm_read_fields", "fslbm_diagnostics",
           "fslbm_last_step_stats", "fslbm_adjoint_workspace_bytes", "fslbm_adjoint_forward",
           "fslbm_adjoint_backward", "fslbm_last_error", "fslbm_destroy"]


class FslbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fslbm status {status}: {msg}")
        self.status = status


class CParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("periodic", ctypes.c_int32 * 3),
                ("collision", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("omega", ctypes.c_double),
                ("trt_lambda", ctypes.c_double), ("gravity", ctypes.c_double * 3),
                ("sigma", ctypes.c_double), ("p_volume", ctypes.c_double),
                ("eps_phi", ctypes.c_double), ("omega_b", ctypes.POINTER(ctypes.c_double)),
                ("gravity_b", ctypes.POINTER(ctypes.c_double)), ("stream", ctypes.c_void_p),
                ("smagorinsky_cs", ctypes.c_double), ("free_slip", ctypes.c_int32),
                ("bubble_model", ctypes.c_int32), ("diag_every", ctypes.c_int32)]


class CDiag(ctypes.Structure):
    _fields_ = [("total_mass", ctypes.c_double), ("reservoir", ctypes.c_double),
                ("max_speed", ctypes.c_double), ("n_liquid", ctypes.c_int64),
                ("n_interface", ctypes.c_int64), ("n_gas", ctypes.c_int64),
                ("finite", ctypes.c_int32), ("pad", ctypes.c_int32)]


class CStepStats(ctypes.Structure):
    _fields_ = [("interface_cells", ctypes.c_int64), ("new_from_gas", ctypes.c_int64),
                ("from_liquid", ctypes.c_int64), ("converted", ctypes.c_int64)]


_lib = None


class CAdjSpec(ctypes.Structure):
    _fields_ = [("nsteps", ctypes.c_int32), ("n_checkpoints", ctypes.c_int32),
                ("x_probe", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("target", ctypes.c_void_p)]


def lib() -> ctypes.CDLL:
    """Load libfslbm.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              f"`python -m paper_2207_14496_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, vp = ctypes.POINTER, ctypes.c_void_p
        L.fslbm_workspace_bytes.argtypes = [P(CParams), P(ctypes.c_size_t)]
        L.fslbm_init.argtypes = [P(CParams), vp, ctypes.c_size_t, vp, vp, vp, vp, vp, vp, P(vp)]
        L.fslbm_init_static.argtypes = [P(CParams), vp, vp, vp, vp, vp, vp, P(vp)]
        L.fslbm_step.argtypes = [vp, ctypes.c_int32]
        L.fslbm_step_timed.argtypes = [vp, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double)]
        L.fslbm_refill_scheme.argtypes = [vp, ctypes.c_int32]
        L.fslbm_use_graphs.argtypes = [vp, ctypes.c_int32]
        L.fslbm_set_stream.argtypes = [vp, vp]
        L.fslbm_read_fields.argtypes = [vp, ctypes.c_uint32, P(vp)]
        L.fslbm_diagnostics.argtypes = [vp, P(CDiag)]
        L.fslbm_last_step_stats.argtypes = [vp, P(CStepStats)]
        L.fslbm_last_step_stats.restype = ctypes.c_int
        L.fslbm_adjoint_workspace_bytes.argtypes = [vp, P(CAdjSpec), P(ctypes.c_size_t)]
        L.fslbm_adjoint_forward.argtypes = [vp, P(CAdjSpec), vp, ctypes.c_size_t, vp, vp]
        L.fslbm_adjoint_backward.argtypes = [vp, P(CAdjSpec), vp, ctypes.c_size_t, vp, vp, vp,
                                             vp, vp, vp]
        L.fslbm_last_error.argtypes = [vp]
        L.fslbm_last_error.restype = ctypes.c_char_p
        L.fslbm_destroy.argtypes = [vp]
        L.fslbm_destroy.restype = None
        for name in ("fslbm_workspace_bytes", "fslbm_init", "fslbm_init_static", "fslbm_step",
                     "fslbm_step_timed",
                     "fslbm_refill_scheme",
                     "fslbm_use_graphs", "fslbm_set_stream", "fslbm_read_fields",
                     "fslbm_diagnostics", "fslbm_adjoint_workspace_bytes",
                     "fslbm_adjoint_forward", "fslbm_adjoint_backward"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    batch: int = 1
    periodic: tuple = (0, 0, 0)
    collision: int = SRT
    storage: int = F64
    refill: int = REFILL_EQ
    omega: float = 1.8
    trt_lambda: float = 3.0 / 16.0
    gravity: tuple = (0.0, 0.0, 0.0)
    sigma: float = 0.0
    p_volume: float = 1.0 / 3.0
    eps_phi: float = 1e-2
    omega_b: tuple | None = None      # per-domain omega [B]
    gravity_b: tuple | None = None    # per-domain gravity [B][3]
    smagorinsky_cs: float = 0.0       # Smagorinsky constant (0 = no turbulence model)
    free_slip: int = 0                # walls: 0 no-slip, 1 free-slip (specular)
    bubble_model: int = 0             # 1: per-bubble volume pressures
    diag_every: int = 0               # stability check period in steps (0 = off)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def to_c(self, stream=None):
        p = CParams()
        p.nx, p.ny, p.nz, p.batch = self.nx, self.ny, self.nz, self.batch
        for a in range(3):
            p.periodic[a] = int(self.periodic[a])
            p.gravity[a] = float(self.gravity[a])
        p.collision, p.storage, p.refill = int(self.collision), int(self.storage), int(self.refill)
        p.omega, p.trt_lambda = float(self.omega), float(self.trt_lambda)
        p.sigma, p.p_volume, p.eps_phi = float(self.sigma), float(self.p_volume), float(self.eps_phi)
        p.smagorinsky_cs = float(self.smagorinsky_cs)
        p.free_slip = int(self.free_slip)
        p.bubble_model = int(self.bubble_model)
        p.diag_every = int(self.diag_every)
        keep = []
        if self.omega_b is not None:
            arr = (ctypes.c_double * self.batch)(*[float(v) for v in self.omega_b])
            keep.append(arr)
            p.omega_b = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        if self.gravity_b is not None:
            flat = [float(v) for row in self.gravity_b for v in row]
            arr = (ctypes.c_double * (3 * self.batch))(*flat)
            keep.append(arr)
            p.gravity_b = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        p.stream = stream
        return p, keep


def _check(status, ctx=None):
    if status != OK:
        msg = lib().fslbm_last_error(ctx).decode()
        raise FslbmError(status, msg)


def workspace_bytes(params: Params) -> int:
    p, _keep = params.to_c()
    n = ctypes.c_size_t()
    _check(lib().fslbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def _dev(t, dtype, device):
    return torch.as_tensor(t).to(device=device, dtype=dtype).contiguous()


class Simulation:
    """B FSLBM domains on one GPU; state lives in a torch-owned workspace.

    flags [B,N] uint8, phi [B,N], rho [B,N], u [B,3,N] (or pdf [B,19,N] and
    optionally mass [B,N]) are the canonical initial fields (any array type;
    copied to the device).  static_workspace=True creates the context with
    fslbm_init_static (the library's own static device workspace, no
    workspace tensor; one such context per device at a time).
    """

    def __init__(self, params: Params, flags, phi, rho=None, u=None, pdf=None, mass=None,
                 device="cuda", stream=None, static_workspace: bool = False):
        self.params = params
        self.device = torch.device(device)
        B, N = params.batch, params.N
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cp, keep = params.to_c(ctypes.c_void_p(self._stream.cuda_stream))
        nbytes = ctypes.c_size_t()
        _check(lib().fslbm_workspace_bytes(ctypes.byref(cp), ctypes.byref(nbytes)))
        if static_workspace:
            self.workspace = None
        else:
            self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
        f = _dev(flags, torch.uint8, self.device).reshape(B, N)
        ph = _dev(phi, torch.float64, self.device).reshape(B, N)
        r = _dev(rho, torch.float64, self.device).reshape(B, N) if rho is not None else None
        uu = _dev(u, torch.float64, self.device).reshape(B, 3, N) if u is not None else None
        pd = _dev(pdf, torch.float64, self.device).reshape(B, 19, N) if pdf is not None else None
        ms = _dev(mass, torch.float64, self.device).reshape(B, N) if mass is not None else None
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device), torch.cuda.stream(self._stream):
            if static_workspace:
                st = lib().fslbm_init_static(ctypes.byref(cp), ptr(f), ptr(ph), ptr(r), ptr(uu),
                                             ptr(pd), ptr(ms), ctypes.byref(ctx))
            else:
                st = lib().fslbm_init(ctypes.byref(cp), ctypes.c_void_p(self._ws_ptr),
                                      nbytes.value, ptr(f), ptr(ph), ptr(r), ptr(uu), ptr(pd),
                                      ptr(ms), ctypes.byref(ctx))
        _check(st, None)
        self._ctx = ctx
        self.steps_done = 0

    # ------------------------------------------------------------------ control
    def step(self, nsteps: int = 1):
        _check(lib().fslbm_step(self._ctx, int(nsteps)), self._ctx)
        self.steps_done += int(nsteps)

    def step_timed(self, nsteps: int):
        """Run nsteps with events around every bulk stream-collide kernel; returns
        (summed bulk-kernel ms, wall ms of the sequence).  Synchronises."""
        bulk, total = ctypes.c_double(), ctypes.c_double()
        _check(lib().fslbm_step_timed(self._ctx, int(nsteps), ctypes.byref(bulk),
                                      ctypes.byref(total)), self._ctx)
        self.steps_done += int(nsteps)
        return bulk.value, total.value

    def set_refill(self, scheme: int):
        _check(lib().fslbm_refill_scheme(self._ctx, int(scheme)), self._ctx)
        self.params.refill = int(scheme)

    def use_graphs(self, enable: bool):
        _check(lib().fslbm_use_graphs(self._ctx, int(bool(enable))), self._ctx)

    def set_stream(self, stream):
        self._stream = stream
        _check(lib().fslbm_set_stream(self._ctx, ctypes.c_void_p(stream.cuda_stream)), self._ctx)

    # ------------------------------------------------------------------ state
    def read(self, fields=("flags", "pdf", "mass", "phi")) -> dict:
        """Canonical fields as new device tensors."""
        B, N = self.params.batch, self.params.N
        shapes = {"flags": ((B, N), torch.uint8), "pdf": ((B, 19, N), torch.float64),
                  "mass": ((B, N), torch.float64), "phi": ((B, N), torch.float64),
                  "rho": ((B, N), torch.float64), "vel": ((B, 3, N), torch.float64),
                  "bubble_pressure": ((B, N), torch.float64)}
        out, mask = {}, 0
        ptrs = (ctypes.c_void_p * 7)()
        for name in fields:
            k = FIELD_NAMES.index(name)
            shp, dt = shapes[name]
            t = torch.empty(shp, dtype=dt, device=self.device)
            out[name] = t
            ptrs[k] = t.data_ptr()
            mask |= 1 << k
        _check(lib().fslbm_read_fields(self._ctx, mask, ptrs), self._ctx)
        return out

    def diagnostics(self, raise_unstable: bool = False) -> list:
        """Per-domain total mass, reservoir, max speed, cell counts, finiteness."""
        B = self.params.batch
        arr = (CDiag * B)()
        st = lib().fslbm_diagnostics(self._ctx, arr)
        if st == EUNSTABLE and not raise_unstable:
            pass
        else:
            _check(st, self._ctx)
        out = []
        for d in arr:
            out.append({"total_mass": d.total_mass, "reservoir": d.reservoir,
                        "max_speed": d.max_speed, "n_liquid": d.n_liquid,
                        "n_interface": d.n_interface, "n_gas": d.n_gas,
                        "finite": bool(d.finite), "stable": st != EUNSTABLE})
        return out

    def last_step_stats(self) -> dict:
        """List sizes of the most recent step (all domains)."""
        st = CStepStats()
        _check(lib().fslbm_last_step_stats(self._ctx, ctypes.byref(st)), self._ctx)
        return {k: getattr(st, k) for k, _ in CStepStats._fields_}

    # ------------------------------------------------------------------ reverse mode
    def adjoint_forward(self, target, nsteps: int, x_probe: int, n_checkpoints: int = 0):
        """Run the loss window of ``nsteps`` steps from the current state with
        checkpoints; ``target`` [B, nsteps] holds h*(t), t = 1..nsteps.  Returns
        (loss [B], height [B, nsteps+1]) as float64 numpy arrays.  The state
        advances to the end of the window."""
        import numpy as np
        B = self.params.batch
        tgt = _dev(target, torch.float64, self.device).reshape(B, int(nsteps)).contiguous()
        spec = CAdjSpec(int(nsteps), int(n_checkpoints), int(x_probe), 0, tgt.data_ptr())
        nbytes = ctypes.c_size_t()
        _check(lib().fslbm_adjoint_workspace_bytes(self._ctx, ctypes.byref(spec),
                                                   ctypes.byref(nbytes)), self._ctx)
        ws = getattr(self, "_adj_ws", None)
        if ws is None or ws.numel() < nbytes.value + 256:
            self._adj_ws = None
            ws = self._adj_ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        wptr = (ws.data_ptr() + 255) & ~255
        loss = np.zeros(B)
        height = np.zeros((B, int(nsteps) + 1))
        _check(lib().fslbm_adjoint_forward(self._ctx, ctypes.byref(spec), ctypes.c_void_p(wptr),
                                           nbytes.value, loss.ctypes.data_as(ctypes.c_void_p),
                                           height.ctypes.data_as(ctypes.c_void_p)), self._ctx)
        self._adj = (spec, tgt, wptr, nbytes.value)
        self.steps_done += int(nsteps)
        return loss, height

    def adjoint_backward(self, dloss=None, state_grads: bool = True) -> dict:
        """Gradient of sum_b dloss[b] L_b for the last adjoint_forward window:
        omega [B] and gravity [B, 3] (numpy), and, with ``state_grads``, the
        start state's pdf [B, 19, N], mass [B, N] and phi [B, N] (device)."""
        import numpy as np
        if getattr(self, "_adj", None) is None:
            raise FslbmError(EINVAL, "adjoint_backward needs a preceding adjoint_forward")
        spec, _tgt, wptr, nbytes = self._adj
        B, N = self.params.batch, self.params.N
        dl = None
        if dloss is not None:
            dl = np.ascontiguousarray(np.asarray(dloss, dtype=np.float64).reshape(B))
        gom = np.zeros(B)
        gg = np.zeros((B, 3))
        out = {}
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        if state_grads:
            out["pdf"] = torch.empty((B, 19, N), dtype=torch.float64, device=self.device)
            out["mass"] = torch.empty((B, N), dtype=torch.float64, device=self.device)
            out["phi"] = torch.empty((B, N), dtype=torch.float64, device=self.device)
        _check(lib().fslbm_adjoint_backward(
            self._ctx, ctypes.byref(spec), ctypes.c_void_p(wptr), nbytes,
            dl.ctypes.data_as(ctypes.c_void_p) if dl is not None else None,
            gom.ctypes.data_as(ctypes.c_void_p), gg.ctypes.data_as(ctypes.c_void_p),
            ptr(out.get("pdf")), ptr(out.get("mass")), ptr(out.get("phi"))), self._ctx)
        out["omega"] = gom
        out["gravity"] = gg
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            lib().fslbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_setup(setup, storage=F64, batch=1, device="cuda", pdf=None, mass=None,
               omega_b=None, gravity_b=None, **over) -> Simulation:
    """Simulation from a ``setups.Setup`` (the same initial state replicated B times
    unless pdf/mass are given per domain)."""
    params = Params(setup.nx, setup.ny, setup.nz, batch, tuple(setup.periodic), setup.collision,
                    storage, setup.refill, setup.omega, setup.trt_lambda, tuple(setup.g),
                    setup.sigma, setup.p_volume, setup.eps_phi, omega_b, gravity_b)
    for k, v in over.items():
        setattr(params, k, v)
    N = setup.N

    def rep(a, shape):
        t = torch.as_tensor(a)
        return t.reshape(1, *shape).expand(batch, *shape).contiguous()

    flags = rep(setup.flags, (N,))
    phi = rep(setup.phi, (N,))
    if pdf is None:
        return Simulation(params, flags, phi, rep(setup.rho, (N,)), rep(setup.u, (3, N)),
                          mass=mass, device=device)
    return Simulation(params, flags, phi, pdf=pdf, mass=mass, device=device)
