"""Plain FP64 CPU oracle of the free-surface lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against (Schwarzmeier & Ruede, arXiv 2207.14496,
Sec. 2 and Sec. 3).  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.

The arithmetic lives in ``fslbm_oracle.c`` (plain scalar C, compiled with
``-O2 -ffp-contract=off``); this module only builds it with gcc, loads it with
ctypes and marshals numpy arrays in the canonical layout:

* ``flags``  uint8  [N]       1 liquid, 2 interface, 4 gas
* ``f``      float64 [19, N]  post-collision PDFs f*_i
* ``m``      float64 [N]      interface mass (0 on liquid and gas cells)
* ``phi``    float64 [N]      fill level
* cell index ``n = (z*ny + y)*nx + x``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fslbm_oracle.c")
_LIB = os.path.join(_HERE, "_fslbm_oracle.so")

LIQUID, INTERFACE, GAS = 1, 2, 4
Q = 19


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction of multiply-adds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("periodic", ctypes.c_int * 3), ("collision", ctypes.c_int),
                ("refill", ctypes.c_int), ("omega", ctypes.c_double),
                ("trt_lambda", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("sigma", ctypes.c_double), ("p_volume", ctypes.c_double),
                ("eps_phi", ctypes.c_double), ("smag_cs", ctypes.c_double),
                ("free_slip", ctypes.c_int), ("bubble_model", ctypes.c_int)]


class Counts(ctypes.Structure):
    _fields_ = [("n_to_liquid", ctypes.c_long), ("n_to_gas", ctypes.c_long),
                ("n_new_from_gas", ctypes.c_long), ("n_from_liquid", ctypes.c_long),
                ("n_cancelled", ctypes.c_long), ("n_reservoir_events", ctypes.c_long)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, p_ = ctypes.c_double, ctypes.c_void_p
        _lib.orc_feq.argtypes = [d, p_, p_]
        _lib.orc_collide.argtypes = [p_, p_, p_]
        _lib.orc_cell_omega.argtypes = [p_, p_, p_]
        _lib.orc_cell_omega.restype = d
        _lib.orc_normal.argtypes = [p_, p_, ctypes.c_long, p_]
        _lib.orc_surface.argtypes = [p_, p_, p_, p_, p_, p_]
        _lib.orc_step.argtypes = [p_, p_, p_, p_, p_, p_, p_, ctypes.c_int, p_]
        _lib.orc_bubble_labels.argtypes = [p_, p_, p_]
        _lib.orc_init_equilibrium.argtypes = [p_, p_, p_, p_, p_]
        _lib.orc_total_mass.argtypes = [p_, p_, p_, p_, d]
        _lib.orc_total_mass.restype = d
        _lib.orc_macroscopic.argtypes = [p_, p_, p_, p_, p_]
        _lib.orc_refill_cell.argtypes = [p_, p_, p_, p_, p_, ctypes.c_long]
        _lib.orc_link_flux.argtypes = [ctypes.c_int, ctypes.c_int, d, d]
        _lib.orc_link_flux.restype = d
        _lib.orc_lattice.argtypes = [p_, p_, p_, p_, p_]
        _lib.orc_stream_cell.argtypes = [p_, p_, p_, p_, ctypes.c_long, p_]
    return _lib


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    periodic: tuple = (0, 0, 0)
    collision: int = 0          # 0 SRT, 1 TRT
    refill: int = 0             # 0 EQ, 1 EQ+NEQ, 2 GEQ, 3 EXT, 4 AVG
    omega: float = 1.8
    trt_lambda: float = 3.0 / 16.0
    g: tuple = (0.0, 0.0, 0.0)
    sigma: float = 0.0
    p_volume: float = 1.0 / 3.0
    eps_phi: float = 1e-2
    smag_cs: float = 0.0        # Smagorinsky constant C_S (0 = no turbulence model)
    free_slip: int = 0          # walls: 0 no-slip (bounce-back), 1 free-slip (specular)
    bubble_model: int = 0       # 1: per-bubble volume pressures (reading R31)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        for a in range(3):
            p.periodic[a] = int(self.periodic[a])
            p.g[a] = float(self.g[a])
        p.collision, p.refill = int(self.collision), int(self.refill)
        p.omega, p.trt_lambda = float(self.omega), float(self.trt_lambda)
        p.sigma, p.p_volume, p.eps_phi = float(self.sigma), float(self.p_volume), float(self.eps_phi)
        p.smag_cs = float(self.smag_cs)
        p.free_slip = int(self.free_slip)
        p.bubble_model = int(self.bubble_model)
        return p


@dataclass
class State:
    flags: np.ndarray
    f: np.ndarray
    m: np.ndarray
    phi: np.ndarray
    reservoir: float = 0.0
    counts: dict = field(default_factory=dict)
    pbub: np.ndarray = None     # bubble pressure per gas / interface cell (bubble model)

    def copy(self) -> "State":
        return State(self.flags.copy(), self.f.copy(), self.m.copy(), self.phi.copy(),
                     self.reservoir, dict(self.counts),
                     None if self.pbub is None else self.pbub.copy())


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def lattice():
    """D3Q19 velocities (19,3), weights (19,), opposite index (19,) as the oracle holds them."""
    cx, cy, cz = (np.zeros(Q, np.int32) for _ in range(3))
    w = np.zeros(Q)
    op = np.zeros(Q, np.int32)
    lib().orc_lattice(_ptr(cx), _ptr(cy), _ptr(cz), _ptr(w), _ptr(op))
    return np.stack([cx, cy, cz], 1), w, op


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(Q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().orc_feq(float(rho), _ptr(uu), _ptr(out))
    return out


def collide(params: Params, f, g=None) -> np.ndarray:
    """Collision of one cell's post-streaming PDFs (returns f*)."""
    out = np.ascontiguousarray(f, dtype=np.float64).copy()
    gg = np.ascontiguousarray(params.g if g is None else g, dtype=np.float64)
    p = params.c()
    lib().orc_collide(ctypes.byref(p), _ptr(gg), _ptr(out))
    return out


def cell_omega(params: Params, f, g=None) -> float:
    """Relaxation rate the collision uses for one cell's post-streaming PDFs
    (the user-chosen omega, or the Smagorinsky-adjusted one)."""
    ff = np.ascontiguousarray(f, dtype=np.float64)
    gg = np.ascontiguousarray(params.g if g is None else g, dtype=np.float64)
    p = params.c()
    return float(lib().orc_cell_omega(ctypes.byref(p), _ptr(gg), _ptr(ff)))


def normal(params: Params, phi: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros(3)
    p = params.c()
    lib().orc_normal(ctypes.byref(p), _ptr(np.ascontiguousarray(phi, np.float64)), int(n), _ptr(out))
    return out


def surface(params: Params, flags: np.ndarray, phi: np.ndarray):
    """Gas density rho_G and mean curvature kappa_m at interface cells."""
    rhoG = np.zeros(params.N)
    kappa = np.zeros(params.N)
    p = params.c()
    lib().orc_surface(ctypes.byref(p), _ptr(np.ascontiguousarray(flags, np.uint8)),
                      _ptr(np.ascontiguousarray(phi, np.float64)), None, _ptr(rhoG), _ptr(kappa))
    return rhoG, kappa


def init_state(params: Params, flags, phi, rho, u, mass=None) -> State:
    """Canonical state with equilibrium PDFs f* = f_eq(rho, u); m = phi rho on interface cells."""
    N = params.N
    flags = np.ascontiguousarray(flags, np.uint8).reshape(N).copy()
    phi = np.ascontiguousarray(phi, np.float64).reshape(N).copy()
    rho = np.ascontiguousarray(rho, np.float64).reshape(N)
    u = np.ascontiguousarray(u, np.float64).reshape(3, N)
    f = np.zeros((Q, N))
    p = params.c()
    lib().orc_init_equilibrium(ctypes.byref(p), _ptr(flags), _ptr(rho), _ptr(u), _ptr(f))
    if mass is None:
        m = np.where(flags == INTERFACE, phi * rho, 0.0)
    else:
        m = np.where(flags == INTERFACE, np.asarray(mass, np.float64).reshape(N), 0.0)
    pbub = None
    if params.bubble_model:
        # every bubble starts at the volume pressure p_V(0)
        pbub = np.where(flags != LIQUID, float(params.p_volume), 0.0)
    return State(flags, f, np.ascontiguousarray(m), phi, pbub=pbub)


def bubble_labels(params: Params, flags) -> np.ndarray:
    """Bubble label of every cell (smallest cell index of its connected set of
    gas and interface cells; -1 on liquid cells), reading R31."""
    lab = np.zeros(params.N, dtype=np.int64)
    p = params.c()
    lib().orc_bubble_labels(ctypes.byref(p), _ptr(np.ascontiguousarray(flags, np.uint8)), _ptr(lab))
    return lab


def step(params: Params, st: State, nsteps: int = 1) -> State:
    """Advance the canonical state in place by ``nsteps`` FSLBM steps."""
    p = params.c()
    res = ctypes.c_double(st.reservoir)
    cnt = Counts()
    if params.bubble_model and st.pbub is None:
        raise ValueError("the bubble model needs the state's bubble pressures (init_state)")
    pb = _ptr(st.pbub) if params.bubble_model else None
    lib().orc_step(ctypes.byref(p), _ptr(st.flags), _ptr(st.f), _ptr(st.m), _ptr(st.phi),
                   ctypes.byref(res), pb, int(nsteps), ctypes.byref(cnt))
    st.reservoir = res.value
    st.counts = cnt.as_dict()
    return st


def total_mass(params: Params, st: State) -> float:
    p = params.c()
    return lib().orc_total_mass(ctypes.byref(p), _ptr(st.flags), _ptr(st.f), _ptr(st.m),
                                float(st.reservoir))


def macroscopic(params: Params, st: State):
    N = params.N
    rho = np.zeros(N)
    u = np.zeros((3, N))
    p = params.c()
    lib().orc_macroscopic(ctypes.byref(p), _ptr(st.flags), _ptr(st.f), _ptr(rho), _ptr(u))
    return rho, u


def refill_cell(params: Params, flags, togas, phi, f, x: int) -> np.ndarray:
    """Refill one newly created interface cell x exactly as the step does; returns f (copy)."""
    ff = np.ascontiguousarray(f, np.float64).copy()
    p = params.c()
    lib().orc_refill_cell(ctypes.byref(p), _ptr(np.ascontiguousarray(flags, np.uint8)),
                          _ptr(np.ascontiguousarray(togas, np.uint8)),
                          _ptr(np.ascontiguousarray(phi, np.float64)), _ptr(ff), int(x))
    return ff


def stream_cell(params: Params, flags, f, rhoG, n: int) -> np.ndarray:
    """Post-streaming PDFs of cell n (bounce-back / anti-bounce-back / pull)."""
    out = np.zeros(Q)
    p = params.c()
    lib().orc_stream_cell(ctypes.byref(p), _ptr(np.ascontiguousarray(flags, np.uint8)),
                          _ptr(np.ascontiguousarray(f, np.float64)),
                          _ptr(np.ascontiguousarray(rhoG, np.float64)), int(n), _ptr(out))
    return out


def link_flux(cc: int, cn: int, fin: float, fout: float) -> float:
    return lib().orc_link_flux(cc, cn, fin, fout)
