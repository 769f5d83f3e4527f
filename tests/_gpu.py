"""GPU-test helpers: load an oracle state into the library through the C ABI
and compare canonical fields element by element."""
import sys

import numpy as np
import torch

import oracle
from paper_2207_14496_amd import fslbm

LIQ, IFC, GAS = 1, 2, 4


def params_from_oracle(p: oracle.Params, storage=fslbm.F64, batch=1, **kw) -> fslbm.Params:
    q = fslbm.Params(p.nx, p.ny, p.nz, batch, tuple(p.periodic), p.collision, storage, p.refill,
                     p.omega, p.trt_lambda, tuple(p.g), p.sigma, p.p_volume, p.eps_phi,
                     smagorinsky_cs=p.smag_cs, free_slip=p.free_slip, bubble_model=p.bubble_model)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def sim_from_states(p: oracle.Params, states, storage=fslbm.F64, **kw) -> fslbm.Simulation:
    """One domain per oracle state (same geometry)."""
    B = len(states)
    q = params_from_oracle(p, storage, B, **kw)
    flags = np.stack([s.flags for s in states])
    phi = np.stack([s.phi for s in states])
    pdf = np.stack([s.f for s in states])
    mass = np.stack([s.m for s in states])
    return fslbm.Simulation(q, flags, phi, pdf=pdf, mass=mass)


def fields_np(sim: fslbm.Simulation):
    out = sim.read(("flags", "pdf", "mass", "phi"))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def compare(got: dict, b: int, st: oracle.State, tol_f=1e-12, tol_m=1e-12, tol_phi=1e-12,
            what=""):
    """Flags bit-exact; PDFs on fluid cells, interface mass and fill level within
    the given absolute tolerances.  Returns the max errors."""
    fl = got["flags"][b]
    mism = np.nonzero(fl != st.flags)[0]
    assert mism.size == 0, f"{what}: {mism.size} flag mismatches, first cells {mism[:8]}, " \
                           f"gpu {fl[mism[:8]]} oracle {st.flags[mism[:8]]}"
    fluid = st.flags != GAS
    ef = np.max(np.abs(got["pdf"][b][:, fluid] - st.f[:, fluid])) if fluid.any() else 0.0
    itf = st.flags == IFC
    em = np.max(np.abs(got["mass"][b][itf] - st.m[itf])) if itf.any() else 0.0
    ep = np.max(np.abs(got["phi"][b] - st.phi))
    assert ef <= tol_f, f"{what}: pdf error {ef:.3e} > {tol_f}"
    assert em <= tol_m, f"{what}: mass error {em:.3e} > {tol_m}"
    assert ep <= tol_phi, f"{what}: phi error {ep:.3e} > {tol_phi}"
    return ef, em, ep


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()
