"""Reduced-precision storage against the FP64 oracle, element by element.

One step from an identical FP64 state in FP32, FP16 (scale 2^10) and BF16
storage of the shifted populations s (f_i - w_i), with FP32 collide arithmetic
and FP64 mass, fill level and thresholds on the GPU.  The only input error is
the rounding of the start state into the storage type, at most u |f - w_i| per
population (u = 2^-24, 2^-11, 2^-8: half an ulp, relative); the arithmetic adds
a few FP32 roundings of O(1) values.  Propagated through one step (worked out
in the design notes, reduced-precision section), with G the largest |f - w_i|
of the start state within two cells:
  populations of cells whose type is kept       <= 40 u G + 32 u32
  populations next to a conversion (refills)    <= 256 u G + 32 u32
  mass and fill level                           <= 64 u G + 32 u32
  mass and fill level next to a conversion      <= 1024 u G + 32 u32
Cell types are bit-exact except within two cells of a cell whose fill level
right before the conversions lies within the fill-level bound of a threshold
(1 + eps or -eps): there both decisions are correct to the storage's
precision, and only the region they can reach is left out."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, fields_np, sim_from_states
from _util import (GAS, IFC, before_conversions, dilate, oracle_params, oracle_state,
                   window_max)
from paper_2207_14496_amd import fslbm, setups

pytestmark = pytest.mark.gpu

U = {fslbm.F32: 2.0 ** -24, fslbm.F16: 2.0 ** -11, fslbm.BF16: 2.0 ** -8}
U32 = 2.0 ** -24
K_F, K_F_NEAR, K_M, K_M_NEAR, K_ARITH = 40, 256, 64, 1024, 32


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cases():
    out = []
    # rows of 192 cells: the middle tile of each interior row takes the bulk
    # kernel's uniform-offset path, the others the general one
    s = setups.random_interface_state(192, 16, 12, 4, periodic=(1, 1, 0), g=(0.0, 0.0, -1e-4),
                                      collision=1, refill=0)
    out.append(("random 192x16x12 TRT EQ", s, 0))
    s = setups.random_interface_state(192, 16, 12, 5, periodic=(1, 1, 1), refill=4)
    out.append(("random 192x16x12 SRT AVG", s, 0))
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=2)
    out.append(("dam break 40x6x24 TRT GEQ at step 115", s, 115))
    return out


@pytest.mark.parametrize("storage", [fslbm.F32, fslbm.F16, fslbm.BF16],
                         ids=["f32", "f16", "bf16"])
@pytest.mark.parametrize("case", range(3))
def test_one_step_against_fp64_oracle(case, storage):
    name, s, warm = _cases()[case]
    p = oracle_params(s)
    st0 = oracle_state(s, p)
    if warm:
        oracle.step(p, st0, warm)
    st0.reservoir = 0.0
    announce(f"codec {fslbm.STORAGE_NAMES[storage]}: {name}")
    u = U[storage]
    _, w, _ = oracle.lattice()
    fluid0 = st0.flags != GAS
    g_cell = np.where(fluid0, np.abs(st0.f - w[:, None]).max(axis=0), 0.0)
    G = window_max(g_cell, p, 2)

    ref = st0.copy()
    oracle.step(p, ref, 1)
    assert ref.counts["n_reservoir_events"] == 0
    pre = before_conversions(p, st0)
    tol_phi = K_M * u * G + K_ARITH * U32
    itf0 = st0.flags == IFC
    eps = p.eps_phi
    marginal = itf0 & ((np.abs(pre.phi - (1 + eps)) <= tol_phi) | (np.abs(pre.phi + eps) <= tol_phi))
    excluded = dilate(marginal, p, 2)
    near = dilate(ref.flags != st0.flags, p, 1)

    sim = sim_from_states(p, [st0], storage)
    sim.step(1)
    got = fields_np(sim)
    sim.close()

    keep = ~excluded
    fl = got["flags"][0]
    bad = np.nonzero(keep & (fl != ref.flags))[0]
    assert bad.size == 0, f"{name}: {bad.size} cell types differ outside the marginal region"
    cmp = keep & (ref.flags != GAS)
    tf = np.where(near, K_F_NEAR, K_F) * u * G + K_ARITH * U32
    tm = np.where(near, K_M_NEAR, K_M) * u * G + K_ARITH * U32
    ef = np.abs(got["pdf"][0] - ref.f).max(axis=0)
    em = np.abs(got["mass"][0] - ref.m)
    ep = np.abs(got["phi"][0] - ref.phi)
    worst = {}
    for what, e, t, sel in (("pdf", ef, tf, cmp), ("mass", em, tm, keep & (ref.flags == IFC)),
                            ("phi", ep, tm, keep)):
        over = np.nonzero(sel & (e > t))[0]
        assert over.size == 0, (f"{name}: {what} error {e[over[0]]:.3e} > bound {t[over[0]]:.3e} "
                                f"at cell {over[0]} ({over.size} cells)")
        scale = u * np.maximum(G, 1e-30)
        worst[what] = float(np.max(np.where(sel, e / scale, 0.0)))
    announce(f"  excluded {int(excluded.sum())} of {p.N} cells ({int(marginal.sum())} marginal); "
             f"max error / (u G): pdf {worst['pdf']:.2f}, mass {worst['mass']:.2f}, "
             f"phi {worst['phi']:.2f}")
