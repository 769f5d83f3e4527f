"""Degenerate domains and reduced-precision storage on the GPU, against the oracle.

* A liquid box with no interface cell (every list empty), a domain of gas only
  (no fluid tile at all) and a single periodic cell: the step matches the
  oracle (FP64: flags bit-exact, PDFs within 1e-12) or leaves the state as it is.
* FP32, FP16 and BF16 storage of the shifted populations (collide in FP32;
  mass, fill level and thresholds in FP64): the small dam break after 200
  steps, with the error against the FP64 oracle stated as mass drift, fluid
  volume (sum of the fill level) and the share of cells whose type differs.
  The bounds are 5-10 times the errors measured on the MI355X, so a codec or
  precision mistake (a wrong scale, a reduced-precision store of the mass)
  fails them.
"""
import numpy as np
import pytest
import torch

import oracle
from _gpu import GAS, LIQ, announce, compare, fields_np, sim_from_states
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import fslbm, setups

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _liquid_state(p, rng):
    N = p.N
    rho = 1.0 + 0.01 * rng.standard_normal(N)
    u = 0.02 * rng.standard_normal((3, N))
    return oracle.init_state(p, np.full(N, LIQ, np.uint8), np.ones(N), rho, u)


@pytest.mark.parametrize("collision", [0, 1])
def test_liquid_box_without_interface(collision):
    """No interface cell: the interface, conversion and excess lists stay empty."""
    rng = np.random.default_rng(61 + collision)
    p = oracle.Params(16, 8, 8, periodic=(1, 1, 1), collision=collision, omega=1.6, g=(0.0, 0.0, -1e-5))
    st = _liquid_state(p, rng)
    announce(f"liquid box 16x8x8 collision {collision}, 4 steps")
    sim = sim_from_states(p, [st])
    for k in range(1, 5):
        sim.step(1)
        oracle.step(p, st, 1)
        compare(fields_np(sim), 0, st, what=f"liquid box step {k}")
    assert sim.last_step_stats()["interface_cells"] == 0
    sim.close()


def test_single_periodic_cell():
    """One liquid cell that is its own neighbour along every direction."""
    rng = np.random.default_rng(67)
    p = oracle.Params(1, 1, 1, periodic=(1, 1, 1), collision=1, omega=1.3, g=(1e-4, 0.0, 0.0))
    st = _liquid_state(p, rng)
    announce("single periodic cell, 5 steps")
    sim = sim_from_states(p, [st])
    for k in range(1, 6):
        sim.step(1)
        oracle.step(p, st, 1)
        compare(fields_np(sim), 0, st, what=f"single cell step {k}")
    sim.close()


def test_gas_only_domain():
    """No fluid at all: no tile is listed, nothing changes, no mass appears."""
    p = oracle.Params(64, 4, 4, periodic=(0, 0, 0), collision=1, omega=1.6, g=(0.0, 0.0, -1e-4))
    N = p.N
    st = oracle.init_state(p, np.full(N, GAS, np.uint8), np.zeros(N), np.ones(N), np.zeros((3, N)))
    announce("gas-only domain 64x4x4, 10 steps")
    sim = sim_from_states(p, [st])
    sim.step(10)
    got = fields_np(sim)
    assert np.array_equal(got["flags"][0], st.flags)
    assert np.all(got["phi"][0] == 0.0)
    d = sim.diagnostics()[0]
    assert d["total_mass"] == 0.0 and d["n_interface"] == 0 and d["n_liquid"] == 0 and d["stable"]
    sim.close()


# (storage, mass drift, fluid volume error, share of differing cell types)
# after 200 steps of a collapsing dam break.  These are sanity bounds on a
# trajectory that diverges from the oracle's through conversion decisions, so
# they move with the rounding order of the collision: two algebraically equal
# forms of it gave FP16 volume errors of 7.0e-7 and 3.0e-5 and type shares of
# 0.0003 and 0.0035 (FP32: 1.3e-8 and 0 for both).  The per-element bound that
# follows from each storage's unit roundoff is held by
# test_gpu_codec_elementwise.py.
PRECISION_BOUNDS = [
    (fslbm.F32, 1e-7, 1e-7, 0.002),
    (fslbm.F16, 1e-6, 1e-4, 0.01),
    (fslbm.BF16, 1e-4, 1e-3, 0.03),
]


@pytest.mark.parametrize("storage,b_mass,b_vol,b_types", PRECISION_BOUNDS)
def test_reduced_precision_error_against_the_oracle(storage, b_mass, b_vol, b_types):
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=0)
    p = oracle_params(s)
    st = oracle_state(s, p)
    steps = 200
    name = {fslbm.F32: "f32", fslbm.F16: "f16", fslbm.BF16: "bf16"}[storage]
    announce(f"small dam break, {name} storage, {steps} steps against the FP64 oracle")
    sim = sim_from_states(p, [st], storage=storage)
    m0 = sim.diagnostics()[0]["total_mass"]
    sim.step(steps)
    d = sim.diagnostics()[0]
    got = fields_np(sim)
    sim.close()
    oracle.step(p, st, steps)
    drift = abs(d["total_mass"] - m0) / m0
    vol_o = float(st.phi.sum())
    vol_err = abs(float(got["phi"][0].sum()) - vol_o) / vol_o
    types = float(np.mean(got["flags"][0] != st.flags))
    print(f"{name}: mass drift {drift:.2e}, fluid volume error {vol_err:.2e}, "
          f"differing cell types {types:.4f}", flush=True)
    assert d["stable"] and d["finite"]
    assert drift <= b_mass
    assert vol_err <= b_vol
    assert types <= b_types
