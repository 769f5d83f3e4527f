"""The bubble model on the GPU against the oracle (Sec. 2.2, volume pressure of
enclosed gas; reading R31), FP64 storage: flags bit-exact, PDFs, interface
mass and fill level within 1e-12, bubble pressures within 1e-12 relative (the
per-bubble sums are atomic on the GPU, in cell order in the oracle)."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, compare, fields_np, sim_from_states
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import setups

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(sim, st, what):
    got = fields_np(sim)
    compare(got, 0, st, 1e-12, 1e-12, 1e-12, what=what)
    pb = sim.read(("bubble_pressure",))["bubble_pressure"][0].cpu().numpy()
    err = np.max(np.abs(pb - st.pbub) / np.maximum(np.abs(st.pbub), 1e-300))
    assert err <= 1e-12, f"{what}: bubble pressure error {err:.2e}"


@pytest.mark.parametrize("graphs", [True, False], ids=["graph-replay", "direct-launches"])
def test_enclosed_bubble_step_by_step_then_in_calls(graphs):
    """Every step after a call's first replays the step and the bubble
    kernels as one graph; with graphs off they are launched one by one."""
    s = setups.rising_bubbles()
    p = oracle_params(s, bubble_model=1)
    st = oracle_state(s, p)
    announce(f"enclosed bubble 24x8x40, bubble model, graphs {'on' if graphs else 'off'}")
    sim = sim_from_states(p, [st])
    sim.use_graphs(graphs)
    for k in range(1, 6):
        sim.step(1)
        oracle.step(p, st, 1)
        _check(sim, st, f"bubble step {k}")
    for k in range(4):
        sim.step(50)
        oracle.step(p, st, 50)
        _check(sim, st, f"bubble step {5 + 50 * (k + 1)}")
    # compressed: the pressure is above p_V(0)
    assert st.pbub[st.flags != 1].max() > p.p_volume
    sim.close()


def test_bubbles_that_merge_and_split():
    s = setups.rising_bubbles(centres=((12.0, 4.0, 9.0), (12.0, 4.0, 18.5)))
    p = oracle_params(s, bubble_model=1)
    st = oracle_state(s, p)
    announce("two stacked bubbles 24x8x40, bubble model, 350 steps")
    sim = sim_from_states(p, [st])
    counts = set()
    for k in range(7):
        sim.step(50)
        oracle.step(p, st, 50)
        _check(sim, st, f"two bubbles step {50 * (k + 1)}")
        lab = oracle.bubble_labels(p, st.flags)
        counts.add(len(np.unique(lab[lab >= 0])))
    assert counts == {1, 2}
    sim.close()


def test_atmosphere_only_dam_break():
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=0)
    p = oracle_params(s, bubble_model=1)
    st = oracle_state(s, p)
    announce("small dam break with the bubble model (atmosphere only)")
    sim = sim_from_states(p, [st])
    for k in range(3):
        sim.step(10)
        oracle.step(p, st, 10)
        _check(sim, st, f"atmosphere dam break step {10 * (k + 1)}")
    sim.close()


def test_enclosed_bubble_with_surface_tension():
    """sigma != 0: the curvature kernel adds the Laplace term to the cell's
    bubble pressure (rho_G = 3 (p_bubble + 2 sigma kappa))."""
    s = setups.rising_bubbles()
    p = oracle_params(s, bubble_model=1, sigma=2e-3)
    st = oracle_state(s, p)
    announce("enclosed bubble with surface tension, bubble model")
    sim = sim_from_states(p, [st])
    for k in range(1, 4):
        sim.step(1)
        oracle.step(p, st, 1)
        _check(sim, st, f"bubble with sigma step {k}")
    sim.step(40)
    oracle.step(p, st, 40)
    _check(sim, st, "bubble with sigma step 43")
    sim.close()


def test_batch_of_two_domains_with_bubbles():
    """Labels are global cell indices and never cross domains: two different
    bubble states in one launch, each against its own oracle run."""
    s1 = setups.rising_bubbles()
    s2 = setups.rising_bubbles(centres=((12.0, 4.0, 9.0), (12.0, 4.0, 18.5)))
    p = oracle_params(s1, bubble_model=1)
    st1, st2 = oracle_state(s1, p), oracle_state(s2, p)
    announce("two domains with bubbles in one launch")
    sim = sim_from_states(p, [st1, st2])
    for k in range(3):
        sim.step(50)
        oracle.step(p, st1, 50)
        oracle.step(p, st2, 50)
        got = fields_np(sim)
        pb = sim.read(("bubble_pressure",))["bubble_pressure"].cpu().numpy()
        for b, st in enumerate((st1, st2)):
            compare(got, b, st, 1e-12, 1e-12, 1e-12, what=f"domain {b} step {50 * (k + 1)}")
            err = np.max(np.abs(pb[b] - st.pbub) / np.maximum(np.abs(st.pbub), 1e-300))
            assert err <= 1e-12, f"domain {b}: bubble pressure error {err:.2e}"
    sim.close()


def test_fp32_storage_keeps_boyle_law():
    """FP32 shifted populations (m, phi and the bubble sums stay FP64): the
    bubble keeps p V = p_V(0) V(0) to rounding, and its pressure stays within
    1e-5 of the FP64 oracle's after 200 steps."""
    from paper_2207_14496_amd import fslbm
    s = setups.rising_bubbles()
    p = oracle_params(s, bubble_model=1)
    st = oracle_state(s, p)
    gas = st.flags != 1
    pv0 = p.p_volume * float(np.sum(np.maximum(0.0, 1.0 - st.phi[gas])))
    announce("enclosed bubble 24x8x40, bubble model, f32 storage, 200 steps")
    sim = sim_from_states(p, [st], storage=fslbm.F32)
    sim.step(200)
    oracle.step(p, st, 200)
    got = fields_np(sim)
    pb = sim.read(("bubble_pressure",))["bubble_pressure"][0].cpu().numpy()
    sim.close()
    g = got["flags"][0] != 1
    pr = np.unique(pb[g])
    assert len(pr) == 1, "one enclosed bubble, one pressure"
    v = float(np.sum(np.maximum(0.0, 1.0 - got["phi"][0][g])))
    assert abs(pr[0] * v - pv0) <= 1e-11 * pv0
    po = np.unique(st.pbub[st.flags != 1])
    assert len(po) == 1 and abs(pr[0] - po[0]) <= 1e-5 * po[0]
    assert pr[0] > p.p_volume
