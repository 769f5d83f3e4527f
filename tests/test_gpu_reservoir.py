"""GPU vs oracle parity of the excess-mass branch with no receiver (Sec. 2.2,
excess-mass equation; reading R16): cells that convert with no interface
neighbour send their excess to the domain's reservoir, which is spread evenly
over every interface cell, or kept while the domain has none.

The states are seeded pools with isolated interface cells planted in the gas
(they empty at once) and in the liquid (they fill at once), and boxes of one
type holding only such cells.  Every case runs one step per call (each step
finishes its own excess-mass work) and eight steps per call (the excess-mass
work of a step, reservoir included, runs inside the next step's bulk kernel).
FP64 storage: flags bit-exact; PDFs, interface mass, fill level within 1e-12;
the reservoir and the total mass of fslbm_diagnostics against the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, compare, fields_np, sim_from_states
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import setups

pytestmark = pytest.mark.gpu

SHAPE = (70, 9, 24)      # 15 120 cells: 237 tiles of 64, the last one ragged


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _states(cases, scheme=0, collision=0):
    """Oracle parameters and start states of the given (seed, base, drops,
    bubbles) cases, all of one geometry."""
    p, sts = None, []
    for seed, base, drops, bubbles in cases:
        s = setups.planted_state(*SHAPE, seed, drops=drops, bubbles=bubbles, base=base,
                                 refill=scheme, collision=collision)
        q = oracle_params(s)
        p = p or q
        sts.append(oracle_state(s, q))
    return p, sts


def _run(p, sts, steps_per_call, calls, what):
    """Advance the GPU batch and one oracle state per domain; compare after each
    call.  Returns the reservoir events the oracle counted per domain."""
    sim = sim_from_states(p, sts)
    refs = [s.copy() for s in sts]
    events = [0] * len(sts)
    for c in range(calls):
        sim.step(steps_per_call)
        for b, r in enumerate(refs):
            for _ in range(steps_per_call):
                oracle.step(p, r, 1)
                events[b] += r.counts["n_reservoir_events"]
        got = fields_np(sim)
        diag = sim.diagnostics()
        for b, r in enumerate(refs):
            step = (c + 1) * steps_per_call
            compare(got, b, r, what=f"{what} domain {b} step {step}")
            assert abs(diag[b]["reservoir"] - r.reservoir) <= 1e-12, \
                f"{what} domain {b} step {step}: reservoir {diag[b]['reservoir']} vs {r.reservoir}"
            M = oracle.total_mass(p, r)
            assert abs(diag[b]["total_mass"] - M) <= 1e-12 * abs(M), \
                f"{what} domain {b} step {step}: total mass {diag[b]['total_mass']} vs {M}"
    sim.close()
    return events, refs


@pytest.mark.parametrize("steps_per_call", [1, 8])
@pytest.mark.parametrize("seed,scheme,collision", [(0, 0, 0), (1, 4, 1), (5, 2, 0)])
def test_planted_cells_spread_reservoir(seed, scheme, collision, steps_per_call):
    """A pool with three drops and three bubbles planted: six conversions with
    no receiver in the first step, whose reservoir is spread over the pool's
    interface cells, next to ordinary conversions."""
    p, sts = _states([(seed, None, 3, 3)], scheme, collision)
    announce(f"planted pool seed {seed} scheme {scheme} collision {collision} "
             f"{steps_per_call} steps per call")
    calls = 3 if steps_per_call == 1 else 2
    events, refs = _run(p, sts, steps_per_call, calls, f"planted seed {seed}")
    assert events[0] >= 6


@pytest.mark.parametrize("base", ["liquid", "gas"])
@pytest.mark.parametrize("steps_per_call", [1, 8])
def test_reservoir_kept_without_interface_cells(base, steps_per_call):
    """A box of liquid (gas) whose only interface cells are planted bubbles
    (drops): all of them convert, no interface cell is left, and the domain
    keeps its reservoir over the following steps."""
    p, sts = _states([(2 if base == "liquid" else 3, base, 3, 3)])
    announce(f"{base} box with planted cells, {steps_per_call} steps per call")
    events, refs = _run(p, sts, steps_per_call, 2, f"{base} box")
    assert events[0] == 3
    assert refs[0].reservoir != 0.0
    assert not np.any(refs[0].flags == 2)


@pytest.mark.parametrize("steps_per_call", [1, 8])
def test_batch_of_domains_with_and_without_reservoir(steps_per_call):
    """Four domains in one batch: a planted pool (spread), a liquid box and a gas
    box (kept), and a pool with nothing planted (no reservoir).  Each domain's
    reservoir stays its own."""
    p, sts = _states([(0, None, 3, 3), (2, "liquid", 3, 3), (3, "gas", 3, 3), (4, None, 0, 0)],
                     scheme=0, collision=1)
    announce(f"batch of four planted domains, {steps_per_call} steps per call")
    events, refs = _run(p, sts, steps_per_call, 2, "batch")
    assert events[0] >= 6 and events[1] == 3 and events[2] == 3
    assert refs[1].reservoir != 0.0 and refs[2].reservoir != 0.0
