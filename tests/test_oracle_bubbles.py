"""Pins of the oracle's bubble model (Sec. 2.2, volume pressure of enclosed gas;
reading R31).

* Labels: the bubbles are the connected sets of gas and interface cells over
  D3Q19 links; checked against scipy's connected-component labelling with the
  same 18-neighbour structure, on random cell types.
* Atmosphere only: when all gas reaches the top layer, the model changes
  nothing (bit-identical to the run without it).
* Boyle's law: a bubble that keeps its cells together keeps p V, and its
  pressure rises as it is compressed.
* Amount: the total p V of the enclosed bubbles is conserved through the
  splits and merges of a run (it moves between bubbles, the sum stays).
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import setups

LIQ = 1


def _bubbles(p, st):
    """[(label, gas volume, pressure)] of every gas/interface set."""
    lab = oracle.bubble_labels(p, st.flags)
    out = []
    for r in np.unique(lab[lab >= 0]):
        sel = lab == r
        out.append((int(r), float(np.sum(np.maximum(0.0, 1.0 - st.phi[sel]))), float(st.pbub[r])))
    return lab, out


@pytest.mark.parametrize("seed", range(4))
def test_labels_are_the_d3q19_connected_sets(seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 9, 7, 6
    flags = rng.choice(np.array([1, 2, 4], np.uint8), size=nx * ny * nz, p=[0.55, 0.2, 0.25])
    p = oracle.Params(nx, ny, nz, periodic=(0, 0, 0), bubble_model=1)
    lab = oracle.bubble_labels(p, flags).reshape(nz, ny, nx)
    struct = np.ones((3, 3, 3), bool)
    for c in np.ndindex(3, 3, 3):
        if sum(abs(k - 1) for k in c) == 3:     # the 8 corners are not D3Q19 links
            struct[c] = False
    ref, nref = ndimage.label(flags.reshape(nz, ny, nx) != LIQ, structure=struct)
    assert np.all((lab >= 0) == (ref > 0))
    # the same partition, each set labelled with its smallest cell index
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    for k in range(1, nref + 1):
        cells = ref == k
        assert np.all(lab[cells] == idx[cells].min())
    assert len(np.unique(lab[lab >= 0])) == nref


def test_atmosphere_only_changes_nothing():
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=0)
    runs = []
    for bm in (0, 1):
        p = oracle_params(s, bubble_model=bm)
        st = oracle_state(s, p)
        oracle.step(p, st, 60)
        runs.append((p, st))
    (p0, a), (p1, b) = runs
    assert np.array_equal(a.flags, b.flags)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.m, b.m) and np.array_equal(a.phi, b.phi)
    assert np.all(b.pbub[b.flags != LIQ] == p1.p_volume)


def test_boyle_law_for_an_enclosed_bubble():
    """One bubble under the hydrostatic load of the liquid above it: it is
    compressed and its pressure rises so that p V stays p_V(0) V(0)."""
    s = setups.rising_bubbles()
    p = oracle_params(s, bubble_model=1)
    st = oracle_state(s, p)
    _, bub = _bubbles(p, st)
    assert len(bub) == 1
    v0 = bub[0][1]
    pv0 = p.p_volume * v0
    for _ in range(5):
        oracle.step(p, st, 100)
        _, bub = _bubbles(p, st)
        assert len(bub) == 1
        v, pr = bub[0][1], bub[0][2]
        assert abs(pr * v - pv0) <= 1e-11 * pv0
    assert v < v0 * (1 - 5e-3) and pr > p.p_volume * (1 + 5e-3)


def test_amount_is_conserved_through_splits_and_merges():
    """Two bubbles stacked one cell apart touch, merge and split again as they
    rise: the number of bubbles changes, their total p V does not."""
    s = setups.rising_bubbles(centres=((12.0, 4.0, 9.0), (12.0, 4.0, 18.5)))
    p = oracle_params(s, bubble_model=1)
    st = oracle_state(s, p)
    _, bub = _bubbles(p, st)
    total0 = sum(b[1] * b[2] for b in bub)
    counts = {len(bub)}
    for _ in range(7):
        oracle.step(p, st, 50)
        _, bub = _bubbles(p, st)
        total = sum(b[1] * b[2] for b in bub)
        assert abs(total - total0) <= 1e-11 * total0
        counts.add(len(bub))
    assert counts == {1, 2}


def test_bubble_pressure_acts_on_the_liquid():
    """The free-surface condition uses the bubble's own pressure: the same
    bubble started at 3% over p_V(0) grows, at p_V(0) it does not."""
    vols = []
    for over in (1.0, 1.03):
        s = setups.rising_bubbles()
        p = oracle_params(s, bubble_model=1)
        st = oracle_state(s, p)
        st.pbub[st.flags != LIQ] *= over
        _, bub = _bubbles(p, st)
        v0 = bub[0][1]
        oracle.step(p, st, 200)
        _, bub = _bubbles(p, st)
        vols.append(bub[0][1] / v0)
    assert vols[0] < 1.0 < vols[1]
