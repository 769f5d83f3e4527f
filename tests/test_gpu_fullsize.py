"""GPU against the oracle at the full sizes of the workloads, in the launch
configuration the benchmark times (several steps per call, so each step's
excess-mass work runs inside the next step's bulk kernel, and graph replay).

FP64 storage: flags bit-exact, PDFs on fluid cells, interface mass and fill
level within 1e-12 (the oracle runs the same steps from the same state).
Longer runs are checked by properties that hold at any size."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, compare, fields_np, sim_from_states
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import fslbm, observe, setups

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _against_oracle(s, chunks, what):
    p = oracle_params(s)
    st = oracle_state(s, p)
    sim = sim_from_states(p, [st])
    t = 0
    for k in chunks:
        announce(f"{what}: GPU {k} steps")
        sim.step(k)
        announce(f"{what}: oracle {k} steps from step {t}")
        oracle.step(p, st, k)
        t += k
        compare(fields_np(sim), 0, st, 1e-12, 1e-12, 1e-12, what=f"{what} step {t}")
    sim.close()
    torch.cuda.empty_cache()


def test_cylindrical_dam_break_512x512x96():
    _against_oracle(setups.cyl_dam_break(), (3, 3), "cylindrical dam break 512x512x96")


def test_rectangular_dam_break_256x128x64():
    _against_oracle(setups.rect_dam_break(), (4, 4), "rectangular dam break 256x128x64")


def test_drop_impact_256_cubed_with_surface_tension():
    _against_oracle(setups.drop_impact(), (2, 2), "drop impact 256^3")


def test_rectangular_dam_break_long_run_properties():
    """20000 steps in FP32 storage with EQ refilling: stable, mass kept to the
    storage precision, the front runs out from the column and stays in the box."""
    s = setups.rect_dam_break(refill=0)
    W, H = s.meta["width"], s.meta["height"]
    sim = fslbm.from_setup(s, storage=fslbm.F32)
    m0 = sim.diagnostics()[0]["total_mass"]
    fronts = []
    for k in range(4):
        announce(f"rectangular dam break FP32, steps {5000 * k}..{5000 * (k + 1)}")
        sim.step(5000)
        d = sim.diagnostics()[0]
        assert d["stable"] and d["finite"], d
        fl = sim.read(("flags",))["flags"][0]
        fronts.append(observe.front_position(fl, s.nx, s.ny, s.nz))
        assert observe.residual_height(fl, s.nx, s.ny, s.nz) <= H + 1
    sim.close()
    assert abs(d["total_mass"] - m0) <= 1e-5 * m0, (m0, d["total_mass"])
    assert fronts[0] > W and fronts[-1] <= s.nx, fronts
    assert all(b >= a - 2 for a, b in zip(fronts, fronts[1:])), fronts


def test_drop_impact_mass_in_fp64():
    """2000 steps (through the impact at about step 1200) in FP64: total mass
    (liquid, interface and reservoir) conserved to 1e-12 relative."""
    s = setups.drop_impact()
    sim = fslbm.from_setup(s, storage=fslbm.F64)
    d0 = sim.diagnostics()[0]
    announce("drop impact FP64, 2000 steps")
    sim.step(2000)
    d1 = sim.diagnostics()[0]
    sim.close()
    assert d1["stable"] and d1["finite"], d1
    assert abs(d1["total_mass"] - d0["total_mass"]) <= 1e-12 * d0["total_mass"], (d0, d1)
