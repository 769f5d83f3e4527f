"""The stability check of fslbm_params.diag_every (Sec. 4: the scheme is
stable while |u| stays below c_s = 1/sqrt(3)).

* With checks every K steps a stable run gives the same state, bit for bit,
  as the same steps without checks (a checked step finishes its own
  excess-mass work, which otherwise runs inside the next step's bulk kernel).
* A uniform flow at |u| = 0.7 > c_s in a periodic liquid box makes fslbm_step
  return FSLBM_EUNSTABLE at the first check, after exactly K steps, with the
  context still usable (its diagnostics report the speed).
* The bubble-model path runs the same checks (same state within rounding:
  its per-bubble sums are floating-point atomics in varying order)."""
import numpy as np
import pytest
import torch

from _gpu import announce
from paper_2207_14496_amd import fslbm, setups

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _fields(sim):
    out = sim.read(("flags", "pdf", "mass", "phi"))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("graphs", [True, False])
def test_checks_leave_a_stable_run_unchanged(graphs):
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=1)
    announce(f"stability checks every 3 steps, dam break 40x6x24, graphs {graphs}")
    runs = []
    for K in (0, 3):
        sim = fslbm.from_setup(s, storage=fslbm.F64, diag_every=K)
        sim.use_graphs(graphs)
        sim.step(10)   # checks after steps 3, 6 and 9
        sim.step(5)    # and 12, 15
        runs.append(_fields(sim))
        sim.close()
    for k in ("flags", "pdf", "mass", "phi"):
        assert np.array_equal(runs[0][k], runs[1][k]), k


def test_uniform_flow_above_sound_speed_is_reported():
    n = (16, 8, 8)
    N = n[0] * n[1] * n[2]
    u = np.zeros((3, N))
    u[0] = 0.7
    params = fslbm.Params(*n, batch=1, periodic=(1, 1, 1), collision=fslbm.SRT, storage=fslbm.F64,
                          omega=1.0, diag_every=4)
    sim = fslbm.Simulation(params, np.full(N, fslbm.LIQUID, np.uint8), np.ones(N), np.ones(N), u)
    announce("uniform flow |u| = 0.7, checks every 4 steps")
    with pytest.raises(fslbm.FslbmError) as e:
        sim.step(10)
    assert e.value.status == fslbm.EUNSTABLE
    assert "after step 4" in str(e.value) and "c_s" in str(e.value), str(e.value)
    d = sim.diagnostics()[0]   # not poisoned
    assert not d["stable"] and abs(d["max_speed"] - 0.7) < 1e-9 and d["finite"]
    sim.close()


def test_bubble_model_runs_the_checks():
    s = setups.rising_bubbles()
    announce("bubble model with checks every 2 steps")
    runs = []
    for K in (0, 2):
        sim = fslbm.from_setup(s, storage=fslbm.F64, bubble_model=1, diag_every=K)
        sim.step(7)
        f = _fields(sim)
        f["p"] = sim.read(("bubble_pressure",))["bubble_pressure"].cpu().numpy()
        runs.append(f)
        sim.close()
    # the per-bubble sums are floating-point atomics, whose order (and so the
    # last bits) varies from run to run: the same state within rounding
    assert np.array_equal(runs[0]["flags"], runs[1]["flags"])
    for k in ("pdf", "mass", "phi", "p"):
        d = np.max(np.abs(runs[0][k] - runs[1][k]))
        assert d <= 1e-12, (k, d)
