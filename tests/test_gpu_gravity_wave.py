"""The gravity wave of Sec. 4.1 on the GPU (FP64) with every refilling scheme,
against the values the paper prints for it (golden/gravity_wave_sec41.json).

At the paper's resolution L = 800, up to t* = 15, per scheme:
* the first four half-periods T*/2 against the paper's series for the same
  scheme: within 1% for EQ, GEQ and AVG, 2% for EQ+NEQ; EXT within 4% over
  its first two, with the long-then-short pair the paper shows for it
  (T*/2 above 1.05 pi, then below 0.95 pi);
* for the four schemes, the half-periods within 2.5% of the analytic pi;
* the first logarithmic decrement (the start and the first positive maximum)
  against the paper's: within 8% for EQ, EQ+NEQ and GEQ, 22% for AVG, whose
  printed first positive amplitude is higher than here (the paper remarks on
  it).  The paper prints no decrement for EXT.
Total mass is conserved to 1e-12 at L = 200."""
import json
import os

import numpy as np
import pytest

from _gpu import announce
from paper_2207_14496_amd import fslbm, setups, waves

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gravity_wave_sec41.json")))
NAMES = ["EQ", "EQ+NEQ", "GEQ", "EXT", "AVG"]
HP_BAND = {"EQ": 0.01, "EQ+NEQ": 0.02, "GEQ": 0.01, "AVG": 0.01}
LD_BAND = {"EQ": 0.08, "EQ+NEQ": 0.08, "GEQ": 0.08, "AVG": 0.22}


@pytest.mark.parametrize("scheme", range(5), ids=NAMES)
def test_gravity_wave_l800_against_the_paper(scheme):
    name = NAMES[scheme]
    announce(f"gravity wave L=800, FP64, {name}, t* up to 15 (about 520k steps)")
    t, a, s, diag = waves.run(800, fslbm.F64, t_star_end=15.0, every=40, refill=scheme)
    hp = waves.half_periods(t, a)
    ld = waves.log_decrements(t, a)
    ref = GOLD["schemes_L800"][name]
    paper_hp = np.asarray(ref["half_period"][:4])
    print(f"{name} T*/2:", np.round(hp[:4], 4).tolist(), "paper:", np.round(paper_hp, 4).tolist(),
          "delta:", [(round(x, 3), round(d, 4)) for x, d in ld[:2]],
          "paper:", ref.get("log_decrement", [])[:2])
    assert diag["finite"] and diag["max_speed"] < 0.1
    assert len(hp) >= 4 and len(ld) >= 1
    if name == "EXT":
        assert np.all(np.abs(hp[:2] - paper_hp[:2]) <= 0.04 * paper_hp[:2]), hp[:2]
        assert hp[0] > 1.05 * np.pi and hp[1] < 0.95 * np.pi, hp[:2]
        return
    band = HP_BAND[name]
    assert np.all(np.abs(hp[:4] - paper_hp) <= band * paper_hp), hp[:4]
    assert np.all(np.abs(hp[:4] - np.pi) <= 0.025 * np.pi), hp[:4]
    paper_ld = ref["log_decrement"][0]
    assert abs(ld[0][0] - paper_ld[0]) < 0.1
    assert abs(ld[0][1] - paper_ld[1]) <= LD_BAND[name] * paper_ld[1], (ld[0], paper_ld)


def test_gravity_wave_mass_conservation():
    announce("gravity wave L=200, FP64 mass over 5000 steps")
    sim = fslbm.from_setup(setups.gravity_wave(200), storage=fslbm.F64)
    m0 = sim.diagnostics()[0]["total_mass"]
    sim.step(5000)
    m1 = sim.diagnostics()[0]["total_mass"]
    sim.close()
    assert abs(m1 - m0) <= 1e-12 * m0, (m0, m1)
