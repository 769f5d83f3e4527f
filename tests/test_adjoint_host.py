"""Host-side pieces of the reverse mode (no GPU):
  * the torch-written standing-wave fill level equals the seeded setup's, and
    its derivative in the amplitude matches a difference of the setup;
  * the stored oracle finite differences are reproducible from the oracle and
    well conditioned where the GPU tests hold the adjoint to 1e-6.
"""
import json
import os

import numpy as np
import pytest
import torch

import _adjoint_ref as R
from paper_2207_14496_amd import adjoint, setups

GOLD_PATH = os.path.join(os.path.dirname(__file__), "golden", "adjoint_fd.json")


@pytest.mark.parametrize("nx,ny,depth,a0", [(64, 128, 64.0, 0.64), (128, 256, 128.0, 1.28),
                                            (32, 40, 20.3, 2.7)])
def test_torch_fill_level_matches_the_setup(nx, ny, depth, a0):
    s = setups.standing_wave(nx=nx, ny=ny, depth=depth, amplitude=a0)
    amp = torch.tensor([a0], dtype=torch.float64)
    phi = adjoint.standing_wave_phi(amp, torch.as_tensor(s.flags)[None], nx, ny, depth)
    np.testing.assert_allclose(phi[0].numpy(), s.phi, rtol=0, atol=2e-15)


def test_torch_fill_level_derivative_in_the_amplitude():
    nx, ny, depth, a0 = 64, 128, 64.0, 0.64
    s = setups.standing_wave(nx=nx, ny=ny, depth=depth, amplitude=a0)
    amp = torch.tensor([a0], dtype=torch.float64, requires_grad=True)
    flags = torch.as_tensor(s.flags)[None]
    phi = adjoint.standing_wave_phi(amp, flags, nx, ny, depth)
    w = torch.linspace(-1.0, 1.0, phi.numel(), dtype=torch.float64).reshape(phi.shape)
    (phi * w).sum().backward()
    d = 1e-7
    sp = setups.standing_wave(nx=nx, ny=ny, depth=depth, amplitude=a0 + d)
    sm = setups.standing_wave(nx=nx, ny=ny, depth=depth, amplitude=a0 - d)
    assert np.array_equal(sp.flags, s.flags) and np.array_equal(sm.flags, s.flags)
    fd = float(((sp.phi - sm.phi) / (2 * d) * w[0].numpy()).sum())
    assert abs(amp.grad.item() - fd) <= 1e-7 * abs(fd)


def test_target_perturbation_ranges():
    xs = np.array([setups.target_perturbation(s) for s in range(64)])
    assert np.all(np.abs(xs[:, 0]) <= 0.01) and np.all(np.abs(xs[:, 1:]) <= 0.05)
    assert len({tuple(x) for x in xs}) == 64


@pytest.mark.skipif(not os.path.exists(GOLD_PATH), reason="adjoint_fd.json not generated")
def test_stored_differences_are_reproducible_and_converged():
    with open(GOLD_PATH) as fh:
        gold = json.load(fh)
    cases = {c["name"]: c for c in gold["cases"]}
    # reproduce one stored loss and one reference derivative from the oracle
    case = cases["wave64_T60"]
    e = case["entries"][0]
    g = case["geometry"]
    prm = e["params"]
    p, st = R.wave_state(g["nx"], g["ny"], g["depth"], prm["a0"], prm["omega"], prm["g"])
    L, h, _, nconv = R.run_loss(p, st, e["target"], case["T"], gold["x_probe"])
    assert L == e["loss"] and nconv == 0
    tgt = R.seeded_target(g["nx"], g["ny"], g["depth"], prm["a0"], prm["omega"], prm["g"], e["seed"],
                          case["T"], gold["x_probe"])
    assert np.array_equal(tgt, np.asarray(e["target"]))
    ref = e["grads"]["a0"]
    d = ref["step"] * prm["a0"]
    vals = {}
    for k in (-2, -1, 1, 2):
        pk, sk = R.wave_state(g["nx"], g["ny"], g["depth"], prm["a0"] + k * d, prm["omega"], prm["g"])
        vals[k] = R.run_loss(pk, sk, e["target"], case["T"], gold["x_probe"])[0]
    c4 = (8.0 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12.0 * d)
    assert c4 == ref["ref"]
    # the d/da0 and d/dg references are converged below half of the 1e-6 bar,
    # so the GPU test's widening to twice the spread never applies to them;
    # d/domega is physically tiny in the short windows (1e-10 .. 1e-8) and is
    # held there to its own spread, but converged to 1e-6 over 300 steps, and
    # below half the bar in the calm conversion-free window of 1500 steps
    assert "wave64_calm_T1500" in cases
    for c in gold["cases"]:
        calm = c["name"].startswith("wave64_calm")
        for ent in c["entries"]:
            if calm:
                assert ent["conversions"] == 0, (c["name"], ent["seed"])
            for name in ("a0", "g", "omega"):
                r = ent["grads"][name]
                assert r is not None, (c["name"], ent["seed"], name)
                spread = abs(r["ref"] - r["confirm"]) / abs(r["ref"])
                if name != "omega" or calm:
                    assert spread <= 5e-7, (c["name"], ent["seed"], name, r)
                elif c["T"] >= 300:
                    assert spread <= 1e-6, (c["name"], ent["seed"], name, r)
