"""GPU vs oracle parity through the C ABI (FP64 storage: flags bit-exact,
PDFs / interface mass / fill level within 1e-12)."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, compare, fields_np, params_from_oracle, sim_from_states
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import fslbm, setups

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run_pair(setup_or_p, st0, nsteps, what, tol=1e-12, **kw):
    p = setup_or_p
    sim = sim_from_states(p, [st0], **kw)
    ref = st0.copy()
    for k in range(1, nsteps + 1):
        sim.step(1)
        oracle.step(p, ref, 1)
        compare(fields_np(sim), 0, ref, tol, tol, tol, what=f"{what} step {k}")
    sim.close()
    return ref


def test_standing_wave_first_steps():
    """64 x 128 standing wave (SRT, EQ): the first four steps (both AA parities)."""
    s = setups.config("standing-wave-64")
    p = oracle_params(s)
    announce("standing wave 64x128, 4 steps from the initial state")
    _run_pair(p, oracle_state(s, p), 4, "standing-wave")


def test_standing_wave_restarts_along_the_run():
    """Start the GPU from oracle states along 1000 steps of the standing wave and
    compare the next two steps each time."""
    s = setups.config("standing-wave-64")
    p = oracle_params(s)
    st = oracle_state(s, p)
    for t in range(0, 1000, 125):
        announce(f"standing wave restart at step {t}")
        _run_pair(p, st.copy(), 2, f"standing-wave@{t}")
        oracle.step(p, st, 125)


@pytest.mark.parametrize("scheme", range(5))
def test_random_states_all_schemes(scheme):
    """Random interface states with fill levels straddling both thresholds, one
    periodic and one walled: conversions, refills and excess mass on the first
    step, for every refilling scheme."""
    for seed, periodic in ((scheme, (1, 1, 1)), (10 + scheme, (0, 1, 0))):
        s = setups.random_interface_state(12, 10, 9, seed, periodic=periodic, refill=scheme,
                                          g=(0.0, 0.0, -1e-4), collision=seed % 2)
        p = oracle_params(s)
        st = oracle_state(s, p)
        announce(f"random state seed {seed} periodic {periodic} scheme {scheme}")
        ref = _run_pair(p, st, 3, f"random seed {seed} scheme {scheme}")
        assert ref.counts is not None


@pytest.mark.parametrize("collision,smag,periodic", [(0, 0.0, (1, 1, 0)), (1, 0.0, (1, 1, 0)),
                                                     (1, 0.15, (1, 1, 0)), (1, 0.0, (0, 1, 0)),
                                                     (0, 0.0, (0, 0, 0)), (1, 0.0, (1, 1, 1))])
def test_random_states_wide_rows(collision, smag, periodic):
    """Rows of 192 cells: the tile in the middle of every interior row is
    updated through the bulk kernel's uniform-offset path in both step
    parities, the tiles at the row ends and on the boundary rows through the
    general one in the layout A -> B step, with walls or periodic wraps on
    each pair of faces.  One domain and a batch of two, one step per call and
    four."""
    s0 = setups.random_interface_state(192, 12, 10, 40 + collision, periodic=periodic,
                                       g=(0.0, 0.0, -1e-4), collision=collision)
    s1 = setups.random_interface_state(192, 12, 10, 50 + collision, periodic=periodic,
                                       g=(0.0, 0.0, -1e-4), collision=collision)
    p = oracle_params(s0, smag_cs=smag)
    announce(f"wide rows 192x12x10 collision {collision} smagorinsky {smag} periodic {periodic}")
    _run_pair(p, oracle_state(s0, p), 3, "wide rows")
    sts = [oracle_state(s0, p), oracle_state(s1, p)]
    sim = sim_from_states(p, sts)
    for k in range(3):
        sim.step(4)
        for st in sts:
            oracle.step(p, st, 4)
        got = fields_np(sim)
        for b, st in enumerate(sts):
            compare(got, b, st, 1e-11, 1e-11, 1e-11, what=f"wide rows batch domain {b} step {4 * (k + 1)}")
    sim.close()


@pytest.mark.parametrize("scheme", range(5))
def test_dam_break_small_all_schemes(scheme):
    """Small 3-D dam break (TRT, walls): 40 steps of collapse with conversions,
    eight steps per call (the excess-mass work of all but the last step of a
    call runs inside the next step's bulk kernel)."""
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=scheme)
    p = oracle_params(s)
    st = oracle_state(s, p)
    announce(f"dam break 40x6x24 scheme {scheme}")
    sim = sim_from_states(p, [st])
    for k in range(5):
        sim.step(8)
        oracle.step(p, st, 8)
        compare(fields_np(sim), 0, st, 1e-11, 1e-11, 1e-11, what=f"dam break step {8 * (k + 1)}")
    sim.close()


def test_dam_break_small_step_by_step():
    """The same collapse one step per call (every step finishes on its own)."""
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=0)
    p = oracle_params(s)
    st = oracle_state(s, p)
    announce("dam break 40x6x24 step by step")
    sim = sim_from_states(p, [st])
    for k in range(24):
        sim.step(1)
        oracle.step(p, st, 1)
        if k % 8 == 7:
            compare(fields_np(sim), 0, st, 1e-11, 1e-11, 1e-11, what=f"dam break step {k + 1}")
    sim.close()


@pytest.mark.parametrize("collision", [0, 1])
def test_smagorinsky_random_states(collision):
    """Turbulence model on (Sec. 2.1): random interface states, three steps,
    SRT and TRT."""
    for seed in (20 + collision, 30 + collision):
        s = setups.random_interface_state(12, 10, 9, seed, periodic=(1, 1, 1), g=(0.0, 0.0, -1e-4),
                                          collision=collision)
        p = oracle_params(s, smag_cs=0.15)
        st = oracle_state(s, p)
        announce(f"Smagorinsky random state seed {seed} collision {collision}")
        _run_pair(p, st, 3, f"Smagorinsky seed {seed}")


def test_smagorinsky_dam_break_multi_step_calls():
    """Turbulence model on: the small dam break (TRT, walls), eight steps per
    call, against the oracle every call."""
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=0, omega=1.99)
    p = oracle_params(s, smag_cs=0.1)
    st = oracle_state(s, p)
    announce("Smagorinsky dam break 40x6x24")
    sim = sim_from_states(p, [st])
    for k in range(5):
        sim.step(8)
        oracle.step(p, st, 8)
        compare(fields_np(sim), 0, st, 1e-11, 1e-11, 1e-11, what=f"LES dam break step {8 * (k + 1)}")
    sim.close()


@pytest.mark.parametrize("collision", [0, 1])
def test_free_slip_random_states(collision):
    """Free-slip (specular) walls on two and three axes: random interface
    states, three steps (populations reflected into neighbouring cells, the
    mass exchange along the reflected links, anti-bounce-back from gas found
    there)."""
    for seed, periodic in ((40 + collision, (0, 1, 0)), (50 + collision, (0, 0, 0))):
        s = setups.random_interface_state(12, 10, 9, seed, periodic=periodic, g=(0.0, 0.0, -1e-4),
                                          collision=collision)
        p = oracle_params(s, free_slip=1)
        st = oracle_state(s, p)
        announce(f"free-slip random state seed {seed} periodic {periodic}")
        _run_pair(p, st, 3, f"free-slip seed {seed}")


@pytest.mark.parametrize("scheme", [0, 1, 2, 4])
def test_free_slip_dam_break_multi_step_calls(scheme):
    """The paper's dam-break walls (free-slip) with its turbulence model at a
    high relaxation rate: the small dam break, eight steps per call."""
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=scheme, omega=1.99)
    p = oracle_params(s, free_slip=1, smag_cs=0.1)
    st = oracle_state(s, p)
    announce(f"free-slip + Smagorinsky dam break scheme {scheme}")
    sim = sim_from_states(p, [st])
    for k in range(5):
        sim.step(8)
        oracle.step(p, st, 8)
        compare(fields_np(sim), 0, st, 1e-11, 1e-11, 1e-11, what=f"free-slip dam break step {8 * (k + 1)}")
    sim.close()


@pytest.mark.parametrize("scheme", [0, 1, 2, 3, 4])
def test_paper_dam_break_multi_step_calls(scheme):
    """The dam break as the paper runs it (Sec. 4.2): 750 x 1 x 200, one cell
    layer between free-slip walls, SRT at omega = 1.9995 with the turbulence
    model, gravity from Ga = 1.83e9; three calls of eight steps."""
    s = setups.paper_dam_break(W=50, refill=scheme)
    p = oracle_params(s, free_slip=1, smag_cs=0.1)
    st = oracle_state(s, p)
    announce(f"paper dam break 750x1x200 scheme {scheme}")
    sim = sim_from_states(p, [st])
    for k in range(3):
        sim.step(8)
        oracle.step(p, st, 8)
        compare(fields_np(sim), 0, st, 1e-11, 1e-11, 1e-11, what=f"paper dam break step {8 * (k + 1)}")
    sim.close()


def test_surface_tension_drop():
    """Curvature path: a small 3-D drop with surface tension (sigma != 0)."""
    n = 20
    c = n / 2
    sd = lambda x, y, z: np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) - 6.0
    phi = setups.shape_fill(n, n, n, sd).ravel()
    flags = setups.types_from_phi(phi)
    setups.close_interface(flags, phi, (n, n, n), (1, 1, 1))
    phi = np.where(flags == 1, 1.0, np.where(flags == 4, 0.0, phi))
    p = oracle.Params(n, n, n, periodic=(1, 1, 1), collision=1, omega=1.7, sigma=5e-3)
    st = oracle.init_state(p, flags, phi, np.ones(n ** 3), np.zeros((3, n ** 3)))
    announce("drop with surface tension, 10 steps")
    _run_pair(p, st, 10, "drop")


def test_batch_of_domains_with_own_parameters():
    """Three domains in one launch, each with its own state, omega and gravity."""
    states, omegas, gravs = [], [1.6, 1.75, 1.9], []
    for k in range(3):
        s = setups.random_interface_state(10, 9, 8, 40 + k, periodic=(1, 0, 1))
        st = oracle_state(s, oracle_params(s))
        states.append(st)
        gravs.append((0.0, -1e-4 * (k + 1), 0.0))
    p = oracle_params(s)
    sim = sim_from_states(p, states, omega_b=omegas, gravity_b=gravs)
    announce("batch of 3 domains")
    sim.step(2)
    got = fields_np(sim)
    for k in range(3):
        pk = oracle.Params(**{**p.__dict__, "omega": omegas[k], "g": gravs[k]})
        oracle.step(pk, states[k], 2)
        compare(got, k, states[k], what=f"domain {k}")


def test_graph_replay_matches_direct_launches():
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=2)
    p = oracle_params(s)
    st = oracle_state(s, p)
    a = sim_from_states(p, [st])
    b = sim_from_states(p, [st])
    b.use_graphs(False)
    announce("graph vs direct launches, 30 steps")
    a.step(30)
    b.step(30)
    fa, fb = fields_np(a), fields_np(b)
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k


def test_mass_conservation_and_diagnostics():
    """Total mass from the device diagnostics stays within 1e-12 relative over
    500 dam-break steps (FP64) and matches the oracle's total."""
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4)
    p = oracle_params(s)
    st = oracle_state(s, p)
    M0 = oracle.total_mass(p, st)
    sim = sim_from_states(p, [st])
    d0 = sim.diagnostics()[0]
    assert abs(d0["total_mass"] - M0) < 1e-12 * M0
    announce("mass conservation 500 steps")
    sim.step(500)
    d = sim.diagnostics()[0]
    assert abs(d["total_mass"] - M0) < 1e-12 * M0
    assert d["finite"] and d["stable"]
