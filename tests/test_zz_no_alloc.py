"""The allocation-free entry point fslbm_init_static against fslbm_init.

fslbm_init_static builds the context on the library's static device workspace
instead of a caller workspace; the kernels are the same.  Two calls in a row,
the second with a smaller input (the static array then still holds the first
context's data): after every call of fslbm_step the canonical fields of the
two contexts agree (flags bit-exact, PDFs, mass and fill level within 1e-12 in
FP64 storage) and both match the oracle.  Also: a workspace larger than the
static array is refused with FSLBM_ENOMEM, and a second live static context
on the device with FSLBM_ESTATE."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, compare, fields_np, params_from_oracle
from _util import oracle_params, oracle_state
from paper_2207_14496_amd import fslbm, setups

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(p, states, static):
    q = params_from_oracle(p, fslbm.F64, len(states))
    stack = lambda name: np.stack([getattr(s, name) for s in states])
    return fslbm.Simulation(q, stack("flags"), stack("phi"), pdf=stack("f"), mass=stack("m"),
                            static_workspace=static)


def _run_both(p, states, calls, what):
    """Advance a caller-workspace context, a static-workspace context and the
    oracle side by side; compare after every call."""
    assert fslbm.workspace_bytes(params_from_oracle(p, fslbm.F64, len(states))) \
        <= fslbm.STATIC_WORKSPACE_BYTES
    ref = _sim(p, states, static=False)
    sta = _sim(p, states, static=True)
    orc = [s.copy() for s in states]
    done = 0
    for n in calls:
        ref.step(n)
        sta.step(n)
        done += n
        for s in orc:
            oracle.step(p, s, n)
        gr, gs = fields_np(ref), fields_np(sta)
        for b, s in enumerate(orc):
            # the static context against the existing entry point's ...
            as_state = oracle.State(gr["flags"][b], gr["pdf"][b], gr["mass"][b], gr["phi"][b])
            compare(gs, b, as_state, what=f"{what} static vs workspace, domain {b} step {done}")
            # ... and both against the oracle
            compare(gs, b, s, 1e-11, 1e-11, 1e-11, what=f"{what} static vs oracle, domain {b} step {done}")
            compare(gr, b, s, 1e-11, 1e-11, 1e-11, what=f"{what} workspace vs oracle, domain {b} step {done}")
        dr, ds = ref.diagnostics(), sta.diagnostics()
        for b in range(len(orc)):
            assert abs(dr[b]["reservoir"] - ds[b]["reservoir"]) <= 1e-12
            assert abs(dr[b]["total_mass"] - ds[b]["total_mass"]) <= 1e-12 * abs(dr[b]["total_mass"])
    sta.close()
    ref.close()


def test_static_workspace_two_calls_second_smaller():
    # first call: the small dam break, 5760 cells, eight steps per call
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=2)
    p = oracle_params(s)
    announce("static workspace, call 1: dam break 40x6x24, GEQ, 3 x 8 steps")
    _run_both(p, [oracle_state(s, p)], [8, 8, 8], "dam break")
    # second call: a smaller input, two random-state domains of 1080 cells,
    # planted so that the reservoir is used
    cases = [setups.planted_state(12, 10, 9, 7, drops=1, bubbles=0, depth=0.3),
             setups.random_interface_state(12, 10, 9, 8, periodic=(1, 1, 0), g=(0.0, 0.0, -1e-4))]
    p2 = oracle_params(cases[0])
    announce("static workspace, call 2: two domains of 12x10x9, steps 1, 2, 3")
    _run_both(p2, [oracle_state(c, p2) for c in cases], [1, 2, 3], "random pair")


def test_static_workspace_refusals():
    # larger than the static array: refused before anything touches the device
    big = fslbm.Params(512, 512, 96, storage=fslbm.F32, omega=1.9)
    assert fslbm.workspace_bytes(big) > fslbm.STATIC_WORKSPACE_BYTES
    cp, _keep = big.to_c(None)
    ctx = ctypes.c_void_p()
    st = fslbm.lib().fslbm_init_static(ctypes.byref(cp), None, None, None, None, None, None,
                                       ctypes.byref(ctx))
    assert st == fslbm.ENOMEM and not ctx.value
    assert b"static workspace" in fslbm.lib().fslbm_last_error(None)
    # one live static context per device
    s = setups.random_interface_state(12, 10, 9, 3)
    p = oracle_params(s)
    first = _sim(p, [oracle_state(s, p)], static=True)
    with pytest.raises(fslbm.FslbmError) as e:
        _sim(p, [oracle_state(s, p)], static=True)
    assert e.value.status == fslbm.ESTATE
    first.step(2)
    first.close()
    again = _sim(p, [oracle_state(s, p)], static=True)
    again.step(1)
    again.close()
