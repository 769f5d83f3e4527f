"""Shared helpers of the test suite (no step arithmetic here)."""
import numpy as np

import oracle
from paper_2207_14496_amd import setups

LIQ, IFC, GAS = 1, 2, 4

D3Q19_OFFSETS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                 (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
                 (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def oracle_params(s: setups.Setup, **kw) -> oracle.Params:
    p = oracle.Params(s.nx, s.ny, s.nz, tuple(s.periodic), s.collision, s.refill, s.omega,
                      s.trt_lambda, tuple(s.g), s.sigma, s.p_volume, s.eps_phi)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def oracle_state(s: setups.Setup, p: oracle.Params = None) -> oracle.State:
    p = p or oracle_params(s)
    return oracle.init_state(p, s.flags, s.phi, s.rho, s.u)


def neighbour_pairs(flags, nx, ny, nz, periodic):
    """Yield boolean masks (a, b) of all D3Q19 links as shifted views."""
    f3 = flags.reshape(nz, ny, nx)
    for dx, dy, dz in D3Q19_OFFSETS:
        sh = f3
        valid = np.ones_like(f3, dtype=bool)
        for axis, d, per, n in ((2, dx, periodic[0], nx), (1, dy, periodic[1], ny),
                                (0, dz, periodic[2], nz)):
            if d == 0:
                continue
            sh = np.roll(sh, -d, axis=axis)
            if not per:
                idx = [slice(None)] * 3
                idx[axis] = slice(n - 1, n) if d > 0 else slice(0, 1)
                valid[tuple(idx)] = False
        yield f3, sh, valid


def check_topology(st: oracle.State, p: oracle.Params):
    """Invariants of a valid free-surface state (Sec. 2.2): known cell types,
    no liquid-gas link, phi = 1 in liquid and 0 in gas, m = 0 off the interface."""
    fl = st.flags
    assert set(np.unique(fl)).issubset({LIQ, IFC, GAS})
    for a, b, valid in neighbour_pairs(fl, p.nx, p.ny, p.nz, p.periodic):
        bad = valid & (((a == LIQ) & (b == GAS)) | ((a == GAS) & (b == LIQ)))
        assert not bad.any(), "liquid cell adjacent to gas cell"
    assert np.all(st.phi[fl == LIQ] == 1.0)
    assert np.all(st.phi[fl == GAS] == 0.0)
    assert np.all(st.m[fl != IFC] == 0.0)


def before_conversions(p: oracle.Params, st: oracle.State) -> oracle.State:
    """The state one step on with conversions switched off (eps_phi so large
    that no fill level crosses it): stream, collide and mass exchange are those
    of the real step, so its phi, m and f* are the values the conversion rules
    see."""
    q = oracle.Params(**{**p.__dict__, "eps_phi": 1e9})
    return oracle.step(q, st.copy(), 1)


def dilate(mask: np.ndarray, p, radius: int) -> np.ndarray:
    """Cells within Chebyshev distance `radius` of a cell in mask (periodic
    axes wrap, walls cut)."""
    return _window(mask.astype(np.float64), p, radius, np.max) > 0


def window_max(v: np.ndarray, p, radius: int) -> np.ndarray:
    """Max of v over the (2 radius + 1)^3 window of every cell (periodic axes
    wrap; beyond a wall counts as 0)."""
    return _window(v, p, radius, np.max)


def _window(v, p, r, red):
    a = v.reshape(p.nz, p.ny, p.nx)
    pads = [(r, r)] * 3
    for axis, per in ((0, p.periodic[2]), (1, p.periodic[1]), (2, p.periodic[0])):
        mode = "wrap" if per else "constant"
        pw = [(0, 0)] * 3
        pw[axis] = (r, r)
        a = np.pad(a, pw, mode=mode)
    from numpy.lib.stride_tricks import sliding_window_view
    w = sliding_window_view(a, (2 * r + 1,) * 3)
    return red(w, axis=(3, 4, 5)).reshape(-1)
