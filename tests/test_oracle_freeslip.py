"""Pins of the oracle's free-slip (specular) walls (Sec. 2.1; reading R30).

* Mirror symmetry: a domain between two free-slip walls evolves exactly as
  the first half of a periodic domain of twice the length that holds the
  mirror image in the second half (the walls are planes of symmetry) -- for
  every direction, including the diagonals that are reflected into a
  neighbouring cell.
* A body-force driven flow between free-slip walls stays a uniform plug
  flow (with no-slip walls it does not); its momentum grows by the force.
* Mass is conserved to rounding in free-surface runs that touch the walls
  (the mass exchange follows the reflected links).
"""
import numpy as np
import pytest

import oracle
from _util import LIQ, oracle_params, oracle_state
from paper_2207_14496_amd import setups

D3Q19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
         (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
MIRROR_Y = [D3Q19.index((cx, -cy, cz)) for cx, cy, cz in D3Q19]


def _all_liquid(p, rho, u):
    N = p.N
    return oracle.init_state(p, np.full(N, LIQ, np.uint8), np.ones(N), rho, u)


@pytest.mark.parametrize("collision,g", [(0, (0.0, 0.0, 0.0)), (1, (2e-5, 0.0, 0.0))])
def test_free_slip_walls_are_mirror_planes(collision, g):
    rng = np.random.default_rng(7)
    nx, ny, nz = 6, 8, 5
    # walls in y only, so the mirror image lives in a periodic y of length 2 ny
    pw = oracle.Params(nx, ny, nz, periodic=(1, 0, 1), collision=collision, omega=1.7, g=g,
                       free_slip=1)
    pp = oracle.Params(nx, 2 * ny, nz, periodic=(1, 1, 1), collision=collision, omega=1.7, g=g)
    rho = 1.0 + 0.01 * rng.standard_normal((nz, ny, nx))
    u = 0.02 * rng.standard_normal((3, nz, ny, nx))
    rho2 = np.concatenate([rho, rho[:, ::-1, :]], axis=1)
    u2 = np.concatenate([u, u[:, :, ::-1, :]], axis=2)
    u2[1, :, ny:, :] *= -1.0                    # u_y is odd under the mirror
    sw = _all_liquid(pw, rho.reshape(-1), u.reshape(3, -1))
    sp = _all_liquid(pp, rho2.reshape(-1), u2.reshape(3, -1))
    oracle.step(pw, sw, 40)
    oracle.step(pp, sp, 40)
    fw = sw.f.reshape(19, nz, ny, nx)
    fp = sp.f.reshape(19, nz, 2 * ny, nx)
    np.testing.assert_allclose(fw, fp[:, :, :ny, :], rtol=0, atol=1e-14)
    # and the mirror half is the reflection of the first
    np.testing.assert_allclose(fp[MIRROR_Y][:, :, ::-1, :][:, :, :ny, :], fp[:, :, :ny, :], rtol=0,
                               atol=1e-14)
    # the mirror test has teeth: with no-slip walls it fails
    pn = oracle.Params(nx, ny, nz, periodic=(1, 0, 1), collision=collision, omega=1.7, g=g)
    sn = _all_liquid(pn, rho.reshape(-1), u.reshape(3, -1))
    oracle.step(pn, sn, 40)
    assert np.abs(sn.f.reshape(19, nz, ny, nx) - fp[:, :, :ny, :]).max() > 1e-6


def test_body_force_flow_between_free_slip_walls_is_a_plug():
    nx, ny, nz, g, t = 4, 8, 6, 1e-5, 100
    for free_slip in (1, 0):
        p = oracle.Params(nx, ny, nz, periodic=(1, 0, 0), collision=1, omega=1.6,
                          g=(g, 0.0, 0.0), free_slip=free_slip)
        st = _all_liquid(p, np.ones(p.N), np.zeros((3, p.N)))
        oracle.step(p, st, t)
        cx = np.array([c[0] for c in D3Q19], dtype=np.float64)
        jx = (st.f * cx[:, None]).sum(0)      # post-collision momentum: t collisions of F = rho g
        rho = st.f.sum(0)
        if free_slip:
            assert np.ptp(jx) < 1e-15 and np.ptp(rho) < 1e-14
            assert abs(jx.mean() - t * g) <= 1e-12 * t * g
        else:
            assert np.ptp(jx) > 1e-3 * t * g   # walls drag: no plug


@pytest.mark.parametrize("scheme", [0, 2, 4])
def test_free_surface_mass_with_free_slip_walls(scheme):
    s = setups.rect_dam_break(40, 6, 24, width=12, height=16, g=2e-4, refill=scheme)
    p = oracle_params(s, free_slip=1)
    st = oracle_state(s, p)
    m0 = oracle.total_mass(p, st)
    oracle.step(p, st, 200)
    m1 = oracle.total_mass(p, st)
    assert abs(m1 - m0) <= 1e-12 * m0
    assert st.counts is not None


def test_paper_dam_break_setup():
    """The Sec. 4.2 dam break: 15W x 1 x 2H with H = 2W, the column W x H at
    x = 0, SRT, and gravity from the Galilei number Ga = g W^3 / nu^2 with the
    lattice viscosity nu = (1/omega - 1/2) / 3."""
    W, omega, Ga = 50, 1.9995, 1.83e9
    s = setups.paper_dam_break(W=W)
    assert (s.nx, s.ny, s.nz) == (15 * W, 1, 4 * W) and s.collision == 0 and s.omega == omega
    nu = (1.0 / omega - 0.5) / 3.0
    assert abs(-s.g[2] * W ** 3 / nu ** 2 / Ga - 1.0) < 1e-14 and s.g[:2] == (0.0, 0.0)
    phi = s.phi.reshape(s.nz, s.ny, s.nx)
    assert phi[: 2 * W - 1, 0, : W - 1].min() == 1.0       # inside the column
    assert phi[2 * W + 1:, 0, :].max() == 0.0 and phi[:, 0, W + 1:].max() == 0.0
    assert abs(phi.sum() - W * 2 * W) <= 1.0                # its volume, up to the top layer


def test_single_cell_layer_between_free_slip_walls_stays_mirror_symmetric():
    """One cell layer between free-slip walls in y (the paper's two-dimensional
    dam break): a population moving up in y is reflected into the one moving
    down, so a y-symmetric start stays y-symmetric, f_i = f_mirror(i) up to
    rounding; mass is conserved; the column collapses (the front advances).
    Small dam break with the turbulence model, 150 steps."""
    s = setups.paper_dam_break(W=10, galilei=5.8e7)
    p = oracle_params(s, free_slip=1, smag_cs=0.1)
    st = oracle_state(s, p)
    m0 = oracle.total_mass(p, st)
    oracle.step(p, st, 150)
    fluid = st.flags != 4
    np.testing.assert_allclose(st.f[MIRROR_Y][:, fluid], st.f[:, fluid], rtol=0, atol=1e-14)
    assert abs(oracle.total_mass(p, st) - m0) <= 1e-12 * m0
    fl = st.flags.reshape(s.nz, s.nx)
    assert np.nonzero(fl[0] != 4)[0].max() + 1 > 12
    # a y-asymmetric start does not stay symmetric by accident: the test sees
    # a sign error in the reflection
    st2 = oracle_state(s, p)
    st2.f[3] += 1e-4 * (st2.flags != 4)
    oracle.step(p, st2, 5)
    fluid = st2.flags != 4
    assert np.abs(st2.f[MIRROR_Y][:, fluid] - st2.f[:, fluid]).max() > 1e-7
