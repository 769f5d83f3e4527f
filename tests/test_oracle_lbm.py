"""Pins of the oracle's lattice Boltzmann core (Sec. 2.1) against closed forms,
invariants and an independent textbook D2Q9 solver."""
import itertools

import numpy as np
import pytest

import oracle
from _util import LIQ

CS2 = 1.0 / 3.0


def test_lattice_isotropy():
    c, w, op = oracle.lattice()
    assert abs(w.sum() - 1.0) < 1e-15
    I = np.eye(3)
    # second and fourth order isotropy of D3Q19 (Krueger et al., textbook)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2, CS2 * I, atol=1e-15)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) * CS2 ** 2
    assert np.allclose(M4, iso, atol=1e-15)
    assert np.all(c[op] == -c)
    assert np.all(np.einsum("i,ia->a", w, c) == 0)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 3)
    c, _, _ = oracle.lattice()
    fe = oracle.feq(rho, u)
    assert abs(fe.sum() - rho) < 1e-15
    assert np.allclose(c.T @ fe, rho * u, atol=1e-15)
    P = np.einsum("i,ia,ib->ab", fe, c, c)
    assert np.allclose(P, rho * (CS2 * np.eye(3) + np.outer(u, u)), atol=1e-15)


@pytest.mark.parametrize("collision,seed", itertools.product([0, 1], range(4)))
def test_collision_conserves_mass_adds_force(collision, seed):
    """Collision keeps rho; momentum grows by exactly F = rho g (Guo forcing)."""
    rng = np.random.default_rng(100 + seed)
    c, _, _ = oracle.lattice()
    g = rng.uniform(-1e-3, 1e-3, 3)
    f = oracle.feq(rng.uniform(0.9, 1.1), rng.uniform(-0.05, 0.05, 3)) + rng.uniform(-1e-3, 1e-3, 19)
    p = oracle.Params(1, 1, 1, collision=collision, omega=rng.uniform(0.6, 1.95), g=tuple(g))
    fs = oracle.collide(p, f)
    rho = f.sum()
    assert abs(fs.sum() - rho) < 1e-15
    assert np.allclose(c.T @ fs - c.T @ f, rho * g, atol=1e-16)


def test_collision_equilibrium_fixed_point():
    u = np.array([0.03, -0.02, 0.01])
    f = oracle.feq(1.02, u)
    for collision in (0, 1):
        p = oracle.Params(1, 1, 1, collision=collision, omega=1.3)
        assert np.allclose(oracle.collide(p, f), f, atol=1e-16)


@pytest.mark.parametrize("omega", [0.7, 1.3, 1.9])
def test_trt_reduces_to_srt(omega):
    """omega- = omega+ (Lambda = (1/omega - 1/2)^2) turns TRT into SRT."""
    rng = np.random.default_rng(7)
    f = oracle.feq(1.0, [0.02, 0.01, -0.03]) + rng.uniform(-1e-3, 1e-3, 19)
    lam = (1.0 / omega - 0.5) ** 2
    g = (1e-4, -2e-4, 3e-5)
    s = oracle.collide(oracle.Params(1, 1, 1, collision=0, omega=omega, g=g), f)
    t = oracle.collide(oracle.Params(1, 1, 1, collision=1, omega=omega, trt_lambda=lam, g=g), f)
    assert np.max(np.abs(s - t)) < 1e-15


def _all_liquid(p, rho, u):
    N = p.N
    flags = np.full(N, LIQ, np.uint8)
    return oracle.init_state(p, flags, np.ones(N), rho, u)


def test_shear_wave_decay():
    """u_x = U sin(k y) decays as exp(-nu k^2 t), nu = c_s^2 (1/omega - 1/2)."""
    ny, omega, U = 64, 1.2, 1e-4
    p = oracle.Params(1, ny, 1, periodic=(1, 1, 1), omega=omega)
    k = 2 * np.pi / ny
    y = np.arange(ny) + 0.5
    u = np.zeros((3, ny))
    u[0] = U * np.sin(k * y)
    st = _all_liquid(p, np.ones(ny), u)
    amps = []
    for t1 in (200, 400):
        oracle.step(p, st, t1 - (200 if amps else 0))
        _, uu = oracle.macroscopic(p, st)
        amps.append(2.0 / ny * np.sum(uu[0] * np.sin(k * y)))
    nu_meas = np.log(amps[0] / amps[1]) / (k * k * 200)
    nu = CS2 * (1.0 / omega - 0.5)
    assert abs(nu_meas / nu - 1) < 1e-3


def test_poiseuille_trt_exact():
    """Force-driven channel between half-way bounce-back walls: TRT with
    Lambda = 3/16 gives the parabola u = g/(2 nu) y (H - y) exactly."""
    H, omega, gx = 12, 1.0, 1e-6
    p = oracle.Params(1, H, 1, periodic=(1, 0, 1), collision=1, omega=omega, g=(gx, 0, 0))
    st = _all_liquid(p, np.ones(H), np.zeros((3, H)))
    oracle.step(p, st, 6000)
    _, u = oracle.macroscopic(p, st)
    y = np.arange(H) + 0.5
    nu = CS2 * (1.0 / omega - 0.5)
    ref = gx / (2 * nu) * y * (H - y)
    assert np.max(np.abs(u[0] - ref)) / ref.max() < 1e-9
    assert np.max(np.abs(u[1:])) < 1e-13


def _d2q9_reference(f2, omega, g, steps):
    """Textbook D2Q9 SRT with Guo forcing on a periodic grid (Krueger et al.)."""
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    g = np.asarray(g)
    for _ in range(steps):
        # stream f*(x) -> f(x + c)
        f2 = np.stack([np.roll(np.roll(f2[i], c[i, 0], axis=1), c[i, 1], axis=0) for i in range(9)])
        rho = f2.sum(0)
        j = np.einsum("ia,iyx->ayx", c, f2)
        F = rho[None] * g[:, None, None]
        u = (j + 0.5 * F) / rho[None]
        cu = np.einsum("ia,ayx->iyx", c, u)
        uu = (u * u).sum(0)
        feq = w[:, None, None] * rho[None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu[None])
        cF = np.einsum("ia,ayx->iyx", c, F)
        uF = (u * F).sum(0)
        Fi = (1 - omega / 2) * w[:, None, None] * (3 * (cF - uF[None]) + 9 * cu * cF)
        f2 = f2 - omega * (f2 - feq) + Fi
    return f2


def test_d3q19_single_layer_equals_d2q9():
    """With nz = 1 and periodic z, summing the D3Q19 populations over c_z gives
    a D2Q9 lattice Boltzmann run (weights 4/9, 1/9, 1/36)."""
    nx, ny, omega = 8, 6, 1.4
    g = (2e-4, -1e-4)
    rng = np.random.default_rng(3)
    rho = 1 + rng.uniform(-0.01, 0.01, nx * ny)
    u = np.zeros((3, nx * ny))
    u[:2] = rng.uniform(-0.03, 0.03, (2, nx * ny))
    p = oracle.Params(nx, ny, 1, periodic=(1, 1, 1), omega=omega, g=(g[0], g[1], 0.0))
    st = _all_liquid(p, rho, u)
    c3, _, _ = oracle.lattice()
    c2 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]

    def project(f):
        out = np.zeros((9, ny, nx))
        for i in range(19):
            k = c2.index((int(c3[i, 0]), int(c3[i, 1])))
            out[k] += f[i].reshape(ny, nx)
        return out

    f2 = project(st.f)
    oracle.step(p, st, 15)
    ref = _d2q9_reference(f2, omega, g, 15)
    assert np.max(np.abs(project(st.f) - ref)) < 1e-14
