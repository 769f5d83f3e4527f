"""Pins of the oracle's Smagorinsky turbulence model (Sec. 2.1, turbulence
model; reading R29).

* Without a non-equilibrium part the relaxation rate is the user-chosen one.
* The relaxation time solves the model's defining relation
  nu_t = c_s^2 (tau - tau0) = (C_S dx)^2 S,  S = Qbar / (2 rho c_s^2 tau),
  for arbitrary populations (Qbar computed here from the populations).
* Physics: in a resolved shear wave the strain rate the model reads off the
  post-streaming populations, Qbar / (2 rho c_s^2 tau), equals the measured
  velocity gradient |du_x/dy| (Chapman-Enskog), so the model's
  viscosity is the Smagorinsky one, (C_S dx)^2 |S|.
* The model raises the viscosity of a decaying shear wave by the predicted
  amount; with C_S = 0 the collision is the plain one.
"""
import numpy as np
import pytest

import oracle
from _util import LIQ

CS2 = 1.0 / 3.0
D3Q19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
         (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
C = np.array(D3Q19, dtype=np.float64)


def _qbar(f, feq):
    ne = f - feq
    Qm = np.einsum("i,ia,ib->ab", ne, C, C)
    return np.sqrt(2.0 * np.sum(Qm * Qm))


@pytest.mark.parametrize("collision", [0, 1])
def test_equilibrium_keeps_the_chosen_relaxation_rate(collision):
    p = oracle.Params(4, 4, 4, collision=collision, omega=1.9, smag_cs=0.1)
    for u in ((0.0, 0.0, 0.0), (0.03, -0.01, 0.02)):
        f = oracle.feq(1.02, u)
        assert abs(oracle.cell_omega(p, f, g=(0.0, 0.0, 0.0)) - 1.9) <= 4e-16


@pytest.mark.parametrize("seed", range(5))
def test_relaxation_time_solves_the_model_relation(seed):
    rng = np.random.default_rng(seed)
    omega, cs = 1.95, 0.1 + 0.3 * rng.random()
    p = oracle.Params(4, 4, 4, omega=omega, smag_cs=cs)
    rho = 1.0 + 0.05 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    feq = oracle.feq(rho, u)
    f = feq + 1e-3 * rng.standard_normal(19)
    # the equilibrium the collision relaxes to is that of f's own moments
    r = f.sum()
    uf = (C * f[:, None]).sum(0) / r
    feq_f = oracle.feq(r, uf)
    tau = 1.0 / oracle.cell_omega(p, f, g=(0.0, 0.0, 0.0))
    tau0 = 1.0 / omega
    S = _qbar(f, feq_f) / (2.0 * r * CS2 * tau)
    lhs, rhs = CS2 * (tau - tau0), cs * cs * S
    assert tau > tau0
    assert abs(lhs - rhs) <= 1e-12 * rhs


def _shear_wave(ny, omega, U, cs, steps):
    p = oracle.Params(1, ny, 1, periodic=(1, 1, 1), omega=omega, smag_cs=cs)
    y = np.arange(ny) + 0.5
    k = 2 * np.pi / ny
    u = np.zeros((3, ny))
    u[0] = U * np.sin(k * y)
    st = oracle.init_state(p, np.full(ny, LIQ, np.uint8), np.ones(ny), np.ones(ny), u)
    oracle.step(p, st, steps)
    return p, st, k, y


def test_strain_rate_read_from_the_populations_is_the_velocity_gradient():
    ny, omega, U, cs = 128, 1.9, 0.02, 0.4
    p, st, k, y = _shear_wave(ny, omega, U, cs, 60)
    # stream the post-collision populations (periodic pull) to get what the
    # next collision sees
    fps = np.empty_like(st.f)
    for i, (cx, cy, cz) in enumerate(D3Q19):
        fps[i] = np.roll(st.f[i], cy)
    rho = fps.sum(0)
    ux = (fps * C[:, 0:1]).sum(0) / rho
    dudy = (np.roll(ux, -1) - np.roll(ux, 1)) / 2.0
    ok = 0
    for n in range(ny):
        if abs(np.cos(k * y[n])) < 0.5:
            continue
        f = fps[:, n]
        uf = (C * f[:, None]).sum(0) / rho[n]
        tau = 1.0 / oracle.cell_omega(p, f, g=(0.0, 0.0, 0.0))
        S = _qbar(f, oracle.feq(rho[n], uf)) / (2.0 * rho[n] * CS2 * tau)
        assert abs(S / abs(dudy[n]) - 1.0) < 0.01, (n, S, dudy[n])
        ok += 1
    assert ok > ny // 2


def test_model_raises_the_shear_wave_viscosity_by_the_smagorinsky_amount():
    """Decay of a shear wave with and without the model; the extra viscosity
    averaged over the wave, (C_S dx)^2 <|du/dy| sin^2>/<sin^2>, predicts the
    faster decay of the amplitude to a few percent."""
    ny, omega, U, cs = 64, 1.9, 0.02, 0.4
    k = 2 * np.pi / ny
    amps = {}
    for c in (0.0, cs):
        p, st, k, y = _shear_wave(ny, omega, U, c, 0)
        a = []
        for t in (100, 200):
            oracle.step(p, st, 100)
            _, uu = oracle.macroscopic(p, st)
            a.append(2.0 / ny * np.sum(uu[0] * np.sin(k * y)))
        amps[c] = a
    nu0 = CS2 * (1.0 / omega - 0.5)
    nu_plain = np.log(amps[0.0][0] / amps[0.0][1]) / (k * k * 100)
    nu_les = np.log(amps[cs][0] / amps[cs][1]) / (k * k * 100)
    assert abs(nu_plain / nu0 - 1) < 1e-3
    # energy-weighted eddy viscosity of the mode at the mean amplitude
    A = np.sqrt(amps[cs][0] * amps[cs][1])
    yy = (np.arange(ny) + 0.5) * k
    nut = cs * cs * A * k * np.mean(np.abs(np.cos(yy)) * np.cos(yy) ** 2) / np.mean(np.cos(yy) ** 2)
    assert nu_les > nu_plain
    assert abs((nu_les - nu_plain) / nut - 1) < 0.05, (nu_les - nu_plain, nut)
