"""Differentiable interface-height loss of the FSLBM behind ``torch.autograd``.

``height_loss`` runs a window of T FSLBM steps on the GPU (the library's
checkpointed forward) and returns, per domain b,

    L_b = (1/T) sum_{t=1..T} (h_b(t) - h*_b(t))^2,
    h_b(t) = sum of the fill level over the plane x = x_probe.

Its backward is the library's hand-written adjoint (``fslbm_adjoint_backward``)
with the cell-type sequence of the forward run held fixed.  Gradients flow to
omega [B], gravity [B, 3] and the start state (pdf, mass, phi); the start state
itself may be a differentiable function of shape parameters, as in
``standing_wave_state`` where phi0 depends on the wave amplitude a0.
The paper does not differentiate the method; this is an addition on top of the
FP64, SRT, EQ-refilling, sigma = 0 configuration of its standing wave
(Sec. 4.1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import fslbm, setups


@dataclass
class Window:
    """Geometry and loss window shared by every domain of a batch."""
    nx: int
    ny: int
    nz: int
    periodic: tuple
    nsteps: int
    x_probe: int
    n_checkpoints: int = 0      # 0: ceil(sqrt(nsteps))
    p_volume: float = 1.0 / 3.0
    eps_phi: float = 1e-2


class _HeightLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega, gravity, pdf0, mass0, phi0, flags, target, win: Window):
        B = omega.shape[0]
        params = fslbm.Params(win.nx, win.ny, win.nz, B, tuple(win.periodic), fslbm.SRT, fslbm.F64,
                              fslbm.REFILL_EQ, float(omega[0]), gravity=tuple(gravity[0].tolist()),
                              p_volume=win.p_volume, eps_phi=win.eps_phi,
                              omega_b=tuple(omega.detach().cpu().tolist()),
                              gravity_b=tuple(tuple(r) for r in gravity.detach().cpu().tolist()))
        sim = fslbm.Simulation(params, flags, phi0.detach(), pdf=pdf0.detach(), mass=mass0.detach(),
                               device=pdf0.device)
        loss, height = sim.adjoint_forward(target, win.nsteps, win.x_probe, win.n_checkpoints)
        ctx.sim = sim
        ctx.height = height
        ctx.dev = omega.device
        return torch.as_tensor(loss, dtype=torch.float64, device=omega.device)

    @staticmethod
    def backward(ctx, gloss):
        g = ctx.sim.adjoint_backward(gloss.detach().to("cpu", torch.float64).numpy())
        dev = ctx.dev
        return (torch.as_tensor(g["omega"], device=dev), torch.as_tensor(g["gravity"], device=dev),
                g["pdf"], g["mass"], g["phi"], None, None, None)


def height_loss(omega, gravity, pdf0, mass0, phi0, flags, target, win: Window):
    """Per-domain loss [B] (float64).  omega [B], gravity [B, 3], pdf0 [B, 19, N],
    mass0 [B, N], phi0 [B, N] are float64 (pdf0/mass0/phi0 on the GPU); flags
    [B, N] uint8 are held fixed; target [B, nsteps] is h*(1..nsteps)."""
    return _HeightLoss.apply(omega, gravity, pdf0, mass0, phi0, flags, target, win)


# ------------------------------------------------------------------ standing wave

def standing_wave_phi(amplitude: torch.Tensor, flags: torch.Tensor, nx: int, ny: int,
                      depth: float, sub: int = 8) -> torch.Tensor:
    """Fill level [B, N] of the 2-D standing wave eta(x) = depth + a cos(2 pi x / nx)
    as a differentiable function of the amplitudes a [B]: the same sub-sampled
    volume fraction as ``setups.height_fill`` (exact in y, ``sub``-point midpoint
    rule in x), with liquid cells at 1 and gas cells at 0 as ``flags`` says."""
    dev = amplitude.device
    k = 2.0 * np.pi / nx
    xs = (np.arange(nx, dtype=np.float64) + 0.5)[:, None] + ((np.arange(sub) + 0.5) / sub - 0.5)[None, :]
    cosv = torch.as_tensor(np.cos(k * xs), dtype=torch.float64, device=dev)          # [nx, sub]
    eta = depth + amplitude[:, None, None] * cosv[None]                               # [B, nx, sub]
    lo = torch.arange(ny, dtype=torch.float64, device=dev)
    frac = torch.clamp(eta[:, None, :, :] - lo[None, :, None, None], 0.0, 1.0).mean(dim=3)  # [B, ny, nx]
    phi = frac.reshape(amplitude.shape[0], ny * nx)
    one, zero = torch.ones_like(phi), torch.zeros_like(phi)
    fl = flags.to(dev)
    return torch.where(fl == fslbm.LIQUID, one, torch.where(fl == fslbm.GAS, zero, phi))


def standing_wave_state(amplitude: torch.Tensor, nx: int, ny: int, depth: float, device="cuda"):
    """Start state of a batch of standing waves (rest fluid, rho = 1).  Cell types
    come from each domain's amplitude and are then fixed; phi0 and the interface
    mass m0 = phi0 rho0 are differentiable in the amplitudes; f* = f_eq(1, 0).
    Returns (flags [B, N] uint8, pdf0 [B, 19, N], mass0 [B, N], phi0 [B, N])."""
    B = amplitude.shape[0]
    N = nx * ny
    flags = np.stack([setups.standing_wave(nx=nx, ny=ny, depth=depth, amplitude=float(a)).flags
                      for a in amplitude.detach().cpu().tolist()])
    flags_t = torch.as_tensor(flags, device=device)
    phi0 = standing_wave_phi(amplitude.to(device), flags_t, nx, ny, depth)
    mass0 = torch.where(flags_t == fslbm.INTERFACE, phi0, torch.zeros_like(phi0))
    w = torch.tensor([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=torch.float64,
                     device=device)
    fluid = (flags_t != fslbm.GAS).to(torch.float64)
    pdf0 = w[None, :, None] * fluid[:, None, :]
    return flags_t, pdf0.reshape(B, 19, N).contiguous(), mass0, phi0
