"""Observables of the dam-break and drop-impact runs, read off the library's
canonical fields (flags, fill level).  Nothing here steps the method.

Dam break (Sec. 4.2 of the paper, monitored quantities): the front position is
the extent of the fluid along x in the bottom cell layer, the residual height
the extent of the fluid along z at the x = 0 wall.  The paper tracks the
rightmost and uppermost interface cell; with a closed interface layer that is
the last fluid (liquid or interface) cell, counted here as a cell count
(index + 1, 0 if there is none).

Drop impact (Sec. 4.5 setup): the liquid height of the centre column
(sum over z of the fill level) and the depth of the cavity below the pool's
initial surface along that column."""
from __future__ import annotations

import torch

LIQUID, INTERFACE = 1, 2


def _fluid(flags: torch.Tensor) -> torch.Tensor:
    return (flags & (LIQUID | INTERFACE)) != 0


def front_position(flags: torch.Tensor, nx: int, ny: int, nz: int) -> int:
    """Largest x + 1 of a fluid cell in the layer z = 0 (any y); flags [N]."""
    f = _fluid(flags.reshape(nz, ny, nx)[0]).any(0)          # [nx]
    idx = torch.nonzero(f)
    return int(idx.max()) + 1 if idx.numel() else 0


def residual_height(flags: torch.Tensor, nx: int, ny: int, nz: int) -> int:
    """Largest z + 1 of a fluid cell at the wall x = 0 (any y); flags [N]."""
    f = _fluid(flags.reshape(nz, ny, nx)[:, :, 0]).any(1)    # [nz]
    idx = torch.nonzero(f)
    return int(idx.max()) + 1 if idx.numel() else 0


def column_height(phi: torch.Tensor, nx: int, ny: int, nz: int, x: int, y: int) -> float:
    """Sum over z of the fill level of column (x, y); phi [N]."""
    return float(phi.reshape(nz, ny, nx)[:, y, x].sum())


def cavity_depth(phi: torch.Tensor, nx: int, ny: int, nz: int, x: int, y: int, depth: float) -> float:
    """How far below the pool's initial surface z = depth the fluid of column
    (x, y) ends: depth minus the lowest z whose fill level is below 1/2 (0 if
    the column is filled up to the surface)."""
    col = phi.reshape(nz, ny, nx)[:, y, x]
    low = torch.nonzero(col < 0.5)
    if not low.numel():
        return 0.0
    return max(0.0, depth - float(low.min()))
