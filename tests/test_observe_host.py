"""The dam-break and drop-impact observables on hand-built fields (no GPU)."""
import torch

from paper_2207_14496_amd import observe

LIQ, IFC, GAS = 1, 2, 4


def _flags(nx, ny, nz):
    return torch.full((nz, ny, nx), GAS, dtype=torch.uint8)


def test_front_and_residual_height():
    nx, ny, nz = 16, 3, 8
    f = _flags(nx, ny, nz)
    f[:5, :, :4] = LIQ          # column x < 4, z < 5
    f[5, :, :4] = IFC           # its top layer
    f[0, 1, 4:9] = IFC          # a tongue along the bottom in one y row
    assert observe.front_position(f.reshape(-1), nx, ny, nz) == 9
    assert observe.residual_height(f.reshape(-1), nx, ny, nz) == 6
    # fluid above the bottom layer does not move the front
    f[3, 0, 12] = IFC
    assert observe.front_position(f.reshape(-1), nx, ny, nz) == 9
    # no fluid at all
    g = _flags(nx, ny, nz)
    assert observe.front_position(g.reshape(-1), nx, ny, nz) == 0
    assert observe.residual_height(g.reshape(-1), nx, ny, nz) == 0


def test_column_height_and_cavity_depth():
    nx, ny, nz = 5, 4, 20
    phi = torch.zeros((nz, ny, nx), dtype=torch.float64)
    phi[:10, 2, 3] = 1.0
    phi[10, 2, 3] = 0.25
    assert observe.column_height(phi.reshape(-1), nx, ny, nz, 3, 2) == 10.25
    # pool surface at z = 12: the column ends 2 cells below it (first cell
    # with phi < 1/2 is z = 10)
    assert observe.cavity_depth(phi.reshape(-1), nx, ny, nz, 3, 2, 12.0) == 2.0
    # a column filled above the surface has no cavity
    phi[:, 1, 1] = 1.0
    assert observe.cavity_depth(phi.reshape(-1), nx, ny, nz, 1, 1, 12.0) == 0.0
    # a drop above a crater: the lowest cell below 1/2 decides
    phi[:4, 0, 0] = 1.0
    phi[15:18, 0, 0] = 1.0
    assert observe.cavity_depth(phi.reshape(-1), nx, ny, nz, 0, 0, 12.0) == 8.0
