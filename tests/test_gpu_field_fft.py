"""GPU parity of the fused 2D field solve (power-of-two grids, three
launches) against the oracle's FFT solve of the same charge, and against the
library-transform path of the same library on the same input (forced with
APIC_FIELD_FFT=library at context creation): E, its binary32 rounding, the
field energy and the charge, for FP64 charge densities and for the mixed
path's fixed-point accumulation, square and elongated grids from 4 to 1024
nodes per axis, and the grounded-wall extension."""
import os

import numpy as np
import pytest

import oracle as O
from oracle import bounded as B

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (8, 32), (64, 16), (128, 128), (512, 512), (1024, 8), (16, 1024), (1024, 1024)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


def _ctx(nx, ny, precision, walls=False, library=False):
    from paper_2608_15249_amd.apic import Context
    old = os.environ.pop("APIC_FIELD_FFT", None)
    if library:
        os.environ["APIC_FIELD_FFT"] = "library"
    try:
        return Context(dim=2, vdim=2, nx=nx, ny=ny, lx=nx * 0.83, ly=ny * 1.21, dt=0.1, n=1024, precision=precision,
                       tile=(min(nx, 4), min(ny, 4)), walls=walls)
    finally:
        os.environ.pop("APIC_FIELD_FFT", None)
        if old is not None:
            os.environ["APIC_FIELD_FFT"] = old


def _solve(torch, c, rho_dev, with32=True):
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.zeros(2 * c.G, dtype=torch.float32, device="cuda") if with32 else None
    we = torch.zeros(1, dtype=torch.float64, device="cuda")
    c.field_solve(rho_dev, E, E32, we)
    c.sync()
    return E.cpu().numpy(), (E32.cpu().numpy() if with32 else None), float(we.item())


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_fused_solve_fp64_matches_oracle_and_library(torch, nx, ny):
    rng = np.random.default_rng(1000 + nx + 7 * ny)
    rho = rng.normal(size=(ny, nx)) + 0.3
    s = O.Setup(2, 2, nx, nx * 0.83, 1024, 0.1, ny=ny, Ly=ny * 1.21)
    Eo = np.stack(O.solve_field(s, rho))
    scale = np.max(np.abs(Eo))
    dev = torch.from_numpy(rho.ravel().copy()).cuda()
    c = _ctx(nx, ny, "fp64")
    Ef, Ef32, wef = _solve(torch, c, dev)
    cl = _ctx(nx, ny, "fp64", library=True)
    El, _, wel = _solve(torch, cl, dev)
    Ef = Ef.reshape(2, ny, nx)
    assert np.max(np.abs(Ef - Eo)) <= 1e-13 * scale
    assert np.max(np.abs(Ef - El.reshape(2, ny, nx))) <= 1e-13 * scale
    assert np.array_equal(Ef32, Ef.ravel().astype(np.float32))
    we_o = 0.5 * s.dV * float(np.sum(Eo ** 2))
    assert abs(wef / we_o - 1) <= 1e-12
    assert abs(wef / wel - 1) <= 1e-13


@pytest.mark.parametrize("nx,ny", [(8, 32), (512, 512), (1024, 1024)])
def test_fused_solve_fixed_point_accumulation(torch, nx, ny):
    """Mixed path: the int64 fixed-point accumulation of CIC weights (scale
    2^-2S per unit) with the ion background, against the oracle's solve of the
    same charge converted in FP64; the standalone solve leaves the buffer
    intact."""
    rng = np.random.default_rng(2000 + nx)
    c = _ctx(nx, ny, "mixed")
    S = c.frac_bits
    I = rng.integers(0, 40 << (2 * S), size=(ny, nx), dtype=np.int64)
    s = O.Setup(2, 2, nx, nx * 0.83, 1024, 0.1, ny=ny, Ly=ny * 1.21)
    rho = O.rho_from_quantised(s, I, S)
    Eo = np.stack(O.solve_field(s, rho))
    dev = torch.from_numpy(I.ravel().copy()).cuda()
    E, E32, we = _solve(torch, c, dev)
    assert np.max(np.abs(E.reshape(2, ny, nx) - Eo)) <= 1e-12 * np.max(np.abs(Eo))
    assert abs(we / (0.5 * s.dV * float(np.sum(Eo ** 2))) - 1) <= 1e-11
    assert np.array_equal(dev.cpu().numpy(), I.ravel())


@pytest.mark.parametrize("nx,ny", [(32, 16), (256, 64), (512, 512)])
def test_fused_solve_with_walls(torch, nx, ny):
    """Grounded walls: the odd extension to 2 nx nodes along x is a power of
    two, so the fused path solves it; against the oracle's sine-transform
    solve and the library path."""
    rng = np.random.default_rng(3000 + nx)
    b = B.Box(nx, nx * 0.83, ny, ny * 1.21, 1024, 0.1)
    rho = rng.normal(size=(ny, nx + 1))
    ext = np.zeros((ny, 2 * nx))
    ext[:, :nx + 1] = rho
    dev = torch.from_numpy(ext.ravel().copy()).cuda()
    c = _ctx(nx, ny, "fp64", walls=True)
    E, _, we = _solve(torch, c, dev, with32=False)
    cl = _ctx(nx, ny, "fp64", walls=True, library=True)
    El, _, wel = _solve(torch, cl, dev, with32=False)
    Eo = B.solve_field(b, rho)
    Eg = E.reshape(2, ny, 2 * nx)[:, :, :nx + 1]
    scale = max(np.max(np.abs(e)) for e in Eo)
    for d in range(2):
        assert np.max(np.abs(Eg[d] - Eo[d])) <= 1e-12 * scale
    assert np.max(np.abs(E - El)) <= 1e-13 * scale
    assert abs(we / B.field_energy(b, Eo) - 1) <= 1e-11
    assert abs(we / wel - 1) <= 1e-13
