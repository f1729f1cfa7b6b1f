"""GPU parity of the fused 3D field solve (power-of-two grids, transforms in
LDS) against the oracle's FFT solve of the same charge, and against the
library-transform path of the same library on the same input (forced with
APIC_FIELD_FFT=library at context creation): E, its binary32 rounding and
the field energy, for FP64 charge densities and for the mixed path's
fixed-point accumulation (whose buffer the standalone solve leaves intact),
on cubic and elongated grids from 4 to 256 nodes per axis (the z work split
changes at 256 nodes along z)."""
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 4), (8, 16, 4), (32, 8, 64), (64, 64, 64), (128, 128, 128), (8, 8, 256), (256, 8, 16),
          (16, 256, 8)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


def _dims(nx, ny, nz):
    return nx * 0.83, ny * 1.21, nz * 0.97


def _ctx(nx, ny, nz, precision, library=False):
    from paper_2608_15249_amd.apic import Context
    lx, ly, lz = _dims(nx, ny, nz)
    old = os.environ.pop("APIC_FIELD_FFT", None)
    if library:
        os.environ["APIC_FIELD_FFT"] = "library"
    try:
        return Context(dim=3, vdim=3, nx=nx, ny=ny, lx=lx, ly=ly, dt=0.1, n=4096, precision=precision,
                       tile=(min(nx, 4), min(ny, 4), min(nz, 4)), nz=nz, lz=lz)
    finally:
        os.environ.pop("APIC_FIELD_FFT", None)
        if old is not None:
            os.environ["APIC_FIELD_FFT"] = old


def _setup(nx, ny, nz):
    lx, ly, lz = _dims(nx, ny, nz)
    return O.Setup(3, 3, nx, lx, 4096, 0.1, ny=ny, Ly=ly, nz=nz, Lz=lz)


def _solve(torch, c, rho_dev):
    E = torch.zeros(3 * c.G, dtype=torch.float64, device="cuda")
    E32 = torch.zeros(3 * c.G, dtype=torch.float32, device="cuda")
    we = torch.zeros(1, dtype=torch.float64, device="cuda")
    c.field_solve(rho_dev, E, E32, we)
    c.sync()
    return E.cpu().numpy(), E32.cpu().numpy(), float(we.item())


@pytest.mark.parametrize("nx,ny,nz", SHAPES)
def test_fused_solve_3d_fp64_matches_oracle_and_library(torch, nx, ny, nz):
    rng = np.random.default_rng(5000 + nx + 3 * ny + 7 * nz)
    s = _setup(nx, ny, nz)
    rho = rng.normal(size=s.grid_shape) + 0.3
    Eo = np.stack(O.solve_field(s, rho))
    scale = np.max(np.abs(Eo))
    dev = torch.from_numpy(rho.ravel().copy()).cuda()
    Ef, Ef32, wef = _solve(torch, _ctx(nx, ny, nz, "fp64"), dev)
    El, _, wel = _solve(torch, _ctx(nx, ny, nz, "fp64", library=True), dev)
    assert np.max(np.abs(Ef.reshape(Eo.shape) - Eo)) <= 1e-13 * scale
    assert np.max(np.abs(Ef - El)) <= 1e-13 * scale
    assert np.array_equal(Ef32, Ef.astype(np.float32))
    assert abs(wef / O.field_energy(s, tuple(Eo)) - 1) <= 1e-12
    assert abs(wef / wel - 1) <= 1e-13


@pytest.mark.parametrize("nx,ny,nz", [(16, 8, 32), (128, 128, 128), (8, 8, 256)])
def test_fused_solve_3d_fixed_point_accumulation(torch, nx, ny, nz):
    """Mixed path: the int64 fixed-point accumulation (scale 2^-3S per unit)
    with the ion background, against the oracle's solve of the same charge
    converted in FP64."""
    rng = np.random.default_rng(6000 + nx + nz)
    c = _ctx(nx, ny, nz, "mixed")
    S = c.frac_bits
    s = _setup(nx, ny, nz)
    I = rng.integers(0, min(40 << (3 * S), 1 << 56), size=s.grid_shape, dtype=np.int64)
    Eo = np.stack(O.solve_field(s, O.rho_from_quantised(s, I, S)))
    dev = torch.from_numpy(I.ravel().copy()).cuda()
    E, E32, we = _solve(torch, c, dev)
    assert np.max(np.abs(E.reshape(Eo.shape) - Eo)) <= 1e-12 * np.max(np.abs(Eo))
    assert np.array_equal(E32, E.astype(np.float32))
    assert abs(we / O.field_energy(s, tuple(Eo)) - 1) <= 1e-11
    assert np.array_equal(dev.cpu().numpy(), I.ravel())
