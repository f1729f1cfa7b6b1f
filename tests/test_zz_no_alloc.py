"""GPU test of apic_step_static, the step that allocates nothing (its
workspace is the library's fixed device array): two calls in a row on two
plasmas, the second smaller, each against apic_step with a caller-allocated
workspace on an identical copy of the same state; bit for bit on the mixed
path (fixed-point deposit, deterministic slots), to rounding on the FP64
path. A context whose workspace exceeds the array is rejected."""

import numpy as np
import pytest

from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


def _pair(torch, w, precision, tile):
    """Two identical initialised simulations of w."""
    from paper_2608_15249_amd.sim import Simulation
    state = W.sample(w)
    a = Simulation(w, precision, state=state, tile=tile)
    b = Simulation(w, precision, state=state, tile=tile)
    for s in (a, b):
        s.initialise()
    return a, b


def _compare(torch, a, b, precision, nsteps):
    da = torch.zeros(4 * nsteps, dtype=torch.float64, device="cuda")
    db = torch.zeros(4 * nsteps, dtype=torch.float64, device="cuda")
    a.ctx.step(a.p, a.E, a.E32, nsteps, da)
    b.ctx.step_static(b.p, b.E, b.E32, nsteps, db)
    a.ctx.sync()
    b.ctx.sync()
    sa, sb = a.p.download(), b.p.download()
    assert np.array_equal(sa["bucket_start"], sb["bucket_start"])
    if precision == "mixed":
        for k in ("cell", "ox", "oy", "vx", "vy"):
            assert np.array_equal(sa[k], sb[k]), k
        assert np.array_equal(a.E.cpu().numpy(), b.E.cpu().numpy())
        assert np.array_equal(a.E32.cpu().numpy(), b.E32.cpu().numpy())
        assert np.array_equal(da.cpu().numpy(), db.cpu().numpy())
    else:
        for k in ("x", "y", "vx", "vy"):
            assert np.max(np.abs(sa[k] - sb[k])) < 1e-12, k
        ea, eb = a.E.cpu().numpy(), b.E.cpu().numpy()
        assert np.max(np.abs(ea - eb)) <= 1e-12 * np.max(np.abs(ea))
        assert np.allclose(da.cpu().numpy(), db.cpu().numpy(), rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_step_static_matches_step(torch, precision):
    big = W.thermal_2d(seed=71, nx=64, ppc=16)       # 65,536 particles, 64 x 64
    small = W.thermal_2d(seed=72, nx=32, ppc=8)      # 8,192 particles, 32 x 32
    a, b = _pair(torch, big, precision, (16, 16))
    _compare(torch, a, b, precision, 3)
    a2, b2 = _pair(torch, small, precision, (8, 8))
    _compare(torch, a2, b2, precision, 2)
    # and the larger plasma once more after the smaller one used the array
    _compare(torch, a, b, precision, 2)


def test_step_static_rejects_large_workspace(torch):
    from paper_2608_15249_amd.apic import ApicError, Context, Particles
    n = 4_000_000
    c = Context(dim=2, vdim=2, nx=256, ny=256, lx=256.0, ly=256.0, dt=0.1, n=n, precision="mixed")
    assert c.ws.numel() > (64 << 20)
    p = Particles(c)
    E = torch.zeros(2 * c.G, dtype=torch.float64, device="cuda")
    with pytest.raises(ApicError) as ei:
        c.step_static(p, E, None, 1)
    assert ei.value.status == -1 and "workspace" in str(ei.value)
