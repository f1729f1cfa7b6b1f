"""apic_step_pair (two caller-owned particle buffers, no copy after an odd
step count) against apic_step through the C ABI: the same calls of 1, 2, 3
and 1 steps give the same bits (field, diagnostics, every particle array and
the bucket table) on the mixed path (2D fused solve, 3D, absorbing walls),
and agree to rounding on the FP64 path, whose deposit sums in FP64 atomics."""
import dataclasses

import numpy as np
import pytest

from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu

CHUNKS = (1, 2, 3, 1)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


def _arrays(p):
    d = p.download()
    return {k: v for k, v in d.items() if v is not None}


def _pair_vs_step(torch, w, precision, tile, walls=False):
    from paper_2608_15249_amd.apic import Particles
    from paper_2608_15249_amd.sim import Simulation
    state = W.sample3(w) if w.dim == 3 else W.sample(w)
    a = Simulation(w, precision, state=state, tile=tile, walls=walls)
    b = Simulation(w, precision, state=state, tile=tile, walls=walls)
    for s in (a, b):
        s.initialise()
    total = sum(CHUNKS)
    da = torch.zeros(4 * total, dtype=torch.float64, device="cuda")
    db = torch.zeros_like(da)
    other = Particles(b.ctx)
    cur, k = b.p, 0
    held = []
    for m in CHUNKS:
        a.ctx.step(a.p, a.E, a.E32, m, da[4 * k:4 * (k + m)])
        nxt = b.ctx.step_pair(cur, other if cur is b.p else b.p, b.E, b.E32, m, db[4 * k:4 * (k + m)])
        held.append(nxt is not cur)
        cur = nxt
        k += m
    a.ctx.sync()
    b.ctx.sync()
    # an odd chunk moves the state to the other buffer, an even one keeps it
    assert held == [m % 2 == 1 for m in CHUNKS]
    return (a.E.cpu().numpy(), da.cpu().numpy(), _arrays(a.p)), (b.E.cpu().numpy(), db.cpu().numpy(), _arrays(cur))


@pytest.mark.parametrize("case", ["2d_fused", "3d", "2d_walls"])
def test_step_pair_mixed_bit_identical(torch, case):
    if case == "2d_fused":
        w, tile, walls = W.magnetized_2d3v(nx=64, ppc=16), (16, 8), False
    elif case == "3d":
        w, tile, walls = W.thermal_3d(seed=71, nx=16, ppc=8), (8, 4, 4), False
    else:
        w = dataclasses.replace(W.thermal_2d(seed=72, nx=32, ppc=16), ny=16, Ly=16.0, n_particles=32 * 16 * 16)
        tile, walls = (8, 4), True
    (Ea, da, pa), (Eb, db, pb) = _pair_vs_step(torch, w, "mixed", tile, walls)
    assert np.array_equal(Ea, Eb)
    assert np.array_equal(da, db)
    live = int(pa["bucket_start"][-1])
    assert live == int(pb["bucket_start"][-1])
    for k in pa:
        # between walls the entries past the live count are unused
        if k == "bucket_start":
            assert np.array_equal(pa[k], pb[k]), k
        else:
            assert np.array_equal(pa[k][:live], pb[k][:live]), k


def test_step_pair_fp64(torch):
    w = W.two_stream_2d(nx=32, ppc=16)
    (Ea, da, pa), (Eb, db, pb) = _pair_vs_step(torch, w, "fp64", (8, 8))
    assert np.max(np.abs(Ea - Eb)) <= 1e-11 * np.max(np.abs(Ea))
    assert np.max(np.abs(da - db) / np.maximum(np.abs(da), 1e-300)) <= 1e-10
    assert np.array_equal(pa["bucket_start"], pb["bucket_start"])
    for k in ("x", "y", "vx", "vy"):
        assert np.max(np.abs(pa[k] - pb[k])) <= 1e-10, k


def test_step_pair_rejects_one_buffer_twice(torch):
    from paper_2608_15249_amd.apic import ApicError
    from paper_2608_15249_amd.sim import Simulation
    s = Simulation(W.two_stream_2d(nx=16, ppc=16), "mixed", tile=(8, 8))
    s.initialise()
    with pytest.raises(ApicError):
        s.ctx.step_pair(s.p, s.p, s.E, s.E32, 1)
    # a second buffer object over the same arrays: refused by the library
    from paper_2608_15249_amd.apic import Particles
    q = Particles(s.ctx)
    for k in ("cell", "ox", "oy", "vx", "vy", "bucket_start"):
        setattr(q, k, getattr(s.p, k))
    with pytest.raises(ApicError):
        s.ctx.step_pair(s.p, q, s.E, s.E32, 1)
