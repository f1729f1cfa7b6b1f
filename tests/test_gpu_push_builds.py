"""The two builds of the mixed electrostatic push (the plain one and the one
that holds the tile and step constants in vector registers; the launch picks
one by resident workgroups, APIC_PUSH_VR=0 / 1 at context creation forces
either) give the same bits: the field, the diagnostics, every particle array
and the bucket table after several steps, in 1D1V, 2D2V, magnetized 2D3V,
between absorbing walls and in 3D3V."""
import dataclasses
import os

import numpy as np
import pytest

from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


def _run(torch, w, tile, walls, vr):
    from paper_2608_15249_amd.sim import Simulation
    old = os.environ.get("APIC_PUSH_VR")
    os.environ["APIC_PUSH_VR"] = vr
    try:
        state = W.sample3(w) if w.dim == 3 else W.sample(w)
        s = Simulation(w, "mixed", state=state, tile=tile, walls=walls)
    finally:
        if old is None:
            os.environ.pop("APIC_PUSH_VR", None)
        else:
            os.environ["APIC_PUSH_VR"] = old
    s.initialise()
    d = s.run(STEPS, diag=True)
    s.ctx.sync()
    arrays = {k: v for k, v in s.p.download().items() if v is not None}
    return s.E.cpu().numpy(), d.cpu().numpy(), arrays


@pytest.mark.parametrize("case", ["1d", "2d2v", "2d3v", "walls", "3d"])
def test_push_builds_give_the_same_bits(torch, case):
    walls = False
    if case == "1d":
        w, tile = W.two_stream_1d(seed=80), (8, 1)
    elif case == "2d2v":
        w, tile = W.thermal_2d(seed=81, nx=48, ppc=16), (8, 8)
    elif case == "2d3v":
        w, tile = W.magnetized_2d3v(nx=64, ppc=16), (16, 8)
    elif case == "walls":
        w = dataclasses.replace(W.thermal_2d(seed=82, nx=32, ppc=16), ny=16, Ly=16.0, n_particles=32 * 16 * 16)
        tile, walls = (8, 4), True
    else:
        w, tile = W.thermal_3d(seed=83, nx=16, ppc=8), (8, 4, 4)
    Ea, da, pa = _run(torch, w, tile, walls, "0")
    Eb, db, pb = _run(torch, w, tile, walls, "1")
    assert np.array_equal(Ea, Eb)
    assert np.array_equal(da, db)
    live = int(pa["bucket_start"][-1])
    assert live == int(pb["bucket_start"][-1])
    for k in pa:
        if k == "bucket_start":
            assert np.array_equal(pa[k], pb[k]), k
        else:
            assert np.array_equal(pa[k][:live], pb[k][:live]), k
