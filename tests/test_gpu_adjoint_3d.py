"""GPU adjoint of the 3D cycle (trilinear weights, the 7-point solve, E_z
kicking v_z, the z motion) through the C ABI, against the oracle's FP64
reference gradient element by element: Boris and Higuera-Cary, both paths,
across checkpoint strides, the zero-step run, dW/d delta0 from the library's
own reduction, and a central difference of the GPU forward run."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import adjoint as OA
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu

BZ = 0.8
C_LIGHT = 3.0


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return t


def _maxabs(a, b):
    return float(np.max(np.abs(np.ravel(a) - np.ravel(b))) / np.max(np.abs(np.ravel(b))))


def _dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(seed=41, nx=8, ny=6, nz=4, ppc=8):
    """A thermal 3D plasma of 8 x 6 x 4 cells (a ragged, non-cubic grid) with
    mode (1, 0) seeded at delta0 = 0.05."""
    w = dataclasses.replace(W.thermal_3d(seed=seed, nx=nx, ny=ny, nz=nz, ppc=ppc), mode=(1, 0), delta0=0.05)
    return w, W.sample3(w)


def _setup(w, n, pusher):
    c = C_LIGHT if pusher == "hc" else float("inf")
    return O.Setup(3, 3, w.nx, w.Lx, n, w.dt, ny=w.ny, Ly=w.Ly, nz=w.nz, Lz=w.Lz, bz=BZ, pusher=pusher, c=c)


def _run(w, n, nsteps, stride, precision, pusher):
    from paper_2608_15249_amd.adjoint import FieldEnergyRun
    return FieldEnergyRun(dim=3, vdim=3, nx=w.nx, ny=w.ny, nz=w.nz, lx=w.Lx, ly=w.Ly, lz=w.Lz, dt=w.dt, n=n,
                          nsteps=nsteps, stride=stride, bz=BZ, precision=precision, pusher=pusher,
                          c_light=C_LIGHT if pusher == "hc" else 0.0)


def _gpu_grad(torch, w, state, nsteps, stride, precision, pusher, dirn=None):
    x, y, z, vx, vy, vz = state
    run = _run(w, len(x), nsteps, stride, precision, pusher)
    Wv = run.forward(*[_dev(torch, a) for a in (x, y, vx, vy, vz)], z=_dev(torch, z))
    if dirn is None:
        out = run.backward()
    else:
        out = run.backward(1.0, _dev(torch, dirn[0]), _dev(torch, dirn[1]))
    run.sync()
    g = [a.cpu().numpy() for a in out[:6]]
    # order (x, y, z, vx, vy, vz)
    g = [g[0], g[1], g[5], g[2], g[3], g[4]]
    gd = float(out[6].item()) if dirn is not None else None
    return float(Wv.item()), g, gd


def _oracle_grad(w, state, nsteps, pusher):
    x, y, z, vx, vy, vz = state
    s = _setup(w, len(x), pusher)
    Wv, lx, lv = OA.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz, z), nsteps)
    return Wv, list(lx) + list(lv)


@pytest.mark.parametrize("pusher", ["boris", "hc"])
def test_fp64_adjoint_3d_matches_oracle_gradient(torch, pusher):
    w, state = _case()
    Wg, gg, _ = _gpu_grad(torch, w, state, 8, 3, "fp64", pusher)
    Wo, go = _oracle_grad(w, state, 8, pusher)
    assert abs(Wg / Wo - 1.0) < 1e-11, (Wg, Wo)
    for k, (a, b) in enumerate(zip(gg, go)):
        assert np.any(b), k                     # every component reaches the field in 3D
        assert _maxabs(a, b) < 1e-9, (k, _maxabs(a, b))


@pytest.mark.parametrize("pusher", ["boris", "hc"])
def test_mixed_adjoint_3d_matches_oracle_gradient(torch, pusher):
    """binary32 forward and adjoint against the FP64 reference gradient: a
    thermal plasma (no instability) over 8 steps keeps the binary32
    trajectories within rounding of the FP64 ones."""
    w, state = _case()
    Wg, gg, _ = _gpu_grad(torch, w, state, 8, 3, "mixed", pusher)
    Wo, go = _oracle_grad(w, state, 8, pusher)
    errs = [_maxabs(a, b) for a, b in zip(gg, go)]
    print("%s mixed 3D: W %.2e, per-element %s" % (pusher, abs(Wg / Wo - 1.0), " ".join("%.2e" % e for e in errs)))
    assert abs(Wg / Wo - 1.0) < 1e-5, (Wg, Wo)
    for k, e in enumerate(errs):
        assert e < 1e-4, (k, e)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_3d_does_not_depend_on_checkpoint_stride(torch, precision):
    w, state = _case(seed=43)
    ref = None
    for stride in (1, 4, 11):               # 11 > nsteps: one segment
        _, g, _ = _gpu_grad(torch, w, state, 9, stride, precision, "boris")
        if ref is None:
            ref = g
            continue
        for a, b in zip(g, ref):
            assert _maxabs(a, b) < (1e-10 if precision == "fp64" else 1e-5), stride


@pytest.mark.parametrize("pusher", ["boris", "hc"])
def test_zero_and_one_step_adjoint_3d(torch, pusher):
    """0 steps: W of the initial field, whose gradient in v^0 is zero; 1
    step: the backward half push enters."""
    w, state = _case(seed=44)
    for nsteps in (0, 1):
        Wg, gg, _ = _gpu_grad(torch, w, state, nsteps, 2, "fp64", pusher)
        Wo, go = _oracle_grad(w, state, nsteps, pusher)
        assert abs(Wg / Wo - 1.0) < 1e-12
        for a, b in zip(gg, go):
            if np.any(b):
                assert _maxabs(a, b) < 1e-10, nsteps
            else:
                assert np.max(np.abs(a)) == 0.0, nsteps


def test_delta0_gradient_3d(torch):
    """dW/d delta0 of the 3D run (mode (1, 0): x and y move): the library's
    fixed-order device sum against the oracle's sum_p lam_x . d, and a
    central difference of the GPU forward run in delta0 against it."""
    w, state = _case(seed=45)
    nsteps = 8
    x, y, z, vx, vy, vz = state
    s = _setup(w, len(x), "boris")
    xu, yu, *_ = W.sample3(dataclasses.replace(w, delta0=0.0))
    dirn = OA.delta0_direction(s, xu, yu, w.mode)
    Wg, g, gd = _gpu_grad(torch, w, state, nsteps, 3, "fp64", "boris", dirn=dirn)
    _, lx, _ = OA.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz, z), nsteps)
    ref = OA.grad_delta0(lx, dirn)
    assert abs(gd / ref - 1.0) < 1e-9, (gd, ref)
    run = _run(w, len(x), nsteps, 3, "fp64", "boris")

    def Wof(d0):
        x2, y2, z2, a, b, c = W.sample3(dataclasses.replace(w, delta0=d0))
        return float(run.forward(*[_dev(torch, q) for q in (x2, y2, a, b, c)], z=_dev(torch, z2)).item())
    h = 1e-6
    fd = (Wof(w.delta0 + h) - Wof(w.delta0 - h)) / (2 * h)
    assert abs(fd / gd - 1.0) < 1e-4, (fd, gd)
