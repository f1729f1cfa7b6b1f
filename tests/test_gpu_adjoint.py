"""GPU adjoint (apic_adjoint_forward / apic_step_adjoint) against the oracle's
FP64 reference gradient, against central differences of the GPU forward run,
across checkpoint strides, and through the torch.autograd.Function."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import adjoint as OA
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return t


def _maxabs(a, b):
    """Largest element-wise difference, relative to the largest element of
    the reference: max_p |a_p - b_p| / max_p |b_p|."""
    return float(np.max(np.abs(np.ravel(a) - np.ravel(b))) / np.max(np.abs(np.ravel(b))))


def _dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _gpu_grad(torch, w, state, nsteps, stride, precision, tile=(0, 0)):
    from paper_2608_15249_amd.adjoint import FieldEnergyRun
    x, y, vx, vy, vz = state
    run = FieldEnergyRun(dim=w.dim, vdim=w.vdim, nx=w.nx, ny=w.ny, lx=w.Lx, ly=w.Ly, dt=w.dt, n=len(x),
                         nsteps=nsteps, stride=stride, bz=w.bz, precision=precision, tile=tile)
    Wv = run.forward(*[_dev(torch, a) for a in (x, y, vx, vy, vz)])
    g = run.backward()
    run.sync()
    return float(Wv.item()), [None if a is None else a.cpu().numpy() for a in g]


def _oracle_grad(w, state, nsteps):
    x, y, vx, vy, vz = state
    s = O.Setup(w.dim, w.vdim, w.nx, w.Lx, len(x), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz)
    Wv, lx, lv = OA.adjoint(s, O.State.from_arrays(x, vx, y, vy, vz), nsteps)
    lx = lx + [None] * (2 - len(lx))
    lv = lv + [None] * (3 - len(lv))
    return Wv, [lx[0], lx[1], lv[0], lv[1], lv[2]]


SMALL = {
    # name: (workload, particles (None = all), steps, stride)
    "1d1v_two_stream": (W.two_stream_1d(), None, 30, 7),
    "2d2v_two_stream": (W.two_stream_2d(nx=32, ppc=16), None, 24, 5),
    "2d3v_magnetized": (dataclasses.replace(W.magnetized_2d3v(nx=16, ppc=32), mode=(1, 0)), None, 20, 6),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_fp64_adjoint_matches_oracle_gradient(torch, name):
    w, n, nsteps, stride = SMALL[name]
    state = W.sample(w, n)
    Wg, gg = _gpu_grad(torch, w, state, nsteps, stride, "fp64")
    Wo, go = _oracle_grad(w, state, nsteps)
    assert abs(Wg / Wo - 1.0) < 1e-11, (Wg, Wo)
    for k, (a, b) in enumerate(zip(gg, go)):
        if b is None:
            assert a is None
        elif not np.any(b):
            assert np.max(np.abs(a)) == 0.0, k      # v_z of a 2D3V plasma never reaches the field
        else:
            assert _maxabs(a, b) < 1e-9, (k, _maxabs(a, b))


@pytest.mark.parametrize("name", sorted(SMALL))
def test_mixed_adjoint_matches_oracle_gradient(torch, name):
    """binary32 forward and adjoint against the FP64 reference: the trajectories
    differ by binary32 rounding of positions and velocities, amplified by the
    instability (measured: about 1e-6 on W and 2e-6 on the gradient norms at
    these sizes)."""
    w, n, nsteps, stride = SMALL[name]
    state = W.sample(w, n)
    Wg, gg = _gpu_grad(torch, w, state, nsteps, stride, "mixed")
    Wo, go = _oracle_grad(w, state, nsteps)
    assert abs(Wg / Wo - 1.0) < 1e-5, (Wg, Wo)
    for k, (a, b) in enumerate(zip(gg, go)):
        if b is None:
            assert a is None
        elif not np.any(b):
            assert np.max(np.abs(a)) == 0.0, k
        else:
            assert _maxabs(a, b) < 2e-5, (k, _maxabs(a, b))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gradient_does_not_depend_on_checkpoint_stride(torch, precision):
    w = W.two_stream_2d(nx=32, ppc=16)
    state = W.sample(w)
    ref = None
    for stride in (1, 4, 13, 40):          # 40 > nsteps: one segment
        _, g = _gpu_grad(torch, w, state, 26, stride, precision)
        if ref is None:
            ref = g
            continue
        for a, b in zip(g, ref):
            if b is not None:
                assert _maxabs(a, b) < (1e-10 if precision == "fp64" else 1e-5), stride


def test_zero_and_one_step_runs_match_oracle(torch):
    w = W.two_stream_2d(nx=16, ppc=16)
    state = W.sample(w)
    for nsteps in (0, 1):
        Wg, gg = _gpu_grad(torch, w, state, nsteps, 3, "fp64")
        Wo, go = _oracle_grad(w, state, nsteps)
        assert abs(Wg / Wo - 1.0) < 1e-12
        for a, b in zip(gg, go):
            if b is not None and np.any(b):
                assert _maxabs(a, b) < 1e-10, nsteps
            elif b is not None:
                assert np.max(np.abs(a)) == 0.0


def _delta0_direction(w):
    xu, yu, *_ = W.sample(dataclasses.replace(w, delta0=0.0))
    s = O.Setup(w.dim, w.vdim, w.nx, w.Lx, len(xu), w.dt, ny=w.ny, Ly=w.Ly, bz=w.bz)
    return OA.delta0_direction(s, xu, yu, w.mode)


def test_delta0_gradient_matches_central_differences_of_gpu_runs(torch):
    """1D two-stream, FP64 path: the central difference of the GPU forward run
    converges to the GPU adjoint's dW/d delta0 as h shrinks (a finite step
    averages the slope over the CIC kinks it crosses)."""
    from paper_2608_15249_amd.adjoint import FieldEnergyRun
    w = W.two_stream_1d()
    nsteps = 40
    state = W.sample(w)
    _, g = _gpu_grad(torch, w, state, nsteps, 10, "fp64")
    dirn = _delta0_direction(w)
    gd = float(np.dot(g[0], dirn[0]))
    run = FieldEnergyRun(dim=1, vdim=1, nx=w.nx, ny=1, lx=w.Lx, ly=1.0, dt=w.dt, n=w.n_particles, nsteps=nsteps,
                         stride=10, precision="fp64")

    def Wof(d0):
        x, y, vx, vy, vz = W.sample(dataclasses.replace(w, delta0=d0))
        return float(run.forward(_dev(torch, x), None, _dev(torch, vx)).item())

    errs = []
    for h in (1e-4, 1e-6, 1e-7):
        fd = (Wof(w.delta0 + h) - Wof(w.delta0 - h)) / (2 * h)
        errs.append(abs(fd / gd - 1.0))
    assert errs[0] < 2e-2 and errs[-1] < 1e-6 and errs[-1] < errs[1] < errs[0], errs
    # single-particle velocities: W is smooth in v
    x, y, vx, vy, vz = state
    for p in (3, 9000):
        def Wv(dv):
            v2 = vx.copy()
            v2[p] += dv
            return float(run.forward(_dev(torch, x), None, _dev(torch, v2)).item())
        fd = (Wv(1e-5) - Wv(-1e-5)) / 2e-5
        assert abs(fd / g[2][p] - 1.0) < 1e-5, (p, fd, g[2][p])


def test_autograd_function_chains_to_delta0(torch):
    """torch.autograd through the library: x0 = wrap(x_u + delta0 d) built in
    torch, W from the Function, backward gives dW/d delta0 = sum lam_x . d and
    the velocity gradients of the C-ABI call."""
    from paper_2608_15249_amd.adjoint import FieldEnergyRun, field_energy
    w = W.two_stream_2d(nx=32, ppc=16)
    nsteps = 20
    xu, yu, vx, vy, _ = W.sample(dataclasses.replace(w, delta0=0.0))
    dx, dy = _delta0_direction(w)
    run = FieldEnergyRun.for_workload(w, stride=6, precision="fp64", nsteps=nsteps)
    d0 = torch.tensor(w.delta0, dtype=torch.float64, device="cuda", requires_grad=True)
    tvx = _dev(torch, vx).requires_grad_(True)
    x0 = torch.remainder(_dev(torch, xu) + d0 * _dev(torch, dx), w.Lx)
    y0 = torch.remainder(_dev(torch, yu) + d0 * _dev(torch, dy), w.Ly)
    Wt = field_energy(run, x0, y0, tvx, _dev(torch, vy))
    Wt.sum().backward()
    state = (x0.detach().cpu().numpy(), y0.detach().cpu().numpy(), vx, vy, None)
    Wg, g = _gpu_grad(torch, w, state, nsteps, 6, "fp64")
    assert abs(Wt.item() / Wg - 1.0) < 1e-12
    ref = float(np.dot(g[0], dx) + np.dot(g[1], dy))
    assert abs(d0.grad.item() / ref - 1.0) < 1e-9
    assert _maxabs(tvx.grad.cpu().numpy(), g[2]) < 1e-10


def test_differentiable_two_stream_full_size(torch):
    """The differentiable 2D2V two-stream at full size: 256 x 256, 1,048,576
    electrons, 200 steps, checkpoints every 20. Both paths against the
    oracle's FP64 gradient (dW/d delta0 from the library's own reduction, and
    every particle's position and velocity gradient element by element), and
    each path's dW/d delta0 against a central difference of its own forward
    run: at h = 1e-5 the FP64 difference meets the 1e-4 target (at h = 1e-4
    the CIC kinks that particles cross move it by about 8e-4); the binary32
    forward run's difference is printed beside its bound."""
    from paper_2608_15249_amd.adjoint import FieldEnergyRun
    w = W.two_stream_2d()
    state = W.sample(w)
    x, y, vx, vy, _ = state
    dirn = _delta0_direction(w)
    Wo, go = _oracle_grad(w, state, w.steps)
    gdo = float(np.dot(go[0], dirn[0]) + np.dot(go[1], dirn[1]))
    # (W, dW/d delta0, per-element gradients, FD at h = 1e-5)
    # mixed per-element: the binary32 trajectories of 200 steps of the
    # instability part from the FP64 ones by rounding amplified about e^{gamma t}
    # times (measured 1.4e-2 .. 6.1e-2 of the largest element; dW/d delta0,
    # a sum over every particle, stays within 2e-5)
    bounds = {"fp64": (1e-11, 1e-10, 1e-9, 1e-4), "mixed": (1e-6, 2e-4, 1e-1, 2e-3)}
    for prec, (bw, bd, bg, bfd) in bounds.items():
        run = FieldEnergyRun.for_workload(w, stride=20, precision=prec)
        args = [_dev(torch, a) for a in (x, y, vx, vy)]
        Wg = float(run.forward(*args).item())
        out = run.backward(1.0, _dev(torch, dirn[0]), _dev(torch, dirn[1]))
        g = [None if a is None else a.cpu().numpy() for a in out[:5]]
        gd = float(out[6].item())
        run.sync()
        gd_host = float(np.dot(g[0], dirn[0]) + np.dot(g[1], dirn[1]))
        assert abs(gd / gd_host - 1.0) < 1e-12, (gd, gd_host)
        errs = [_maxabs(g[k], go[k]) for k in range(4)]
        print("%s: W %.3e, dW/d delta0 %.3e, per-element gradients %s" % (
            prec, abs(Wg / Wo - 1.0), abs(gd / gdo - 1.0), " ".join("%.2e" % e for e in errs)))
        assert abs(Wg / Wo - 1.0) < bw, (prec, Wg, Wo)
        assert abs(gd / gdo - 1.0) < bd, (prec, gd, gdo)
        for k in range(4):
            assert errs[k] < bg, (prec, k, errs[k])

        def Wof(d0):
            xx, yy, *_ = W.sample(dataclasses.replace(w, delta0=d0))
            return float(run.forward(_dev(torch, xx), _dev(torch, yy), args[2], args[3]).item())
        fds = {}
        for h in (1e-4, 1e-5):
            fd = (Wof(w.delta0 + h) - Wof(w.delta0 - h)) / (2 * h)
            fds[h] = abs(fd / gd - 1.0)
        print("%s: central difference against the adjoint: h=1e-4 %.2e, h=1e-5 %.2e" % (prec, fds[1e-4], fds[1e-5]))
        assert fds[1e-5] < bfd, (prec, fds)
