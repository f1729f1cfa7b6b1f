"""The paper's own example on the GPU path ("Illustrative examples": the 2D3V
electrostatic two-stream case, "Results and validation"): 64 x 64 cells,
L = 64 Debye lengths, 524,288 electrons in beams N(+-3, 1) in v_x and N(0, 1)
in v_y and v_z, dt = 0.05, mode (2, 1) seeded with delta0 = 0.005, run to
omega_pe t = 40 (800 steps), in both precisions. The paper fits
gamma_PIC = 0.2603 over 10 <= t <= 19 against the kinetic root 0.2616
(reproduced: 0.26160) and reports a largest total-energy error of 0.0183 %
of W0. Checked here: the GPU's fitted rate within 2 % of 0.26160, R^2 of the
fit above 0.9, and the largest energy error over the whole run below 1e-3;
the measured figures are printed."""
import numpy as np
import pytest

import oracle as O
from paper_2608_15249_amd import workloads as W

pytestmark = pytest.mark.gpu

GAMMA_TH = 0.26160


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2608_15249_amd import apic
    apic.load_library()
    return t


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paper_two_stream_on_the_gpu(torch, precision):
    from paper_2608_15249_amd.sim import Simulation
    w = W.paper_two_stream()
    state = W.sample(w)
    x, y, vx, vy, vz = state
    sim = Simulation(w, precision, state=state)
    sim.initialise()
    s = O.Setup(2, 3, w.nx, w.Lx, w.n_particles, w.dt, ny=w.ny, Ly=w.Ly)
    # t = 0: W_E of the initial field, kinetic energy of v^0 (as uploaded)
    if precision == "mixed":
        v2 = sum(np.sum(v.astype(np.float32).astype(np.float64) ** 2) for v in (vx, vy, vz))
    else:
        v2 = sum(np.sum(v ** 2) for v in (vx, vy, vz))
    W0 = float(sim.we0.item()) + 0.5 * sim.ctx.q_macro / -1.0 * v2
    nsteps = w.steps
    diag = torch.zeros(4 * nsteps, dtype=torch.float64, device="cuda")
    amp = [O.mode_amplitude(s, sim.field(), 2, 1)]
    for k in range(nsteps):
        sim.ctx.step(sim.p, sim.E, sim.E32, 1, diag[4 * k:4 * k + 4])
        amp.append(O.mode_amplitude(s, sim.field(), 2, 1))
    sim.ctx.sync()
    d = diag.cpu().numpy().reshape(nsteps, 4)
    amp = np.array(amp)
    t = np.arange(nsteps + 1) * w.dt
    g, r2 = O.growth_rate(t, amp, 10.0, 19.0)
    # total energy at levels 1..nsteps-1: W_E^n (step n-1) + KE^n (step n)
    Wt = d[:-1, 1] + d[1:, 2]
    err = float(np.max(np.abs(np.concatenate([[W0], Wt]) - W0)) / W0)
    peak = float(t[np.argmax(amp)])
    print("%s: gamma %.7f (R^2 %.5f, %.3f%% from %.5f), largest energy error %.6e of W0, mode peak at t = %.2f"
          % (precision, g, r2, 100 * abs(g / GAMMA_TH - 1), GAMMA_TH, err, peak))
    assert abs(g / GAMMA_TH - 1) < 0.02, g
    assert r2 > 0.9, r2
    assert err < 1e-3, err
    # charge exact on the mixed path at every step; within rounding on FP64
    if precision == "mixed":
        assert np.all(d[:, 0] == np.float64(sim.ctx.q_macro) * w.n_particles)
    else:
        assert np.max(np.abs(d[:, 0] / (sim.ctx.q_macro * w.n_particles) - 1)) < 1e-12
