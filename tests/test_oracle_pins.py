"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: hand values,
closed forms, brute-force linear algebra, conservation laws and the exact
properties of the Boris map."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2608_15249_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _setup2d(nx, ny, Lx, Ly, n, dt=0.1, bz=0.0, vdim=2):
    return O.Setup(2, vdim, nx, Lx, n, dt, ny=ny, Ly=Ly, bz=bz)


# --------------------------------------------------------------------- CIC

def test_deposit_and_gather_hand_values():
    g = json.load(open(os.path.join(GOLD, "deposit_tiny.json")))
    gr = g["grid"]
    xs = np.array([p["x"] for p in g["particles"]])
    ys = np.array([p["y"] for p in g["particles"]])
    s = _setup2d(gr["nx"], gr["ny"], gr["Lx"], gr["Ly"], len(xs))
    w = O.deposit_counts(s, O.State.from_arrays(xs, np.zeros(3), ys, np.zeros(3)))
    expect = np.zeros((gr["ny"], gr["nx"]))
    for k, v in g["weight_sum_by_node"].items():
        if k == "comment":
            continue
        ix, iy = map(int, k.split(","))
        expect[iy, ix] = v
    assert np.array_equal(w, expect)
    ix, iy = np.meshgrid(np.arange(4), np.arange(4))
    Ex = (ix + 10 * iy).astype(np.float64)
    Epx, Epy = O.gather(s, O.State.from_arrays(xs, np.zeros(3), ys, np.zeros(3)), (Ex, np.zeros_like(Ex)))
    assert np.array_equal(Epx, np.array(g["gather"]["values"]))
    assert np.all(Epy == 0.0)


def test_quantised_hand_values():
    g = json.load(open(os.path.join(GOLD, "deposit_tiny.json")))
    S = g["quantised"]["S"]
    s = _setup2d(4, 4, 2.0, 2.0, 1)
    for c in g["quantised"]["cases"]:
        I = O.deposit_quantised(s, np.array([c["ix"]]), np.array([c["ox"]], np.float32), S,
                                np.array([c["iy"]]), np.array([c["oy"]], np.float32))
        expect = np.zeros((4, 4), np.int64)
        for k, v in c["nodes"].items():
            ix, iy = map(int, k.split(","))
            expect[iy, ix] = v
        assert np.array_equal(I, expect), c


def test_weights_sum_to_one_and_edge():
    rng = np.random.default_rng(3)
    n, L = 20000, 7.3
    x = rng.uniform(0, L, n)
    x[:4] = [0.0, np.nextafter(L, 0), L / 16 * 5, 1e-300]
    s = O.Setup(1, 1, 16, L, n, 0.1)
    w = O.deposit_counts(s, O.State.from_arrays(x, np.zeros(n)))
    assert abs(w.sum() - n) <= 1e-12 * n
    for xi in x[:64]:
        i = ctypes_weights(xi, 16, L / 16)
        assert abs(i[2] + i[3] - 1.0) <= 1e-15
        assert 0 <= i[0] < 16 and i[1] == (i[0] + 1) % 16


def ctypes_weights(x, n, d):
    import ctypes
    L = O._load()
    i = ctypes.c_int64()
    ip = ctypes.c_int64()
    w0 = ctypes.c_double()
    w1 = ctypes.c_double()
    L.or_cic_weights_1d.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double] + [ctypes.c_void_p] * 4
    L.or_cic_weights_1d(x, n, d, ctypes.byref(i), ctypes.byref(ip), ctypes.byref(w0), ctypes.byref(w1))
    return i.value, ip.value, w0.value, w1.value


@pytest.mark.parametrize("dim", [1, 2])
def test_charge_conservation(dim):
    rng = np.random.default_rng(5)
    n = 50000
    if dim == 1:
        s = O.Setup(1, 1, 37, 5.0, n, 0.1)
        st = O.State.from_arrays(rng.uniform(0, 5.0, n), np.zeros(n))
    else:
        s = _setup2d(24, 17, 6.0, 3.0, n)
        st = O.State.from_arrays(rng.uniform(0, 6, n), np.zeros(n), rng.uniform(0, 3, n), np.zeros(n))
    rho = O.deposit(s, st)
    total = float(np.sum(rho - s.rho_ion)) * s.dV
    assert abs(total - n * s.Q) <= 1e-12 * abs(n * s.Q)
    # mean of rho vanishes (neutral plasma)
    assert abs(rho.mean()) <= 1e-12


@pytest.mark.parametrize("S", [20, 24])
def test_quantised_exact_charge_and_agreement(S):
    rng = np.random.default_rng(9)
    n, nx, ny = 40000, 16, 12
    x = rng.uniform(0, nx, n)
    y = rng.uniform(0, ny, n)
    ix, ox = W.to_cell_offset(x, 1.0, nx)
    iy, oy = W.to_cell_offset(y, 1.0, ny)
    s = _setup2d(nx, ny, float(nx), float(ny), n)
    I = O.deposit_quantised(s, ix, ox, S, iy, oy)
    # every particle deposits exactly 2^(2S); sum in Python integers (no wrap)
    assert sum(int(v) for v in I.ravel()) == n << (2 * S)
    w = O.deposit_counts(s, O.State.from_arrays(x, np.zeros(n), y, np.zeros(n)))
    # fixed-point weights differ from FP64 ones by at most 2^-S per axis per particle
    err = np.abs(I * 2.0 ** (-2 * S) - w).max()
    assert err <= (n * 2.0 ** (-S + 1)) / (nx * ny) * 4 + 1e-9
    rho_q = O.rho_from_quantised(s, I, S)
    assert abs(rho_q.mean()) < 1e-12


# ----------------------------------------------------------------- Poisson

def test_poisson_cos_mode_closed_form():
    nx, ny, Lx, Ly = 32, 24, 10.0, 7.0
    s = _setup2d(nx, ny, Lx, Ly, 1)
    X = np.arange(nx) * s.dx
    Y = np.arange(ny) * s.dy
    XX, YY = np.meshgrid(X, Y)
    mx, my, A = 3, 2, 0.7
    kx, ky = 2 * np.pi * mx / Lx, 2 * np.pi * my / Ly
    rho = A * np.cos(kx * XX + ky * YY)
    K2 = (2 / s.dx * np.sin(kx * s.dx / 2)) ** 2 + (2 / s.dy * np.sin(ky * s.dy / 2)) ** 2
    Ex, Ey = O.solve_field(s, rho)
    ph = O.solve_potential(s, rho)
    assert np.allclose(ph, A / K2 * np.cos(kx * XX + ky * YY), atol=1e-13, rtol=0)
    assert np.allclose(Ex, A / K2 * np.sin(kx * s.dx) / s.dx * np.sin(kx * XX + ky * YY), atol=1e-13, rtol=0)
    assert np.allclose(Ey, A / K2 * np.sin(ky * s.dy) / s.dy * np.sin(kx * XX + ky * YY), atol=1e-13, rtol=0)


def test_poisson_dense_bruteforce():
    """Solve the periodic FD system directly (dense) and differentiate by hand."""
    nx, ny = 7, 6
    s = _setup2d(nx, ny, 3.5, 2.0, 1)
    rng = np.random.default_rng(1)
    rho = rng.normal(size=(ny, nx))
    rho -= rho.mean()
    G = nx * ny
    A = np.zeros((G + 1, G))
    for j in range(ny):
        for i in range(nx):
            r = j * nx + i
            A[r, r] += 2 / s.dx ** 2 + 2 / s.dy ** 2
            A[r, j * nx + (i + 1) % nx] -= 1 / s.dx ** 2
            A[r, j * nx + (i - 1) % nx] -= 1 / s.dx ** 2
            A[r, ((j + 1) % ny) * nx + i] -= 1 / s.dy ** 2
            A[r, ((j - 1) % ny) * nx + i] -= 1 / s.dy ** 2
    A[G, :] = 1.0
    b = np.concatenate([rho.ravel(), [0.0]])
    phi = np.linalg.lstsq(A, b, rcond=None)[0].reshape(ny, nx)
    assert np.allclose(O.solve_potential(s, rho), phi, atol=1e-12)
    Ex = -(np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)) / (2 * s.dx)
    Ey = -(np.roll(phi, -1, axis=0) - np.roll(phi, 1, axis=0)) / (2 * s.dy)
    E = O.solve_field(s, rho)
    assert np.allclose(E[0], Ex, atol=1e-12) and np.allclose(E[1], Ey, atol=1e-12)


def test_poisson_1d_scan_equals_fft():
    rng = np.random.default_rng(2)
    for nx in (5, 64, 173, 512):
        s = O.Setup(1, 1, nx, 4 * np.pi, 1, 0.1)
        rho = rng.normal(size=nx)
        (Ef,) = O.solve_field(s, rho)
        Es = O.solve_field_1d_scan(rho, s.dx)
        assert np.allclose(Ef, Es, atol=1e-13 * max(1.0, np.abs(Ef).max()))


# --------------------------------------------------- momentum conservation

def test_zero_self_force_and_pair_forces():
    rng = np.random.default_rng(4)
    s = _setup2d(16, 16, 8.0, 8.0, 1)
    for _ in range(20):
        x, y = rng.uniform(0, 8, 1), rng.uniform(0, 8, 1)
        st = O.State.from_arrays(x, np.zeros(1), y, np.zeros(1))
        E = O.solve_field(s, O.deposit(s, st))
        Epx, Epy = O.gather(s, st, E)
        assert abs(Epx[0]) < 1e-13 and abs(Epy[0]) < 1e-13
    s2 = _setup2d(16, 16, 8.0, 8.0, 2)
    for _ in range(20):
        x, y = rng.uniform(0, 8, 2), rng.uniform(0, 8, 2)
        st = O.State.from_arrays(x, np.zeros(2), y, np.zeros(2))
        E = O.solve_field(s2, O.deposit(s2, st))
        Epx, Epy = O.gather(s2, st, E)
        assert abs(Epx[0] + Epx[1]) < 1e-13 * (1 + abs(Epx[0]))
        assert abs(Epy[0] + Epy[1]) < 1e-13 * (1 + abs(Epy[0]))


def test_momentum_conserved_thermal_run():
    w = W.thermal_2d(seed=77, nx=32, ppc=16)
    x, y, vx, vy, _ = W.sample(w)
    s = _setup2d(w.nx, w.ny, w.Lx, w.Ly, w.n_particles)
    st = O.State.from_arrays(x, vx, y, vy)
    P0 = O.momentum(s, st)
    E, _ = O.initialise(s, st)
    P_half = O.momentum(s, st)
    for _ in range(20):
        E, _, _ = O.step(s, st, E)
    P1 = O.momentum(s, st)
    scale = w.n_particles * s.M * 1.0
    assert np.all(np.abs(P1 - P_half) <= 1e-12 * scale)
    assert np.all(np.abs(P_half - P0) <= 1e-12 * scale)


# ------------------------------------------------------------------- Boris

def _single(vx, vy, vz, L=100.0):
    return O.State.from_arrays(np.array([L / 2]), np.array([vx]), np.array([L / 2]),
                               np.array([vy]), np.array([vz]))


def test_boris_gyration_closed_form():
    wc, dt = 2.0, 0.05
    s = O.Setup(2, 3, 4, 100.0, 1, dt, ny=4, Ly=100.0, bz=wc)  # q/m = -1, |omega_c| = 2
    st = _single(0.8, -0.6, 0.3)
    v0 = np.array([0.8, -0.6])
    theta = 2 * np.arctan(wc * dt / 2)
    assert abs(theta - 0.0999168) < 1e-7
    zero = (np.zeros(1), np.zeros(1))
    xs, ys = [], []
    for n in range(1, 400):
        O.boris(s, st, zero, dt)
        O.move(s, st)
        xs.append(st.x[0])
        ys.append(st.y[0])
        # |v| exactly preserved up to rounding
        assert abs(np.hypot(st.vx[0], st.vy[0]) - 1.0) < 1e-14 * n + 1e-15
        # closed form: rotation by n*theta; electrons gyrate counter-clockwise for bz > 0
        c, sn = np.cos(n * theta), np.sin(n * theta)
        vx_cf = c * v0[0] - sn * v0[1]
        vy_cf = sn * v0[0] + c * v0[1]
        assert abs(st.vx[0] - vx_cf) < 1e-13 * n and abs(st.vy[0] - vy_cf) < 1e-13 * n
        assert st.vz[0] == 0.3
    # positions lie on a circle of radius r_L sqrt(1 + (wc dt/2)^2)
    xs, ys = np.array(xs) - 50.0, np.array(ys) - 50.0
    A = np.vstack([2 * xs, 2 * ys, np.ones_like(xs)]).T
    b = xs ** 2 + ys ** 2
    cx, cy, c0 = np.linalg.lstsq(A, b, rcond=None)[0]
    R = np.sqrt(c0 + cx ** 2 + cy ** 2)
    R_expect = (1.0 / wc) * np.sqrt(1 + (wc * dt / 2) ** 2)
    assert abs(R / R_expect - 1) < 1e-9
    assert abs(R_expect * wc - 1.0012492) < 1e-7


def test_boris_exb_drift_is_fixed_point():
    bz, Ex, dt = 2.0, 0.3, 0.05
    s = O.Setup(2, 3, 4, 100.0, 1, dt, ny=4, Ly=100.0, bz=bz)
    # E x B / B^2 with E = Ex x^, B = bz z^  ->  -Ex/bz y^
    vd = -Ex / bz
    st = _single(0.0, vd, 0.0)
    E = (np.array([Ex]), np.array([0.0]))
    for _ in range(100):
        O.boris(s, st, E, dt)
    assert abs(st.vx[0]) < 1e-15 and abs(st.vy[0] - vd) < 1e-15


def test_boris_reduces_to_kick_without_b():
    s = O.Setup(2, 2, 4, 10.0, 3, 0.1, ny=4, Ly=10.0)
    st = O.State.from_arrays(np.zeros(3), np.array([1.0, -2.0, 0.5]), np.zeros(3), np.array([0.0, 1.0, 2.0]))
    Ep = (np.array([0.5, 0.25, -1.0]), np.array([2.0, -0.5, 0.125]))
    O.boris(s, st, Ep, 0.1)
    assert np.allclose(st.vx, np.array([1.0, -2.0, 0.5]) - 0.1 * Ep[0], rtol=0, atol=1e-15)
    assert np.allclose(st.vy, np.array([0.0, 1.0, 2.0]) - 0.1 * Ep[1], rtol=0, atol=1e-15)


# -------------------------------------------------------------------- sort

def test_counting_sort_bruteforce():
    rng = np.random.default_rng(6)
    nx, ny, tx, ty = 20, 12, 4, 4
    ix = rng.integers(0, nx, 3000)
    iy = rng.integers(0, ny, 3000)
    key = O.bucket_key(ix, iy, tx, ty, nx)
    nb = 5 * 3
    perm, start = O.counting_sort(key, nb)
    # brute force: walk buckets in order, keep input order inside a bucket
    bf = [i for b in range(nb) for i in range(len(key)) if key[i] == b]
    assert np.array_equal(perm, np.array(bf))
    for b in range(nb):
        assert start[b] == sum(1 for k in key if k < b)
    assert start[-1] == len(key)
    assert key.max() < nb and np.all(key == (iy // ty) * 5 + ix // tx)
