"""Serial FP64 CPU reference for the PIC particle-grid coupling loop.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the CPU-baseline leg of the benchmark, never by the product library. It
shares no code with the HIP path; the two meet only through the seeded input
generators, which hold none of the method's arithmetic.

What it computes follows the paper (AlgoPlasma):
  * the modules of the particle-grid coupling loop ("Core functionality":
    I_Initializer, A_Pusher with the Boris pusher, B_Scatter, C_Gather,
    D_Poisson), written out from the textbook schemes the paper cites;
  * the PIC cycle of the two-stream example's application driver ("Example
    setup and implementation"): field from the initial charge, initial half
    push, then per step full push -> position update with periodic wrap ->
    deposit -> Poisson -> field;
  * the diagnostics of "Results and validation": field and kinetic energy,
    total-energy error normalised by the initial total energy, Fourier
    amplitude 2|E_par(m)| of a seeded mode and its least-squares growth rate.

Particle loops live in ``apic_oracle.c`` (plain serial C, FP64, built with
gcc -O2 -ffp-contract=off); the periodic Poisson solve uses numpy's FFT as a
library primitive. Normalised units: omega_pe = 1, eps0 = 1, electron q/m = -1,
n0 = 1, immobile uniform ion background rho_ion = +n0.

Readings where the paper is silent (each listed with its reason in the design
notes of the repository):
  * node-centred periodic grid X_j = j*dx, linear (CIC) weights;
  * Poisson: the periodic 7-point (3D) / 5-point (2D) / 3-point (1D)
    finite-difference Laplacian, solved exactly in Fourier space with the
    modified wavenumber
    K^2 = sum_d (2/d_d)^2 sin^2(k_d d_d / 2); the k = 0 mode is zero;
  * E = -(centred difference of phi), i.e. E_hat = -i sin(k d)/d * phi_hat;
  * initial half push: backward, v^{-1/2} = Boris(v^0, E^0, -dt/2);
  * kinetic energy at integer time: mean of the two half-step values;
  * field energy: 1/2 sum_j |E_j|^2 dV.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apic_oracle.c")
_SO = os.path.join(_HERE, "_apic_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (serial, FP64, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    from . import em
    em.build(force)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build(force=True)
    L = ctypes.CDLL(_SO)
    sig = {
        "or_deposit_1d": [_i64, _D, _int, _dbl, _dbl, _D],
        "or_deposit_2d": [_i64, _D, _D, _int, _int, _dbl, _dbl, _dbl, _D],
        "or_deposit_3d": [_i64, _D, _D, _D, _int, _int, _int, _dbl, _dbl, _dbl, _dbl, _D],
        "or_deposit_q_3d": [_i64, _I32, _I32, _I32, _F, _F, _F, _int, _int, _int, _int, _I64],
        "or_gather_3d": [_i64, _D, _D, _D, _int, _int, _int, _dbl, _dbl, _dbl, _D, _D, _D, _D, _D, _D],
        "or_move_3d": [_i64, _D, _D, _D, _D, _D, _D, _dbl, _dbl, _dbl, _dbl],
        "or_hc": [_i64, _D, _D, _D, _D, _D, _D, _dbl, _dbl, _dbl, _dbl],
        "or_move_u": [_i64, _int, _D, _D, _D, _D, _D, _D, _dbl, _dbl, _dbl, _dbl, _dbl],
        "or_deposit_q_1d": [_i64, _I32, _F, _int, _int, _I64],
        "or_deposit_q_2d": [_i64, _I32, _I32, _F, _F, _int, _int, _int, _I64],
        "or_gather_1d": [_i64, _D, _int, _dbl, _D, _D],
        "or_gather_2d": [_i64, _D, _D, _int, _int, _dbl, _dbl, _D, _D, _D, _D],
        "or_boris": [_i64, _int, _D, _D, _D, _D, _D, _D, _dbl, _dbl, _dbl],
        "or_move_1d": [_i64, _D, _D, _dbl, _dbl],
        "or_move_2d": [_i64, _D, _D, _D, _D, _dbl, _dbl, _dbl],
        "or_adj_deposit_1d": [_i64, _D, _int, _dbl, _dbl, _D, _D],
        "or_adj_deposit_2d": [_i64, _D, _D, _int, _int, _dbl, _dbl, _dbl, _D, _D, _D],
        "or_adj_gather_1d": [_i64, _D, _int, _dbl, _D, _D, _D, _D],
        "or_adj_gather_2d": [_i64, _D, _D, _int, _int, _dbl, _dbl, _D, _D, _D, _D, _D, _D, _D, _D],
        "or_adj_boris": [_i64, _int, _D, _D, _D, _D, _dbl, _dbl, _dbl],
        "or_adj_deposit_3d": [_i64, _D, _D, _D, _int, _int, _int, _dbl, _dbl, _dbl, _dbl, _D, _D, _D, _D],
        "or_adj_gather_3d": [_i64, _D, _D, _D, _int, _int, _int, _dbl, _dbl, _dbl, _D, _D, _D, _D, _D, _D, _D, _D,
                             _D, _D, _D, _D],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = None
    _lib = L
    return L


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ct)


def _c64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


# ---------------------------------------------------------------------------
# Problem description (units and charges; "Example setup and implementation")
# ---------------------------------------------------------------------------

@dataclass
class Setup:
    """One periodic electrostatic plasma.

    dim: 1, 2 or 3 spatial dimensions; vdim: 1, 2 or 3 velocity components
    (3 when dim = 3). nx, ny, nz: grid nodes per axis (ny = 1 in 1D, nz = 1
    below 3D); Lx, Ly, Lz: box lengths.
    n_particles: number of macro-electrons N. Macro charge Q = -n0 V / N and
    mass M = n0 V / N (so q/m = -1); ions are a uniform +n0 background."""
    dim: int
    vdim: int
    nx: int
    Lx: float
    n_particles: int
    dt: float
    ny: int = 1
    Ly: float = 1.0
    qm: float = -1.0
    bz: float = 0.0
    n0: float = 1.0
    nz: int = 1
    Lz: float = 1.0
    # velocity advance: "boris", or "hc" (Higuera-Cary; the state's velocities
    # are then u = gamma v, and c is the speed of light; needs vdim = 3)
    pusher: str = "boris"
    c: float = float("inf")

    @property
    def dx(self):
        return self.Lx / self.nx

    @property
    def dy(self):
        return self.Ly / self.ny if self.dim >= 2 else 1.0

    @property
    def dz(self):
        return self.Lz / self.nz if self.dim == 3 else 1.0

    @property
    def volume(self):
        return self.Lx * (self.Ly if self.dim >= 2 else 1.0) * (self.Lz if self.dim == 3 else 1.0)

    @property
    def dV(self):
        return self.dx * self.dy * self.dz

    @property
    def Q(self):
        return -self.n0 * self.volume / self.n_particles

    @property
    def M(self):
        return self.n0 * self.volume / self.n_particles

    @property
    def rho_ion(self):
        return self.n0

    @property
    def grid_shape(self):
        return {1: (self.nx,), 2: (self.ny, self.nx), 3: (self.nz, self.ny, self.nx)}[self.dim]


@dataclass
class State:
    """FP64 particle state (structure of arrays); unused components are None."""
    x: np.ndarray
    vx: np.ndarray
    y: Optional[np.ndarray] = None
    vy: Optional[np.ndarray] = None
    vz: Optional[np.ndarray] = None
    z: Optional[np.ndarray] = None

    def copy(self):
        c = lambda a: None if a is None else a.copy()
        return State(c(self.x), c(self.vx), c(self.y), c(self.vy), c(self.vz), c(self.z))

    @staticmethod
    def from_arrays(x, vx, y=None, vy=None, vz=None, z=None):
        c = lambda a: None if a is None else _c64(a).copy()
        return State(c(x), c(vx), c(y), c(vy), c(vz), c(z))


# ---------------------------------------------------------------------------
# B_Scatter: charge deposition
# ---------------------------------------------------------------------------

def deposit(s: Setup, st: State) -> np.ndarray:
    """rho_j = rho_ion + (Q/dV) sum_p W_j(x_p) with CIC weights (FP64)."""
    L = _load()
    n = st.x.shape[0]
    rho = np.full(s.grid_shape, s.rho_ion, dtype=np.float64)
    c = s.Q / s.dV
    _deposit_into(L, s, st, c, rho)
    return rho


def _deposit_into(L, s: Setup, st: State, c: float, out: np.ndarray) -> None:
    n = st.x.shape[0]
    if s.dim == 1:
        L.or_deposit_1d(n, _p(st.x, _D), s.nx, s.dx, c, _p(out, _D))
    elif s.dim == 2:
        L.or_deposit_2d(n, _p(st.x, _D), _p(st.y, _D), s.nx, s.ny, s.dx, s.dy, c, _p(out, _D))
    else:
        L.or_deposit_3d(n, _p(st.x, _D), _p(st.y, _D), _p(st.z, _D), s.nx, s.ny, s.nz, s.dx, s.dy, s.dz, c,
                        _p(out, _D))


def deposit_counts(s: Setup, st: State) -> np.ndarray:
    """Sum of CIC weights per node (no charge scale, no ion background)."""
    L = _load()
    n = st.x.shape[0]
    w = np.zeros(s.grid_shape, dtype=np.float64)
    _deposit_into(L, s, st, 1.0, w)
    return w


def deposit_quantised(s: Setup, ix, ox, frac_bits: int, iy=None, oy=None, iz=None, oz=None) -> np.ndarray:
    """Integer CIC deposit: I_j = sum_p w_pj with w = round-half-even(o 2^S).

    ix/iy/iz: int32 cell indices, ox/oy/oz: float32 in-cell offsets in [0,1).
    Returns the int64 node sums; each particle contributes exactly 2^(S*dim)."""
    L = _load()
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    ox = np.ascontiguousarray(ox, dtype=np.float32)
    n = ix.shape[0]
    I = np.zeros(s.grid_shape, dtype=np.int64)
    if s.dim == 1:
        L.or_deposit_q_1d(n, _p(ix, _I32), _p(ox, _F), s.nx, frac_bits, _p(I, _I64))
    elif s.dim == 3:
        a = [np.ascontiguousarray(v, dtype=np.int32) for v in (iy, iz)]
        o = [np.ascontiguousarray(v, dtype=np.float32) for v in (oy, oz)]
        L.or_deposit_q_3d(n, _p(ix, _I32), _p(a[0], _I32), _p(a[1], _I32), _p(ox, _F), _p(o[0], _F),
                          _p(o[1], _F), s.nx, s.ny, s.nz, frac_bits, _p(I, _I64))
    else:
        iy = np.ascontiguousarray(iy, dtype=np.int32)
        oy = np.ascontiguousarray(oy, dtype=np.float32)
        L.or_deposit_q_2d(n, _p(ix, _I32), _p(iy, _I32), _p(ox, _F), _p(oy, _F),
                          s.nx, s.ny, frac_bits, _p(I, _I64))
    return I


def rho_from_quantised(s: Setup, I: np.ndarray, frac_bits: int) -> np.ndarray:
    """rho_j = rho_ion + Q * I_j * 2^(-S*dim) / dV (FP64)."""
    scale = s.Q * np.ldexp(1.0, -frac_bits * s.dim) / s.dV
    return s.rho_ion + I.astype(np.float64) * scale


# ---------------------------------------------------------------------------
# D_Poisson: periodic finite-difference Poisson solve and E = -grad(phi)
# ---------------------------------------------------------------------------

def _kvec(n: int, d: float) -> np.ndarray:
    return 2.0 * np.pi * np.fft.fftfreq(n, d=d)


def modified_k2(n: int, d: float) -> np.ndarray:
    """Eigenvalues of minus the periodic 3-point second difference."""
    k = _kvec(n, d)
    return (2.0 / d * np.sin(k * d / 2.0)) ** 2


def centred_kappa(n: int, d: float) -> np.ndarray:
    """Eigenvalues (divided by i) of the periodic centred first difference."""
    k = _kvec(n, d)
    return np.sin(k * d) / d


def _axes(s: Setup):
    """(n, d) per array axis of the grid, outermost first."""
    return {1: [(s.nx, s.dx)], 2: [(s.ny, s.dy), (s.nx, s.dx)],
            3: [(s.nz, s.dz), (s.ny, s.dy), (s.nx, s.dx)]}[s.dim]


def _broadcast(v: np.ndarray, axis: int, ndim: int) -> np.ndarray:
    shape = [1] * ndim
    shape[axis] = v.shape[0]
    return v.reshape(shape)


def _k2_grid(s: Setup) -> np.ndarray:
    """Sum over axes of the modified wavenumbers: the symbol of -lap_h."""
    ax = _axes(s)
    K2 = 0.0
    for a, (n, d) in enumerate(ax):
        K2 = K2 + _broadcast(modified_k2(n, d), a, len(ax))
    return np.broadcast_to(K2, tuple(n for n, _ in ax)).copy()


def solve_potential(s: Setup, rho: np.ndarray) -> np.ndarray:
    """phi with -lap_h phi = rho, sum(phi) = 0 (the k = 0 mode is dropped)."""
    K2 = _k2_grid(s)
    rh = np.fft.fftn(rho)
    K2.flat[0] = 1.0
    ph = rh / K2
    ph.flat[0] = 0.0
    return np.real(np.fft.ifftn(ph))


def solve_field(s: Setup, rho: np.ndarray) -> Tuple[np.ndarray, ...]:
    """E = -centred_grad(phi) of the FD Poisson solution, via FFT.

    Returns (E,) in 1D, (Ex, Ey) in 2D and (Ex, Ey, Ez) in 3D, FP64, on the
    nodes."""
    if s.dim == 3:
        K2 = _k2_grid(s)
        K2[0, 0, 0] = 1.0
        ph = np.fft.fftn(rho) / K2
        ph[0, 0, 0] = 0.0
        out = []
        for a, (n, d) in reversed(list(enumerate(_axes(s)))):   # x, then y, then z
            Eh = -1j * _broadcast(centred_kappa(n, d), a, 3) * ph
            out.append(np.real(np.fft.ifftn(Eh)))
        return tuple(out)
    if s.dim == 1:
        K2 = modified_k2(s.nx, s.dx).copy()
        rh = np.fft.fft(rho)
        K2[0] = 1.0
        ph = rh / K2
        ph[0] = 0.0
        Eh = -1j * centred_kappa(s.nx, s.dx) * ph
        return (np.real(np.fft.ifft(Eh)),)
    K2 = modified_k2(s.ny, s.dy)[:, None] + modified_k2(s.nx, s.dx)[None, :]
    K2[0, 0] = 1.0
    rh = np.fft.fft2(rho)
    ph = rh / K2
    ph[0, 0] = 0.0
    Exh = -1j * centred_kappa(s.nx, s.dx)[None, :] * ph
    Eyh = -1j * centred_kappa(s.ny, s.dy)[:, None] * ph
    return (np.real(np.fft.ifft2(Exh)), np.real(np.fft.ifft2(Eyh)))


def solve_field_1d_scan(rho: np.ndarray, dx: float) -> np.ndarray:
    """1D periodic field by Gauss's law on the staggered half nodes.

    From -(phi_{j+1} - 2 phi_j + phi_{j-1})/dx^2 = rho_j with
    E_{j+1/2} = -(phi_{j+1} - phi_j)/dx it follows E_{j+1/2} - E_{j-1/2} =
    rho_j dx; periodicity of phi fixes sum_j E_{j+1/2} = 0, and the node field
    is the centred difference E_j = (E_{j-1/2} + E_{j+1/2})/2. The mean of rho
    is removed first (the k = 0 mode carries no field)."""
    r = rho - rho.mean()
    half = np.cumsum(r * dx)          # E_{j+1/2} up to a constant
    half = half - half.mean()
    prev = np.roll(half, 1)           # E_{j-1/2}
    return 0.5 * (prev + half)


# ---------------------------------------------------------------------------
# C_Gather, A_Pusher (Boris) and the position update
# ---------------------------------------------------------------------------

def gather(s: Setup, st: State, E) -> Tuple[np.ndarray, ...]:
    L = _load()
    n = st.x.shape[0]
    if s.dim == 1:
        Ep = np.empty(n)
        L.or_gather_1d(n, _p(st.x, _D), s.nx, s.dx, _p(_c64(E[0]), _D), _p(Ep, _D))
        return (Ep,)
    if s.dim == 3:
        Ex, Ey, Ez = (_c64(e) for e in E)
        Ep = [np.empty(n) for _ in range(3)]
        L.or_gather_3d(n, _p(st.x, _D), _p(st.y, _D), _p(st.z, _D), s.nx, s.ny, s.nz, s.dx, s.dy, s.dz,
                       _p(Ex, _D), _p(Ey, _D), _p(Ez, _D), *[_p(e, _D) for e in Ep])
        return tuple(Ep)
    Ex, Ey = _c64(E[0]), _c64(E[1])
    Epx = np.empty(n)
    Epy = np.empty(n)
    L.or_gather_2d(n, _p(st.x, _D), _p(st.y, _D), s.nx, s.ny, s.dx, s.dy,
                   _p(Ex, _D), _p(Ey, _D), _p(Epx, _D), _p(Epy, _D))
    return (Epx, Epy)


def boris(s: Setup, st: State, Ep, dt: float) -> None:
    """In-place velocity advance by dt under Ep and bz: Boris, or Higuera-Cary
    when s.pusher == "hc"."""
    L = _load()
    n = st.x.shape[0]
    Epy = Ep[1] if len(Ep) > 1 else None
    Epz = Ep[2] if len(Ep) > 2 else None
    if s.pusher == "hc":
        L.or_hc(n, _p(st.vx, _D), _p(st.vy, _D), _p(st.vz, _D), _p(_c64(Ep[0]), _D), _p(_c64(Epy), _D),
                _p(None if Epz is None else _c64(Epz), _D), s.qm, dt, s.bz, s.c)
        return
    L.or_boris(n, s.vdim, _p(st.vx, _D), _p(st.vy, _D), _p(st.vz, _D),
               _p(_c64(Ep[0]), _D), _p(None if Epy is None else _c64(Epy), _D),
               _p(None if Epz is None else _c64(Epz), _D), s.qm, dt, s.bz)


def move(s: Setup, st: State) -> None:
    L = _load()
    n = st.x.shape[0]
    if s.pusher == "hc":
        L.or_move_u(n, s.dim, _p(st.x, _D), _p(st.y, _D), _p(st.z, _D), _p(st.vx, _D), _p(st.vy, _D),
                    _p(st.vz, _D), s.dt, s.c, s.Lx, s.Ly, s.Lz)
        return
    if s.dim == 1:
        L.or_move_1d(n, _p(st.x, _D), _p(st.vx, _D), s.dt, s.Lx)
    elif s.dim == 2:
        L.or_move_2d(n, _p(st.x, _D), _p(st.y, _D), _p(st.vx, _D), _p(st.vy, _D), s.dt, s.Lx, s.Ly)
    else:
        L.or_move_3d(n, _p(st.x, _D), _p(st.y, _D), _p(st.z, _D), _p(st.vx, _D), _p(st.vy, _D), _p(st.vz, _D),
                     s.dt, s.Lx, s.Ly, s.Lz)


# ---------------------------------------------------------------------------
# Counting sort by cell bucket (the plain definition: stable sort by key)
# ---------------------------------------------------------------------------

def bucket_key(ix, iy, tile_x: int, tile_y: int, nx: int, iz=None, tile_z: int = 1, ny: int = 1) -> np.ndarray:
    """Bucket index of a cell: tiles of tile_x * tile_y (* tile_z) cells,
    tiles numbered x fastest, then y, then z."""
    nbx = -(-nx // tile_x)
    ix = np.asarray(ix, dtype=np.int64)
    if iy is None:
        return (ix // tile_x).astype(np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    key = (iy // tile_y) * nbx + ix // tile_x
    if iz is None:
        return key
    nby = -(-ny // tile_y)
    return (np.asarray(iz, dtype=np.int64) // tile_z) * (nbx * nby) + key


def counting_sort(keys: np.ndarray, n_buckets: int):
    """Stable ascending sort by integer key.

    Returns (perm, start): sorted[i] = input[perm[i]]; start[b] is the first
    sorted position of bucket b, start[n_buckets] = len(keys)."""
    keys = np.asarray(keys, dtype=np.int64)
    perm = np.argsort(keys, kind="stable")
    counts = np.bincount(keys, minlength=n_buckets)
    start = np.zeros(n_buckets + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    return perm, start


# ---------------------------------------------------------------------------
# Diagnostics ("Results and validation")
# ---------------------------------------------------------------------------

def field_energy(s: Setup, E) -> float:
    return 0.5 * sum(float(np.sum(e * e)) for e in E) * s.dV


def kinetic_sum(s: Setup, st: State) -> float:
    """Sum over particles of twice the kinetic energy per unit mass: |v|^2,
    or 2 (gamma - 1) c^2 = 2 |u|^2 / (gamma + 1) for the Higuera-Cary state."""
    if s.pusher != "hc":
        return kinetic_sum_v2(st)
    u2 = st.vx * st.vx + st.vy * st.vy + st.vz * st.vz
    g = np.sqrt(1.0 + u2 / (s.c * s.c))
    return float(np.sum(2.0 * u2 / (g + 1.0)))


def kinetic_sum_v2(st: State) -> float:
    tot = float(np.dot(st.vx, st.vx))
    if st.vy is not None:
        tot += float(np.dot(st.vy, st.vy))
    if st.vz is not None:
        tot += float(np.dot(st.vz, st.vz))
    return tot


def momentum(s: Setup, st: State) -> np.ndarray:
    comps = [st.vx, st.vy, st.vz]
    return np.array([s.M * float(np.sum(c)) for c in comps if c is not None])


def mode_amplitude(s: Setup, E, mx: int, my: int = 0) -> float:
    """2|E_par_hat(m)| with E_par = k.E/|k| and E_hat = mean_j E_j e^{-i k.X_j}.
    In 3D the mode is (mx, my, 0)."""
    if s.dim == 3:
        kx = 2 * np.pi * mx / s.Lx
        ky = 2 * np.pi * my / s.Ly
        kk = np.hypot(kx, ky)
        epar = (kx * E[0] + ky * E[1]) / kk
        Eh = np.fft.fftn(epar) / (s.nx * s.ny * s.nz)
        return 2.0 * abs(Eh[0, my % s.ny, mx % s.nx])
    if s.dim == 1:
        e = E[0]
        Eh = np.fft.fft(e) / s.nx
        return 2.0 * abs(Eh[mx % s.nx])
    kx = 2 * np.pi * mx / s.Lx
    ky = 2 * np.pi * my / s.Ly
    kk = np.hypot(kx, ky)
    epar = (kx * E[0] + ky * E[1]) / kk
    Eh = np.fft.fft2(epar) / (s.nx * s.ny)
    return 2.0 * abs(Eh[my % s.ny, mx % s.nx])


def growth_rate(t: np.ndarray, amp: np.ndarray, t0: float, t1: float):
    """Least-squares slope of ln(amp) over t0 <= t <= t1, and its R^2."""
    sel = (t >= t0) & (t <= t1)
    tt = t[sel]
    yy = np.log(amp[sel])
    A = np.vstack([tt, np.ones_like(tt)]).T
    coef, *_ = np.linalg.lstsq(A, yy, rcond=None)
    pred = A @ coef
    ss_res = float(np.sum((yy - pred) ** 2))
    ss_tot = float(np.sum((yy - yy.mean()) ** 2))
    return float(coef[0]), 1.0 - ss_res / ss_tot


# ---------------------------------------------------------------------------
# The PIC cycle of the two-stream driver
# ---------------------------------------------------------------------------

@dataclass
class History:
    t: list = field(default_factory=list)
    WE: list = field(default_factory=list)
    KE: list = field(default_factory=list)
    charge: list = field(default_factory=list)
    modes: list = field(default_factory=list)
    momentum: list = field(default_factory=list)

    def arrays(self):
        return {k: np.asarray(v) for k, v in self.__dict__.items()}


def initialise(s: Setup, st: State):
    """Field of the initial charge, then the backward half push to v^{-1/2}.

    Returns E^0 and the particle kinetic sum |v^0|^2 (for the t = 0 energy)."""
    rho = deposit(s, st)
    E = solve_field(s, rho)
    v2_0 = kinetic_sum(s, st)
    boris(s, st, gather(s, st, E), -0.5 * s.dt)
    return E, v2_0


def step(s: Setup, st: State, E):
    """One leapfrog cycle: v^{n-1/2} -> v^{n+1/2} under E^n, x^n -> x^{n+1},
    deposit -> Poisson -> E^{n+1}. Returns (E^{n+1}, rho^{n+1}, KE^n) with KE^n
    the mean of the half-step kinetic energies around time level n."""
    v2_old = kinetic_sum(s, st)
    boris(s, st, gather(s, st, E), s.dt)
    v2_new = kinetic_sum(s, st)
    move(s, st)
    rho = deposit(s, st)
    E_new = solve_field(s, rho)
    KE = 0.5 * s.M * 0.5 * (v2_old + v2_new)
    return E_new, rho, KE


def run(s: Setup, st: State, nsteps: int, modes=(), every: int = 1) -> History:
    """Initialise and advance nsteps cycles, recording diagnostics.

    Record n (time t = n dt) holds W_E^n, KE^n, the deposited charge and the
    seeded-mode amplitudes of E^n. KE^0 uses |v^0|^2; KE^n for n >= 1 is the
    mean of the half-step values around n."""
    h = History()
    E, v2_0 = initialise(s, st)
    rho = deposit(s, st)
    n = 0

    def record(n, E, KE, rho):
        h.t.append(n * s.dt)
        h.WE.append(field_energy(s, E))
        h.KE.append(KE)
        h.charge.append(float(np.sum(rho - s.rho_ion)) * s.dV)
        h.modes.append([mode_amplitude(s, E, *m) for m in modes])
        h.momentum.append(momentum(s, st))

    pending_E, pending_rho = E, rho
    record(0, E, 0.5 * s.M * v2_0, rho)
    for n in range(nsteps):
        E_new, rho_new, KE_n = step(s, st, pending_E)
        if n > 0 and n % every == 0:
            record(n, pending_E, KE_n, pending_rho)
        pending_E, pending_rho = E_new, rho_new
    return h
