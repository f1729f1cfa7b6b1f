"""Linear-theory roots used to pin the oracle's plasma physics.

TEST INFRASTRUCTURE ONLY.

* Warm symmetric two-stream (and, with zero drift, single-Maxwellian Landau)
  dielectric function of the paper's "Results and validation" section:
      eps(w, k) = 1 + 1/(2 (k lambda_D)^2) sum_{s=+-1} [1 + zeta_s Z(zeta_s)],
      zeta_s = (w - s k_x u_d) / (sqrt(2) k v_te),
  with Z the plasma dispersion function, Z(z) = i sqrt(pi) w(z) (Faddeeva w).
  lambda_D = v_te / omega_pe, omega_pe = 1.
* Electron Bernstein waves (perpendicular propagation, uniform B, Maxwellian):
      1 + (1/(k lambda_D)^2) [1 - sum_n w/(w - n w_c) I_n(b) e^{-b}] = 0,
      b = (k v_th / w_c)^2.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import fsolve
from scipy.special import ive, wofz


def plasma_z(z):
    return 1j * np.sqrt(np.pi) * wofz(z)


def two_stream_eps(w: complex, k: float, kx: float, ud: float, vte: float) -> complex:
    tot = 0.0 + 0.0j
    for sgn in (1.0, -1.0):
        zeta = (w - sgn * kx * ud) / (np.sqrt(2.0) * k * vte)
        tot += 1.0 + zeta * plasma_z(zeta)
    return 1.0 + tot / (2.0 * (k * vte) ** 2)


def two_stream_root(k: float, kx: float, ud: float, vte: float, guess: complex) -> complex:
    f = lambda p: [two_stream_eps(p[0] + 1j * p[1], k, kx, ud, vte).real,
                   two_stream_eps(p[0] + 1j * p[1], k, kx, ud, vte).imag]
    r = fsolve(f, [guess.real, guess.imag], xtol=1e-14)
    return complex(r[0], r[1])


def bernstein_eps(w: float, k: float, wc: float, vth: float, nmax: int = 60) -> float:
    b = (k * vth / wc) ** 2
    s = 0.0
    for n in range(-nmax, nmax + 1):
        s += w / (w - n * wc) * ive(abs(n), b)
    return 1.0 + (1.0 - s) / (k * vth) ** 2


def bernstein_root(k: float, wc: float, vth: float, guess: float) -> float:
    r = fsolve(lambda p: [bernstein_eps(p[0], k, wc, vth)], [guess], xtol=1e-14)
    return float(r[0])


def cold_two_stream_growth(a: float) -> float:
    """Cold symmetric two-stream growth rate at a = k u_d / omega_pe (each
    beam carrying half the density): gamma^2 = (sqrt(8 a^2 + 1) - (2 a^2 + 1))/2."""
    g2 = (np.sqrt(8 * a * a + 1) - (2 * a * a + 1)) / 2.0
    return float(np.sqrt(max(g2, 0.0)))
