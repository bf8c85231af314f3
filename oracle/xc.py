"""Oracle: local density approximation, spin-unpolarized (Section 2.1).

TEST INFRASTRUCTURE ONLY.

The paper takes "the LDA" from a library without naming the functional.  The
reading used here is Slater exchange plus the Perdew-Wang 1992 correlation
fit, Hartree atomic units, written from the published formulas:

  r_s   = (3 / (4 pi rho))^(1/3)
  eps_x = -(3/4) (3 rho / pi)^(1/3),            v_x = (4/3) eps_x
  eps_c = -2A (1 + a1 r_s) ln(1 + 1 / (2A (b1 r_s^1/2 + b2 r_s + b3 r_s^3/2 + b4 r_s^2)))
  v_c   = eps_c - (r_s / 3) d eps_c / d r_s

The potential is the derivative of the energy density, v = d(rho eps)/d rho
(reading of the garbled definition of V_xc, consistent with E_xc = int eps rho).
Densities below RHO_FLOOR are treated as vacuum: eps = v = 0.
"""
from __future__ import annotations

import math

import numpy as np

PW92_A = 0.031091
PW92_ALPHA1 = 0.21370
PW92_BETA = (7.5957, 3.5876, 1.6382, 0.49294)
RHO_FLOOR = 1e-30


def slater_exchange(rho: np.ndarray):
    c = (3.0 * rho / math.pi) ** (1.0 / 3.0)
    eps = -0.75 * c
    return eps, -c


def pw92_correlation(rs: np.ndarray):
    A, a1 = PW92_A, PW92_ALPHA1
    b1, b2, b3, b4 = PW92_BETA
    srs = np.sqrt(rs)
    Q0 = -2.0 * A * (1.0 + a1 * rs)
    Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    Q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)   # dQ1/drs
    lg = np.log1p(1.0 / Q1)
    eps = Q0 * lg
    deps = -2.0 * A * a1 * lg - Q0 * Q1p / (Q1 * Q1 + Q1)
    v = eps - rs / 3.0 * deps
    return eps, v


def lda_xc(rho: np.ndarray):
    """Energy per particle eps_xc(rho) and potential v_xc(rho), elementwise."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.zeros_like(rho)
    v = np.zeros_like(rho)
    m = rho > RHO_FLOOR
    r = rho[m]
    ex, vx = slater_exchange(r)
    rs = (3.0 / (4.0 * math.pi * r)) ** (1.0 / 3.0)
    ec, vc = pw92_correlation(rs)
    eps[m] = ex + ec
    v[m] = vx + vc
    return eps, v
