"""Pins of the oracle's LDA (Slater exchange + PW92 correlation)."""
import math

import numpy as np

from oracle import xc


def _rs(rho):
    return (3.0 / (4.0 * math.pi * rho)) ** (1.0 / 3.0)


def test_slater_exchange_uniform_gas_constant():
    # Dirac exchange of the uniform gas: eps_x = -(3/(4 pi)) (9 pi / 4)^(1/3) / r_s
    c = 3.0 / (4.0 * math.pi) * (9.0 * math.pi / 4.0) ** (1.0 / 3.0)
    assert abs(c - 0.458165) < 1e-6
    rho = np.array([1e-4, 1e-2, 0.3, 10.0])
    ex, _ = xc.slater_exchange(rho)
    assert np.allclose(ex, -c / _rs(rho), rtol=1e-13)


def test_potential_is_derivative_of_energy_density():
    rho = np.geomspace(1e-6, 1e3, 40)
    h = 1e-6 * rho
    ep, _ = xc.lda_xc(rho + h)
    em, _ = xc.lda_xc(rho - h)
    fd = ((rho + h) * ep - (rho - h) * em) / (2 * h)
    _, v = xc.lda_xc(rho)
    assert np.allclose(v, fd, rtol=1e-7)


def test_pw92_high_density_limit():
    """Gell-Mann--Brueckner: eps_c -> c0 ln r_s - c1 as r_s -> 0, with
    c0 = (1 - ln 2) / pi^2 and c1 = 0.046644; PW92's A and beta_1 are fixed by
    these (A = c0, beta_1 = exp(-c1 / (2A)) / (2A), beta_2 = 2 A beta_1^2)."""
    c0 = (1.0 - math.log(2.0)) / math.pi ** 2
    c1 = 0.046644
    assert abs(xc.PW92_A - c0) <= 5e-7          # A is published rounded to 6 decimals
    b1 = math.exp(-c1 / (2 * c0)) / (2 * c0)
    assert abs(xc.PW92_BETA[0] - b1) < 2e-3
    assert abs(xc.PW92_BETA[1] - 2 * c0 * b1 ** 2) < 2e-3
    for rs in (1e-6, 1e-8):
        ec, _ = xc.pw92_correlation(np.array([rs]))
        assert abs(ec[0] - (c0 * math.log(rs) - c1)) < 5 * math.sqrt(rs) + 1e-4


def test_correlation_is_negative_and_vanishes_at_low_density():
    rs = np.geomspace(1e-3, 1e4, 50)
    ec, vc = xc.pw92_correlation(rs)
    assert np.all(ec < 0) and np.all(np.diff(ec) > 0)       # |eps_c| decreases with r_s
    assert abs(ec[-1]) < 1e-3
    eps, v = xc.lda_xc(np.array([0.0, 1e-40]))
    assert np.all(eps == 0) and np.all(v == 0)
