"""Pins of the oracle's Gaussian line fitting (the alternative to moments of
Bekiaris et al. 2016, Sec. 2.2.5, fitted on the CPU with mpfit in Sec. 5.2).

Noise-free Gaussian spectra give their parameters back; noisy spectra give
scipy's least-squares optimum; a whole-channel shift moves only the centre
and a scale factor only the amplitude; an empty spectrum has no line.
"""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import fitters as F

DV = 20.0
V = -600.0 + DV * np.arange(61)


def gauss(v, a, m, s):
    return a * np.exp(-0.5 * ((v - m) / s) ** 2)


@pytest.mark.parametrize("a,m,s", [(1.0, 13.7, 45.0), (3.5, -222.2, 18.0), (0.02, 301.0, 90.0)])
def test_noise_free_lines_come_back(a, m, s):
    f = F.fit_gaussian_line(gauss(V, a, m, s), V, DV)
    assert f.status == 1
    assert abs(f.amp - a) <= 1e-8 * a and abs(f.vel - m) <= 1e-7 and abs(f.disp - s) <= 1e-7


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_noisy_lines_reach_the_least_squares_optimum(seed):
    rng = np.random.default_rng([77, seed])
    a, m, s = 2.0, rng.uniform(-200, 200), rng.uniform(25, 70)
    spec = gauss(V, a, m, s) + 0.1 * rng.standard_normal(V.size)
    f = F.fit_gaussian_line(spec, V, DV)
    ref, cov = curve_fit(gauss, V, spec, p0=(a, m, s), xtol=1e-14, ftol=1e-14, gtol=1e-14)
    err = np.sqrt(np.diag(cov))
    assert f.status == 1
    for got, want, e in zip((f.amp, f.vel, f.disp), ref, err):
        assert abs(got - want) <= 1e-4 * e, (got, want, e)


def test_shift_and_scale_invariance():
    rng = np.random.default_rng(5)
    spec = gauss(V, 1.5, -40.0, 35.0) + 0.05 * rng.standard_normal(V.size)
    f0 = F.fit_gaussian_line(spec, V, DV)
    f1 = F.fit_gaussian_line(spec, V + 3 * DV, DV)          # same spectrum, shifted band
    assert abs(f1.vel - (f0.vel + 3 * DV)) <= 1e-7
    assert abs(f1.disp - f0.disp) <= 1e-7 and abs(f1.amp - f0.amp) <= 1e-9
    f2 = F.fit_gaussian_line(4.0 * spec, V, DV)
    assert abs(f2.amp - 4.0 * f0.amp) <= 1e-8 and abs(f2.vel - f0.vel) <= 1e-7
    assert abs(f2.disp - f0.disp) <= 1e-7


def test_flux_is_the_line_area_and_empty_spectra_have_no_line():
    cube = np.zeros((V.size, 1, 2))
    cube[:, 0, 0] = gauss(V, 2.0, 10.0, 40.0)
    maps, st = F.fit_gaussian_lines(cube, V, DV)
    assert st[0, 0] == 1 and st[0, 1] == 0
    # a well-sampled Gaussian's area equals dv times its channel sum
    assert abs(maps[0, 0, 0] - DV * cube[:, 0, 0].sum()) <= 1e-9 * maps[0, 0, 0]
    assert maps[0, 0, 1] == 0.0 and math.isnan(maps[1, 0, 1]) and math.isnan(maps[2, 0, 1])
