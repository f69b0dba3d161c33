"""Pins of the oracle's Levenberg-Marquardt against closed forms."""
import math

import numpy as np
import pytest

from oracle import fitters as F
from paper_1510_01815_amd import inputs as I


def test_lm_linear_least_squares_matches_lstsq():
    """A linear residual r = X p - y is solved exactly (library routine)."""
    rng = np.random.default_rng(0)
    X = rng.normal(size=(40, 4))
    y = rng.normal(size=40)
    lo, hi = np.full(4, -1e9), np.full(4, 1e9)
    res = F.levenberg_marquardt(lambda p: X @ p - y, np.zeros(4), [1] * 4, lo, hi, h=0.1)
    ref = np.linalg.lstsq(X, y, rcond=None)[0]
    np.testing.assert_allclose(res.p, ref, rtol=1e-9, atol=1e-9)
    # parameter errors of a linear model: sqrt(diag((X^T X)^-1))
    np.testing.assert_allclose(res.errors, np.sqrt(np.diag(np.linalg.inv(X.T @ X))), rtol=1e-6)


def test_lm_box_constraint_active():
    """Minimum outside the box: the solution sits on the bound."""
    X = np.eye(2)
    y = np.array([3.0, -0.5])
    res = F.levenberg_marquardt(lambda p: X @ p - y, np.zeros(2), [1, 1],
                                np.array([-1.0, -1.0]), np.array([1.0, 1.0]))
    np.testing.assert_allclose(res.p, [1.0, -0.5], atol=1e-9)


def test_lm_rosenbrock():
    """Rosenbrock residuals (10 (y - x^2), 1 - x): minimum at (1, 1)."""
    res = F.levenberg_marquardt(lambda p: np.array([10 * (p[1] - p[0] ** 2), 1 - p[0]]),
                                np.array([-1.2, 1.0]), [1, 1], np.full(2, -10.0),
                                np.full(2, 10.0), h=1e-4, max_iter=500)
    np.testing.assert_allclose(res.p, [1.0, 1.0], atol=1e-5)


def test_lm_frozen_zero_column():
    """A free slot with no influence (like I0 on the velocity maps) is frozen."""
    X = np.array([[1.0, 0.0], [2.0, 0.0], [3.0, 0.0]])
    y = np.array([1.0, 2.0, 3.0])
    res = F.levenberg_marquardt(lambda p: X @ p - y, np.array([0.0, 5.0]), [1, 1],
                                np.full(2, -10.0), np.full(2, 10.0))
    np.testing.assert_allclose(res.p, [1.0, 5.0], atol=1e-9)
    assert res.errors[1] == 0.0


def test_lm_systemic_velocity_weighted_mean(O):
    """Only Vsys free, dispersion term off: m1 shifts rigidly with Vsys (lines
    well inside the band), so the optimum is the 1/E^2-weighted mean of
    v_obs - m1(Vsys = 0)."""
    d = O.Desc(16, 16, 96, 1, 10.0, crpix=47.5, psf_fwhm=2.0, lsf_sigma=15.0)
    truth = np.array([8.0, 7.5, 30.0, 50.0, 0.0, 120.0, 3.0, 25.0, 4.0, 1.0, 1.0, 1.0])
    base = O.evaluate(d, truth)
    rng = np.random.default_rng(4)
    obs = I.make_observation(base, 5.0, rng, W=0.0)
    obs.evel = (obs.evel * rng.uniform(0.5, 2.0, obs.evel.shape)).astype(np.float32)
    resid = F.model_residuals(d, obs)
    free = [0] * 12
    free[4] = 1
    lo, hi = np.full(12, -1e9), np.full(12, 1e9)
    res = F.levenberg_marquardt(resid, truth, free, lo, hi)
    mk = obs.mask.astype(bool)
    w = 1.0 / obs.evel.astype(np.float64)[mk] ** 2
    expect = np.sum(w * (obs.vel.astype(np.float64)[mk] - base[1][mk])) / np.sum(w)
    assert abs(res.p[4] - expect) < 1e-6
    assert abs(res.errors[4] - 1 / math.sqrt(np.sum(w))) < 1e-6


def test_nested_grid_quadratic_bowl():
    """A separable quadratic bowl: every level contains the minimum, so the
    final best node is within one final spacing of it; node 0 wins ties."""
    c = np.array([0.3, -1.7])
    f = lambda p: float(np.sum((p[:2] - c) ** 2 * np.array([1.0, 4.0])))
    r = F.nested_grid(f, [-5.0, -5.0], [5.0, 5.0], [1, 1], [0.0, 0.0], n=16, max_levels=4)
    assert np.all(np.abs(r.best - c) <= r.spacing + 1e-12) and r.n_evals == 4 * 256
    flat = F.nested_grid(lambda p: 1.0, [0.0], [1.0], [1], [0.0], n=5, max_levels=1)
    assert flat.best_index == 0 and flat.best[0] == 0.0


def test_nested_grid_accuracy_stop():
    r = F.nested_grid(lambda p: (p[0] - 0.25) ** 2, [0.0], [1.0], [1], [0.0], n=11,
                      max_levels=10, accuracy=[0.01])
    assert r.levels == 3 and r.spacing[0] < 0.01 and abs(r.best[0] - 0.25) <= r.spacing[0]


def test_nested_grid_per_slot_node_counts():
    """Per-slot node counts (the paper's grids of 7, 11, 11, 5, 5, 5 nodes,
    Sec. 4): the first level's nodes are exactly the mixed-radix product of
    the per-slot grids, enumerated by brute force here; on a quadratic bowl
    the search stops at the requested accuracy per slot with the bowl's
    minimum inside the last box."""
    import itertools
    lo, hi = [0.0, -1.0, 2.0], [6.0, 1.0, 4.0]
    n = [4, 3, 5]
    seen = []
    F.nested_grid(lambda p: seen.append(p.copy()) or 0.0, lo, hi, [1, 1, 1], [0.0, 0.0, 0.0],
                  n=n, max_levels=1)
    expect = [np.array(t) for t in itertools.product(np.linspace(0, 6, 4), np.linspace(-1, 1, 3),
                                                     np.linspace(2, 4, 5))]
    assert len(seen) == 60
    for a, b in zip(seen, expect):
        np.testing.assert_allclose(a, b, atol=1e-15)
    mu = np.array([2.3, 0.37, 3.11])
    f = lambda p: float(np.sum((p - mu) ** 2 * [1.0, 4.0, 9.0]))
    acc = [0.01, 0.1, 0.1]
    r = F.nested_grid(f, lo, hi, [1, 1, 1], [0.0, 0.0, 0.0], n=[7, 11, 5], max_levels=50,
                      accuracy=acc)
    assert all(r.spacing[k] < acc[k] for k in range(3))
    assert np.all(np.abs(r.best - mu) <= r.spacing)
    # an index on a tie goes to the lowest linear index (first slot slowest)
    r = F.nested_grid(lambda p: 0.0, lo, hi, [1, 1, 1], [0.0, 0.0, 0.0], n=n, max_levels=1)
    assert r.best_index == 0
