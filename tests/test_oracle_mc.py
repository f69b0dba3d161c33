"""Pins of the oracle's Monte-Carlo parameter errors (Bekiaris et al. 2016,
Sec. 4.2 shuffled residuals, Sec. 4.3 perturbations by the error maps).

The simulated observations are pinned by what they must preserve (identity
permutation and zero noise give the observation back; a shuffle re-deals the
very residuals of the best fit), and the refits by the closed form of a
problem whose only free parameter enters linearly: with only V_sys free the
least-squares V_sys of a velocity field is the best one plus the
1/E_v^2-weighted mean of (simulated - best-fit) velocities.
"""
import numpy as np
import pytest

from oracle import fitters as F
from paper_1510_01815_amd import inputs as I


@pytest.fixture(scope="module")
def case(O):
    grid = I.Grid(23, 19, 1, 1.0, 0.0, 0.0, rc=I.RC_EPINAT, strategy=1)
    d = O.Desc(grid.nx, grid.ny, 1, rc=grid.rc)
    truth = I.ghasp_draw(I.rng_for(90, 0, 0), 1, 20)[0]
    truth[[I.XO, I.YO]] = 11.3, 9.1
    maps = O.vfield(d, truth)
    obs = I.make_observation(maps, 5.0, I.rng_for(90, 0, 1), flux_frac=I.GHASP_FLUX_FRAC,
                             random_mask=0.2, W=0.0)
    # uneven errors, so that a shuffle moves the weighted mean
    obs.evel = (obs.evel * (1.0 + I.rng_for(90, 0, 2).random(obs.evel.shape))).astype(np.float32)
    return d, truth, maps, obs


def test_identity_shuffle_and_zero_noise_give_the_observation(case):
    d, truth, maps, obs = case
    nv = int(obs.mask.sum())
    sims = F.mc_simulations(maps, obs, "shuffle", perm=[np.arange(nv)])
    np.testing.assert_array_equal(sims[0].vel, obs.vel)
    np.testing.assert_array_equal(sims[0].sig, obs.sig)
    sims = F.mc_simulations(maps, obs, "perturb", noise=np.zeros((1, 2) + obs.vel.shape))
    np.testing.assert_array_equal(sims[0].vel, obs.vel)


def test_shuffle_redeals_the_best_fit_residuals(case):
    d, truth, maps, obs = case
    mk = obs.mask.astype(bool)
    nv = int(mk.sum())
    perm = I.mc_permutations(I.rng_for(90, 1, 0), 3, nv)
    sims = F.mc_simulations(maps, obs, "shuffle", perm=perm)
    res = (obs.vel.astype(np.float64) - maps[1])[mk]
    for s, sim in enumerate(sims):
        new = (sim.vel.astype(np.float64) - maps[1])[mk]
        # pixel k carries residual perm[s][k]; float32 storage of the sum only
        np.testing.assert_allclose(new, res[perm[s]], rtol=0, atol=1e-3)
        np.testing.assert_array_equal(sim.vel[~mk], obs.vel[~mk])
        assert not np.array_equal(new, res)


def test_perturbation_is_error_times_draw(case):
    d, truth, maps, obs = case
    mk = obs.mask.astype(bool)
    noise = I.mc_normals(I.rng_for(90, 2, 0), 2, *obs.vel.shape)
    sims = F.mc_simulations(maps, obs, "perturb", noise=noise)
    for s, sim in enumerate(sims):
        dv = sim.vel.astype(np.float64) - obs.vel
        np.testing.assert_allclose(dv[mk], (obs.evel * noise[s, 0])[mk], rtol=0, atol=1e-3)
        assert (dv[~mk] == 0).all()
        np.testing.assert_array_equal(sim.sig, obs.sig)  # W = 0: dispersion untouched


@pytest.mark.parametrize("mode", ["shuffle", "perturb"])
def test_vsys_only_refits_are_weighted_means(O, case, mode):
    d, truth, maps, obs = case
    mk = obs.mask.astype(bool)
    nv = int(mk.sum())
    free = np.zeros(12, dtype=np.uint8)
    free[I.VSYS] = 1
    lo = np.full(12, -1e9)
    hi = np.full(12, 1e9)
    perm = I.mc_permutations(I.rng_for(90, 3, 0), 6, nv) if mode == "shuffle" else None
    noise = I.mc_normals(I.rng_for(90, 3, 1), 6, *obs.vel.shape) if mode == "perturb" else None
    fits, sd = F.mc_errors(lambda o: F.vfield_residuals(d, o), truth, maps, obs, free, lo, hi,
                           mode, perm=perm, noise=noise)
    sims = F.mc_simulations(maps, obs, mode, perm, noise)
    w = 1.0 / obs.evel.astype(np.float64)[mk] ** 2
    expect = np.array([truth[I.VSYS] + np.sum(w * (s.vel.astype(np.float64)[mk] - maps[1][mk]))
                       / np.sum(w) for s in sims])
    np.testing.assert_allclose(fits[:, I.VSYS], expect, rtol=0, atol=1e-7)
    other = np.delete(np.arange(12), I.VSYS)
    np.testing.assert_array_equal(fits[:, other], np.tile(truth[other], (6, 1)))
    assert abs(sd[I.VSYS] - np.std(expect, ddof=1)) <= 1e-7
    assert (sd[other] == 0).all()
