"""Ragged multi-model batches (gk_survey_*) against the single-model path
and the oracle: same kernels, so results must be bit-identical."""
import numpy as np
import pytest

from paper_1510_01815_amd import inputs as I
from parity import assert_chi2_close, oracle_desc

pytestmark = pytest.mark.gpu


def survey_models(O, gbk, n, seed, with_u2=True):
    rng = np.random.default_rng(seed)
    grids, truths, models, obs = [], [], [], []
    for k in range(n):
        side = int(rng.integers(12, 72))
        nz = int(rng.integers(20, 80))
        fw = float(rng.uniform(1.5, 4.0))
        u = 2 if (with_u2 and k % 7 == 3) else 1
        g = I.Grid(side, side, nz, 30.0, psf_fwhm=fw, lsf_sigma=30.0, u=u,
                   rc=[I.RC_ARCTAN, I.RC_BOISSIER, I.RC_EPINAT][k % 3])
        t = I.c1_box_draw(rng, 1, side, fw)[0]
        d = oracle_desc(O, g.as_dict())
        ob = I.make_observation(O.evaluate(d, t), float(rng.uniform(3, 15)), rng,
                                random_mask=0.1)
        m = gbk.Model.from_grid(g)
        m.set_obs(ob)
        grids.append(g); truths.append(t); models.append(m); obs.append(ob)
    return grids, truths, models, obs


def test_survey_chi2_bit_identical_to_single_model(O, gbk):
    import torch
    grids, truths, models, obs = survey_models(O, gbk, 14, 1)
    sv = gbk.Survey(models)
    rng = np.random.default_rng(2)
    B = 300
    midx = rng.integers(0, len(models), B)
    rows = np.stack([truths[i] for i in midx])
    rows[:, I.PA] += rng.normal(0, 5, B)
    rows[:, I.VT] *= rng.uniform(0.9, 1.1, B)
    rows[17, I.INC] = 95.0  # out of domain
    c = sv.chi2(midx, rows).cpu().numpy()
    c_dev = sv.chi2(midx, torch.tensor(rows, device="cuda")).cpu().numpy()
    np.testing.assert_array_equal(c, c_dev)
    for i in range(len(models)):
        sel = np.where(midx == i)[0]
        if len(sel) == 0:
            continue
        ref, _ = models[i].chi2(rows[sel])
        np.testing.assert_array_equal(c[sel], ref.cpu().numpy())
    assert np.isinf(c[17])
    # a few rows against the oracle
    for b in (0, 50, 299):
        g, ob = grids[midx[b]], obs[midx[b]]
        v, n = O.eval_chi2(oracle_desc(O, g.as_dict()), rows[b], ob.vel, ob.sig, ob.evel,
                           ob.esig, ob.mask, ob.W)
        assert_chi2_close(c[b], v, n, f"row {b}", obs=ob)


def test_survey_lm_equals_per_galaxy_lm(O, gbk):
    """All galaxies fitted at once reach exactly the parameters of fitting
    each galaxy alone (same step rule, same reductions)."""
    grids, truths, models, obs = survey_models(O, gbk, 8, 3, with_u2=False)
    rng = np.random.default_rng(4)
    free = [1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0]
    starts, lo, hi = [], [], []
    for t, g in zip(truths, grids):
        s = t.copy()
        s[:8] *= 1 + rng.uniform(-0.05, 0.05, 8)
        s[I.VSYS] = rng.uniform(-3, 3)
        starts.append(s)
        lo.append(np.array([0.3 * g.nx, 0.3 * g.ny, -720, 3, -50, 10, 0.2, 5, 0.5, 0.1, 0.1, 0.1]))
        hi.append(np.array([0.7 * g.nx, 0.7 * g.ny, 720, 87, 50, 500, 20, 200, 30, 10, 5, 5]))
    sv = gbk.Survey(models)
    r = sv.fit_lm(np.stack(starts), free, np.stack(lo), np.stack(hi), max_iter=60)
    for k, m in enumerate(models):
        one = m.fit_lm(starts[k], free, lo[k], hi[k], max_iter=60)
        np.testing.assert_array_equal(r["p"][k], one["p"])
        assert r["chi2"][k] == one["chi2"] and r["iterations"][k] == one["iterations"]


def test_survey_retiles_64x32_models(O, gbk):
    """A u = 1 model forced to the 64 x 32 register-blocked tile (which the
    survey kernels do not run) takes the 32 x 32 tile inside a survey: its
    survey chi2 equals, bit for bit, the single-model chi2 with the 32 x 32
    tile, agrees with the 64 x 32 single-model chi2 to summation rounding,
    and matches the oracle."""
    import torch
    g = I.Grid(96, 80, 40, 30.0, psf_fwhm=2.5, lsf_sigma=30.0)
    rng = np.random.default_rng(12)
    truth = I.c1_box_draw(rng, 1, 80, 2.5)[0]
    truth[I.XO], truth[I.YO] = 47.5, 40.2
    d = oracle_desc(O, g.as_dict())
    ob = I.make_observation(O.evaluate(d, truth), 5.0, rng, random_mask=0.1)
    m = gbk.Model.from_grid(g)
    m.set_obs(ob)
    m.set_conv_config("direct", 64, 32)
    other = gbk.Model.from_grid(I.Grid(40, 40, 32, 30.0, psf_fwhm=2.0, lsf_sigma=30.0))
    ob2 = I.make_observation(O.evaluate(oracle_desc(O, I.Grid(40, 40, 32, 30.0, psf_fwhm=2.0,
                                                                lsf_sigma=30.0).as_dict()),
                                        np.array([20.0, 19.5, 30, 50, 0, 180, 3, 40, 5, 1, 1, 1.0])),
                             5.0, rng)
    other.set_obs(ob2)
    sv = gbk.Survey([m, other])
    rows = np.stack([truth] * 6)
    rows[:, I.PA] += np.linspace(-10, 10, 6)
    midx = np.array([0, 0, 1, 0, 0, 0])
    rows[2] = np.array([20.0, 19.5, 35, 55, 2, 170, 3, 40, 5, 1, 1, 1.0])
    c = sv.chi2(midx, rows).cpu().numpy()
    sel = np.where(midx == 0)[0]
    wide, _ = m.chi2(rows[sel])
    wide = wide.cpu().numpy()
    m.set_conv_config("direct", 32, 32)
    sv32 = gbk.Survey([m, other])
    c32 = sv32.chi2(midx, rows).cpu().numpy()
    single32, _ = m.chi2(rows[sel])
    np.testing.assert_array_equal(c[sel], single32.cpu().numpy())
    np.testing.assert_array_equal(c, c32)
    np.testing.assert_allclose(c[sel], wide, rtol=1e-12)
    for b in sel[:2]:
        v, n = O.eval_chi2(d, rows[b], ob.vel, ob.sig, ob.evel, ob.esig, ob.mask, ob.W)
        assert_chi2_close(c[b], v, n, f"row {b}", obs=ob)
