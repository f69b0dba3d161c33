"""FFT path of the spatial PSF convolution against the FP64 oracle (literal
direct convolution) and against the direct GPU path.

Bound: the radix-2 FFTs run in FP64, so a convolved plane value carries an
absolute error of order log2(P) * 1e-16 of the plane's largest value.  Maps
are held to the benchmark spec's tolerances where the oracle's flux is at least
1e-8 of its maximum (there that error is below 1e-7 relative); fainter
spaxels must be finite.
"""
import numpy as np
import pytest

from paper_1510_01815_amd import inputs as I
from parity import assert_chi2_close, assert_maps_close, oracle_desc
from test_gpu_eval import make_obs, oracle_chi2, oracle_maps, rows_for

pytestmark = pytest.mark.gpu
FFT_BRIGHT = 1e-8

GRIDS = {
    "c1_32x32x64": I.Grid(32, 32, 64, 30.0, psf_fwhm=2.5, lsf_sigma=30.0),
    "ragged_41x27x33": I.Grid(41, 27, 33, 25.0, psf_fwhm=3.3, lsf_sigma=20.0, rc=I.RC_EPINAT,
                              v0=10.0, crpix=13.3),
    "wide_psf_u2": I.Grid(30, 30, 64, 30.0, psf_fwhm=6.0, lsf_sigma=30.0, u=2),
    "u3_odd": I.Grid(11, 9, 13, 35.0, psf_fwhm=2.2, lsf_sigma=25.0, u=3),
    "very_wide_psf": I.Grid(40, 36, 32, 30.0, psf_fwhm=12.0, lsf_sigma=30.0),
    "no_psf": I.Grid(20, 18, 40, 20.0, psf_fwhm=0.0, lsf_sigma=15.0),
    "single_pixel": I.Grid(1, 1, 24, 30.0, psf_fwhm=2.5, lsf_sigma=30.0),
}


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_fft_maps_match_oracle(O, gbk, name):
    grid = GRIDS[name]
    rows = rows_for(grid, 5, 31 + len(name))
    m = gbk.Model.from_grid(grid, conv="fft")
    assert m.conv_path() == "fft"
    ref = oracle_maps(O, grid, rows)
    out = m.evaluate(rows).cpu().numpy()
    for b in range(len(rows)):
        assert_maps_close(out[b], ref[b], f"{name} row {b}", bright_frac=FFT_BRIGHT)


@pytest.mark.parametrize("name", ["c1_32x32x64", "ragged_41x27x33", "wide_psf_u2"])
def test_fft_equals_direct_path(gbk, name):
    grid = GRIDS[name]
    rows = rows_for(grid, 16, 5)
    a = gbk.Model.from_grid(grid, conv="direct")
    f = gbk.Model.from_grid(grid, conv="fft")
    assert a.conv_path() == "direct" and f.conv_path() == "fft"
    ma, mf = a.evaluate(rows).cpu().numpy(), f.evaluate(rows).cpu().numpy()
    for b in range(len(rows)):
        assert_maps_close(mf[b], ma[b].astype(np.float64), f"{name} row {b}", bright_frac=FFT_BRIGHT)


@pytest.mark.parametrize("name,W,rmask", [("c1_32x32x64", 1.0, 0.0), ("wide_psf_u2", 0.2, 0.1),
                                          ("very_wide_psf", 1.0, 0.1)])
def test_fft_chi2_and_residuals_match_oracle(O, gbk, name, W, rmask):
    grid = GRIDS[name]
    rows = rows_for(grid, 6, 17)
    obs = make_obs(O, grid, rows[0], 9, random_mask=rmask, W=W)
    d = oracle_desc(O, grid.as_dict())
    # parity region of this path: drop the spaxels fainter than its bound
    m0 = O.evaluate(d, rows[0])[0]
    obs.mask = (obs.mask.astype(bool) & (m0 >= FFT_BRIGHT * m0.max())).astype(np.uint8)
    m = gbk.Model.from_grid(grid, conv="fft")
    m.set_obs(obs)
    c, n = m.chi2(rows)
    c, n = c.cpu().numpy(), n.cpu().numpy()
    rc, rn = oracle_chi2(O, grid, rows, obs)
    np.testing.assert_array_equal(n, rn)
    for b in range(len(rows)):
        assert_chi2_close(c[b], rc[b], rn[b], f"{name} row {b}", obs=obs)
    r = m.residuals(rows[:2]).cpu().numpy()
    assert np.isfinite(r[:, :, obs.mask.astype(bool)]).all()


def test_auto_takes_fft_for_psf_beyond_the_direct_kernels(gbk):
    narrow = gbk.Model.from_grid(GRIDS["c1_32x32x64"])
    wide = gbk.Model.from_grid(GRIDS["very_wide_psf"])   # half-width 21 > 16
    assert narrow.conv_path() == "direct" and wide.conv_path() == "fft"


def test_fft_out_of_domain_rows_are_nan(O, gbk):
    grid = GRIDS["c1_32x32x64"]
    rows = rows_for(grid, 3, 2)
    rows[1, I.INC] = 95.0
    m = gbk.Model.from_grid(grid, conv="fft")
    out = m.evaluate(rows).cpu().numpy()
    assert np.isnan(out[1]).all() and np.isfinite(out[[0, 2]]).all()
