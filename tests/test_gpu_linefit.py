"""GPU parity of Gaussian line fitting (gk_fit_lines; the alternative to
moments of Bekiaris et al. 2016, Sec. 2.2.5 and 5.2) against the oracle's
per-spectrum LM, through the C ABI.

Cubes: the oracle's convolved, down-sampled model cube plus seeded noise (a
ragged number of spectra), noise-free Gaussian lines, a 128 x 128 x 48 cube
stacked 16 times (sampled spectra), spectra longer than the 64 channels
staged in LDS, and the degenerate cases (empty spectra, a single channel, a
single spectrum).
"""
import math

import numpy as np
import pytest

from oracle import fitters as F
from paper_1510_01815_amd import inputs as I
from parity import oracle_desc

pytestmark = pytest.mark.gpu


def velocities(nz, v0, dv, crpix):
    return v0 + (np.arange(nz) - crpix) * dv


def oracle_cube(O, grid, p):
    """Convolved, down-sampled model cube [nz][ny][nx] of the oracle."""
    d = oracle_desc(O, grid.as_dict())
    nxe, nye, nze, hp, hl = O.cube_dims(d)
    kp = O.kernel_taps(grid.u * grid.psf_fwhm / I.FWHM_PER_SIGMA if grid.psf_fwhm > 0 else 0.0)
    kl = O.kernel_taps(grid.u * grid.lsf_sigma / grid.dv if grid.lsf_sigma > 0 else 0.0)
    c = O.convolve3(O.model_cube(d, p), kl, kp, kp)
    return O.downsample(c, grid.u)


def line_errors(spec, v, amp, vel, disp):
    """1-sigma errors of a converged fit from its curvature (for tolerances)."""
    t = (v - vel) / disp
    e = np.exp(-0.5 * t * t)
    J = np.stack([e, amp * e * t / disp, amp * e * t * t / disp], axis=1)
    r = amp * e - spec
    dof = max(len(v) - 3, 1)
    return np.sqrt(np.diag(np.linalg.inv(J.T @ J)) * max(r @ r / dof, 1e-30))


def check_against_oracle(gmaps, gst, cube, v, dv, picks):
    nz = cube.shape[0]
    flat = cube.reshape(nz, -1)
    gm = gmaps.reshape(3, -1)
    gs = gst.reshape(-1)
    agree = 0
    for p in picks:
        f = F.fit_gaussian_line(flat[:, p], v, dv)
        if f.status == 0:
            assert gs[p] == 0 and gm[0, p] == 0 and math.isnan(gm[1, p]) and math.isnan(gm[2, p])
            agree += 1
            continue
        agree += gs[p] == f.status
        # converged (1) or stopped at the damping limit (2, the step no longer
        # lowers chi2 at ftol = xtol = 1e-12): both at the optimum, so the
        # parameters are compared whichever of the two each side reports;
        # fits stopped by the iteration cap (3) are not at an optimum
        if f.status not in (1, 2) or gs[p] not in (1, 2):
            continue
        err = line_errors(flat[:, p].astype(np.float64), v, f.amp, f.vel, f.disp)
        for k, (got, want) in enumerate(((gm[1, p], f.vel), (gm[2, p], f.disp))):
            assert abs(got - want) <= 1e-3 * err[k + 1] + 2e-6 * abs(want), (p, k, got, want, err)
        flux = f.amp * f.disp * math.sqrt(2.0 * math.pi)
        assert abs(gm[0, p] - flux) <= 1e-5 * abs(flux) + 1e-3 * err[0] * f.disp * 2.5066, (p, gm[0, p], flux)
    assert agree >= 0.98 * len(picks), (agree, len(picks))


def test_line_fit_matches_oracle_on_a_model_cube(O, gbk):
    import torch
    grid = I.Grid(23, 19, 40, 25.0, psf_fwhm=2.2, lsf_sigma=20.0)
    p = np.array([11.2, 9.4, 35.0, 55.0, 10.0, 170.0, 3.0, 40.0, 4.0, 1.0, 1.0, 1.0])
    cube = oracle_cube(O, grid, p)
    rng = I.rng_for(97, 0, 0)
    cube = (cube + 0.002 * cube.max() * rng.standard_normal(cube.shape)).astype(np.float32)
    crpix = grid.nz / 2.0
    v = velocities(grid.nz, 0.0, grid.dv, crpix)
    maps, st, it = gbk.fit_lines(torch.tensor(cube, device="cuda"), 0.0, grid.dv, crpix)
    gm, gs = maps.cpu().numpy(), st.cpu().numpy()
    assert (gs == 1).mean() > 0.9
    check_against_oracle(gm, gs, cube, v, grid.dv, range(grid.nx * grid.ny))


def test_noise_free_lines_are_recovered(gbk):
    import torch
    nz, dv, crpix = 48, 16.0, 23.5
    v = velocities(nz, 5.0, dv, crpix)
    rng = I.rng_for(97, 1, 0)
    n = 1000  # ragged: not a multiple of 256
    amp = rng.uniform(0.5, 3.0, n)
    mu = rng.uniform(-150.0, 150.0, n)
    sig = rng.uniform(15.0, 60.0, n)
    cube = (amp * np.exp(-0.5 * ((v[:, None] - mu) / sig) ** 2)).astype(np.float32)
    maps, st, it = gbk.fit_lines(torch.tensor(cube, device="cuda"), 5.0, dv, crpix)
    gm, gs = maps.cpu().numpy(), st.cpu().numpy()
    # float32 data: the fit ends on its rounding floor, where no trial lowers
    # chi2 any more and the damping limit stops it (status 2) as often as ftol
    assert np.isin(gs, [1, 2]).all()
    np.testing.assert_allclose(gm[1], mu, rtol=0, atol=2e-3)
    np.testing.assert_allclose(gm[2], sig, rtol=1e-4, atol=0)
    np.testing.assert_allclose(gm[0], amp * sig * math.sqrt(2 * math.pi), rtol=1e-4)


def test_degenerate_spectra(gbk):
    import torch
    nz, dv = 30, 20.0
    v = velocities(nz, 0.0, dv, 15.0)
    cube = np.zeros((nz, 5), dtype=np.float32)
    cube[:, 1] = -1.0                                   # negative only: no line
    cube[12, 2] = 4.0                                   # one channel: zero width, no line
    cube[:, 3] = np.exp(-0.5 * ((v - 30.0) / 40.0) ** 2)
    cube[:, 4] = 2.0 * np.exp(-0.5 * ((v + 90.0) / 25.0) ** 2)
    maps, st, it = gbk.fit_lines(torch.tensor(cube, device="cuda"), 0.0, dv, 15.0)
    gm, gs, gi = maps.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()
    assert list(gs[:3]) == [0, 0, 0] and (gi[:3] == 0).all()
    assert (gm[0, :3] == 0).all() and np.isnan(gm[1:, :3]).all()
    assert gs[3] == 1 and abs(gm[1, 3] - 30.0) < 1e-3 and abs(gm[2, 3] - 40.0) < 1e-3
    assert gs[4] == 1 and abs(gm[1, 4] + 90.0) < 1e-3 and abs(gm[2, 4] - 25.0) < 1e-3
    # one channel per spectrum: the moments have no width
    one = torch.ones((1, 7), dtype=torch.float32, device="cuda")
    maps, st, it = gbk.fit_lines(one, 0.0, dv, 0.0)
    assert (st.cpu().numpy() == 0).all()
    # a single spectrum
    maps, st, it = gbk.fit_lines(torch.tensor(cube[:, 4:5].copy(), device="cuda"), 0.0, dv, 15.0)
    assert st.cpu().numpy()[0] == 1


def test_line_fit_large_stack_sampled(O, gbk):
    """A noisy 128 x 128 x 48 model cube stacked 16 times (262,144 spectra):
    every spectrum fitted on the GPU; sampled spectra against the oracle."""
    import torch
    grid = I.Grid(128, 128, 48, 16.0, psf_fwhm=3.0, lsf_sigma=I.C2_LSF_SIGMA, rc=I.RC_BOISSIER)
    p = I.c2_draw(I.rng_for(2, 0, 0), 1)[0]
    base = oracle_cube(O, grid, p)
    rng = I.rng_for(97, 2, 0)
    cube = np.concatenate([base + 0.003 * base.max() * rng.standard_normal(base.shape)
                           for _ in range(16)], axis=1).astype(np.float32)  # [48][16*128][128]
    crpix = grid.nz / 2.0
    maps, st, it = gbk.fit_lines(torch.tensor(cube, device="cuda"), 0.0, grid.dv, crpix)
    gm, gs = maps.cpu().numpy(), st.cpu().numpy()
    assert gm.shape == (3, 16 * 128, 128)
    assert np.isin(gs, [0, 1, 2, 3]).all() and (gs == 1).mean() > 0.5
    picks = I.rng_for(97, 2, 1).choice(cube.shape[1] * cube.shape[2], 200, replace=False)
    check_against_oracle(gm, gs, cube, velocities(grid.nz, 0.0, grid.dv, crpix), grid.dv, picks)


def test_line_fit_refuses_bad_arguments(gbk):
    import torch
    cube = torch.ones((10, 4), dtype=torch.float32, device="cuda")
    for args in ((0.0, 0.0, 5.0), (0.0, -1.0, 5.0), (math.nan, 10.0, 5.0)):
        with pytest.raises(gbk.GkError) as e:
            gbk.fit_lines(cube, *args)
        assert e.value.status == gbk.GK_EINVAL
    with pytest.raises(gbk.GkError):
        gbk.fit_lines(cube, 0.0, 10.0, 5.0, max_iter=0)


def test_long_spectra_read_from_the_cube(gbk):
    """More than 64 channels: the spectra are read from the cube at every pass
    instead of being staged in LDS; noisy lines against the oracle."""
    import torch
    nz, dv, crpix = 96, 10.0, 47.5
    v = velocities(nz, 0.0, dv, crpix)
    rng = I.rng_for(97, 3, 0)
    n = 300
    amp = rng.uniform(0.5, 3.0, n)
    mu = rng.uniform(-250.0, 250.0, n)
    sig = rng.uniform(15.0, 80.0, n)
    cube = (amp * np.exp(-0.5 * ((v[:, None] - mu) / sig) ** 2)
            + 0.05 * rng.standard_normal((nz, n))).astype(np.float32)
    maps, st, it = gbk.fit_lines(torch.tensor(cube, device="cuda"), 0.0, dv, crpix)
    check_against_oracle(maps.cpu().numpy(), st.cpu().numpy(), cube, v, dv, range(n))
