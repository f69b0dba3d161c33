"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one step of the evaluation (Bekiaris et al. 2016, Sec. 2.1 and
2.2) to a closed form, a library routine, a brute-force computation, a
hand-computed fixture or an exact invariant, chosen so that a dropped term, a
wrong sign, a wrong index or a transposed operand anywhere in the oracle fails
at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import signal, stats

P = dict(xo=0, yo=1, pa=2, inc=3, vsys=4, vt=5, rt=6, sig=7, r0=8, i0=9, a=10, g=11)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def par(xo=16.0, yo=16.0, pa=0.0, inc=45.0, vsys=0.0, vt=200.0, rt=4.0, sig=40.0, r0=6.0,
        i0=1.0, a=1.0, g=1.0):
    return np.array([xo, yo, pa, inc, vsys, vt, rt, sig, r0, i0, a, g], dtype=np.float64)


# ---------------------------------------------------------------------------
# Independent restatements used as expected values
# ---------------------------------------------------------------------------

def vrot_textbook(rc, r, p):
    """Rotation curves written from their published definitions: arctan
    (Courteau 1997; eq. 6), Epinat et al. 2008 (eq. 7), and the exponential
    rise Vt (1 - exp(-r/rt))."""
    vt, rt = p[P["vt"]], p[P["rt"]]
    if rc == 0:
        return vt * math.atan2(r, rt) / (math.pi / 2)
    if rc == 1:
        return vt * (r / rt) ** p[P["g"]] / (1 + (r / rt) ** p[P["a"]])
    return vt * (-math.expm1(-r / rt))


def projected_velocity(rc, p, x, y):
    """Line-of-sight velocity of a thin rotating disc in polar form.

    A sky point at projected distance d and projected angle phi from the
    receding major axis lies on the disc circle of radius
    r = d sqrt(cos^2 phi + sin^2 phi / cos^2 i) at disc azimuth theta with
    cos(theta) = d cos(phi) / r, so v = Vsys + V(r) sin(i) cos(theta).
    The receding major axis points along +y for PA = 0 and turns towards -x
    as PA grows (PA measured from +y through -x).
    """
    pa, inc = math.radians(p[P["pa"]]), math.radians(p[P["inc"]])
    dx, dy = x - p[P["xo"]], y - p[P["yo"]]
    d = math.hypot(dx, dy)
    if d == 0:
        return p[P["vsys"]]
    ang_point = math.atan2(dy, dx)
    ang_axis = math.atan2(math.cos(pa), -math.sin(pa))
    phi = ang_point - ang_axis
    r = d * math.sqrt(math.cos(phi) ** 2 + math.sin(phi) ** 2 / math.cos(inc) ** 2)
    return p[P["vsys"]] + vrot_textbook(rc, r, p) * math.sin(inc) * d * math.cos(phi) / r


def deprojected_radius(p, x, y):
    pa, inc = math.radians(p[P["pa"]]), math.radians(p[P["inc"]])
    dx, dy = x - p[P["xo"]], y - p[P["yo"]]
    d = math.hypot(dx, dy)
    if d == 0:
        return 0.0
    phi = math.atan2(dy, dx) - math.atan2(math.cos(pa), -math.sin(pa))
    return d * math.sqrt(math.cos(phi) ** 2 + math.sin(phi) ** 2 / math.cos(inc) ** 2)


def clean_desc(O, rc=0, nx=33, ny=33, nz=128, dv=10.0, u=1, **kw):
    """No PSF, no LSF, a wide band: moments of the cube reduce to closed forms."""
    return O.Desc(nx, ny, nz, u, dv, v0=0.0, crpix=(nz - 1) / 2.0, psf_fwhm=0.0,
                  lsf_sigma=0.0, rc=rc, **kw)


# ---------------------------------------------------------------------------
# Kernel taps (eq. 9, one axis)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [0.5, 1.0, 1.0617, 1.274, 2.5, 3.3])
def test_taps_match_normal_pdf(O, sigma):
    t = O.kernel_taps(sigma, 4.0)
    h = math.ceil(4.0 * sigma)
    assert len(t) == 2 * h + 1
    ref = stats.norm.pdf(np.arange(-h, h + 1), scale=sigma)
    ref /= ref.sum()
    np.testing.assert_allclose(t, ref, rtol=1e-13, atol=0)
    assert abs(t.sum() - 1) < 1e-14


def test_taps_off(O):
    np.testing.assert_array_equal(O.kernel_taps(0.0), [1.0])


def test_cube_dims_halo(O):
    # FWHM 2.5 px -> sigma 1.0617 -> 11 taps; LSF 30 km/s at 30 km/s channels -> 9 taps
    d = O.Desc(32, 32, 64, 1, 30.0, psf_fwhm=2.5, lsf_sigma=30.0)
    assert O.cube_dims(d) == (42, 42, 72, 5, 4)
    d = O.Desc(32, 32, 64, 2, 30.0, psf_fwhm=2.5, lsf_sigma=30.0)
    assert O.cube_dims(d) == (64 + 18, 64 + 18, 128 + 16, 9, 8)


# ---------------------------------------------------------------------------
# Rotation curves at special radii (eqs. 6, 7)
# ---------------------------------------------------------------------------

def test_rotation_curves_special_values(O):
    p = par(vt=180.0, rt=5.0, a=1.0, g=1.0)
    assert abs(O.vrot(0, 5.0, p) - 90.0) < 1e-12                    # atan(1) = pi/4
    assert abs(O.vrot(1, 5.0, p) - 90.0) < 1e-12                    # a = g: half of Vt
    assert abs(O.vrot(2, 5.0, p) - 180.0 * (1 - math.exp(-1))) < 1e-12
    p2 = par(vt=180.0, rt=5.0, a=1.0, g=2.0)
    assert abs(O.vrot(1, 10.0, p2) - 180.0 * 4 / 3) < 1e-12        # (2)^2 / (1 + 2)
    for rc in (0, 1, 2):
        assert O.vrot(rc, 0.0, p) == 0.0
        assert abs(O.vrot(rc, 1e9, p) - 180.0) < 1e-5 * 180


# ---------------------------------------------------------------------------
# Pin (a): closed-form velocity field with no PSF
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rc,pa,inc", [(0, 0.0, 45.0), (0, 60.0, 30.0), (1, 137.0, 70.0),
                                       (2, 251.0, 55.0), (0, -20.0, 10.0)])
def test_velocity_field_closed_form(O, rc, pa, inc):
    p = par(pa=pa, inc=inc, vsys=13.0, vt=150.0, rt=3.0, sig=20.0, r0=8.0,
            a=1.4 if rc == 1 else 1.0, g=0.8 if rc == 1 else 1.0, xo=16.3, yo=15.6)
    d = clean_desc(O, rc=rc)
    m = O.evaluate(d, p)
    err = 0.0
    for y in range(d.ny):
        for x in range(d.nx):
            err = max(err, abs(m[1, y, x] - projected_velocity(rc, p, x, y)))
    assert err < 1e-6


def test_velocity_field_directions(O):
    """PA = 0: receding side on +y, approaching on -y, systemic on the minor
    axis (+/- x).  PA = 90: receding side on -x."""
    d = clean_desc(O)
    p = par(pa=0.0, inc=30.0, vsys=5.0, vt=100.0, rt=4.0, sig=20.0)
    m1 = O.evaluate(d, p)[1]
    s = math.sin(math.radians(30.0))
    assert abs(m1[20, 16] - (5.0 + 50.0 * s)) < 1e-6      # r = rt on the receding axis
    assert abs(m1[12, 16] - (5.0 - 50.0 * s)) < 1e-6
    assert abs(m1[16, 20] - 5.0) < 1e-6 and abs(m1[16, 12] - 5.0) < 1e-6
    p[P["pa"]] = 90.0
    m1 = O.evaluate(d, p)[1]
    assert abs(m1[16, 12] - (5.0 + 50.0 * s)) < 1e-6
    assert abs(m1[16, 20] - (5.0 - 50.0 * s)) < 1e-6
    assert abs(m1[20, 16] - 5.0) < 1e-6


# ---------------------------------------------------------------------------
# Surface brightness and line normalisation through m0 (eq. 5)
# ---------------------------------------------------------------------------

def test_m0_is_surface_brightness(O):
    d = clean_desc(O)
    p = par(pa=30.0, inc=50.0, vt=120.0, sig=20.0, r0=6.0, i0=2.5)
    m0 = O.evaluate(d, p)[0]
    for (y, x) in [(16, 16), (3, 7), (25, 30), (16, 5)]:
        r = deprojected_radius(p, x, y)
        assert abs(m0[y, x] - 2.5 * math.exp(-r / 6.0)) < 1e-12 * 2.5
    # one scale length along the major axis (PA = 0, axis along +y)
    p = par(pa=0.0, inc=50.0, sig=20.0, r0=6.0, i0=2.5)
    m0 = O.evaluate(d, p)[0]
    assert abs(m0[22, 16] - 2.5 / math.e) < 1e-12


def test_surface_brightness_floor(O):
    d = clean_desc(O)
    p = par(r0=0.2, sig=20.0, inc=40.0)
    m0 = O.evaluate(d, p)[0]
    # the corner lies beyond 60 scale lengths: brightness held at I0 exp(-60)
    assert deprojected_radius(p, 0, 0) / 0.2 > 60
    assert abs(m0[0, 0] / math.exp(-60.0) - 1) < 1e-9


def test_upsampled_subpixels(O):
    """u = 2: data pixel i covers fine pixels at i -/+ 1/4; m0 is the mean of
    the four sub-pixel brightnesses and m1 their brightness-weighted mean velocity."""
    d = clean_desc(O, u=2, nx=17, ny=15, nz=96)
    p = par(xo=8.2, yo=7.1, pa=40.0, inc=60.0, vt=160.0, rt=2.0, sig=20.0, r0=3.0)
    m = O.evaluate(d, p)
    for (y, x) in [(7, 8), (3, 2), (11, 14), (7, 9)]:
        pts = [(x + sx, y + sy) for sx in (-0.25, 0.25) for sy in (-0.25, 0.25)]
        inten = [math.exp(-deprojected_radius(p, a, b) / 3.0) for a, b in pts]
        vel = [projected_velocity(0, p, a, b) for a, b in pts]
        assert abs(m[0, y, x] - np.mean(inten)) < 1e-12
        assert abs(m[1, y, x] - np.dot(inten, vel) / np.sum(inten)) < 1e-6


# ---------------------------------------------------------------------------
# Pin (c): LSF -- variances of discrete distributions add under convolution
# ---------------------------------------------------------------------------

def test_lsf_variance_addition(O):
    dv, sig, lsf = 10.0, 20.0, 25.0
    d = O.Desc(33, 33, 128, 1, dv, v0=0.0, crpix=63.5, psf_fwhm=0.0, lsf_sigma=lsf)
    p = par(pa=75.0, inc=40.0, vt=150.0, rt=3.0, sig=sig)
    m = O.evaluate(d, p)
    s_ch = lsf / dv
    h = math.ceil(4 * s_ch)
    taps = stats.norm.pdf(np.arange(-h, h + 1), scale=s_ch)
    taps /= taps.sum()
    var_kernel = dv * dv * np.sum(taps * np.arange(-h, h + 1) ** 2)
    expect = math.sqrt(sig * sig + var_kernel)
    np.testing.assert_allclose(m[2], expect, rtol=1e-10, atol=0)
    # and the truncated kernel is within the R = 4 truncation deficit of sigma_LSF
    assert abs(expect - math.sqrt(sig ** 2 + lsf ** 2)) / expect < 2e-3
    # symmetric taps leave the first moment on the closed form
    err = max(abs(m[1, y, x] - projected_velocity(0, p, x, y))
              for y in range(33) for x in range(33))
    assert err < 1e-6


# ---------------------------------------------------------------------------
# Pin (b): PSF conserves flux; impulse response is the kernel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("u", [1, 2])
def test_psf_flux_conservation(O, u):
    base = dict(nx=80, ny=80, nz=64, dv=20.0, u=u)
    p = par(xo=40.0, yo=40.0, pa=20.0, inc=35.0, vt=100.0, rt=2.0, sig=30.0, r0=1.0)
    d0 = O.Desc(base["nx"], base["ny"], base["nz"], u, base["dv"], crpix=31.5, psf_fwhm=0.0,
                lsf_sigma=15.0)
    d1 = O.Desc(base["nx"], base["ny"], base["nz"], u, base["dv"], crpix=31.5, psf_fwhm=3.0,
                lsf_sigma=15.0)
    a, b = O.evaluate(d0, p)[0], O.evaluate(d1, p)[0]
    assert abs(a.sum() - b.sum()) / a.sum() < 1e-10
    assert b.max() < 0.8 * a.max()  # the PSF did spread the light


def test_convolve3_impulse_is_outer_product(O):
    rng = np.random.default_rng(5)
    kz, ky, kx = rng.random(7), rng.random(3), rng.random(5)
    # an impulse in the middle of a cube exactly one kernel wide gives the
    # kernel itself as the "valid" output
    cube = np.zeros((7 + 6, 3 + 2, 5 + 4))
    cube[6, 2, 4] = 1.0
    out = O.convolve3(cube, kz, ky, kx)
    ref = kz[:, None, None] * ky[None, :, None] * kx[None, None, :]
    np.testing.assert_allclose(out, ref, rtol=1e-14, atol=0)
    # in a larger cube the kernel lands centred on the impulse: input voxel
    # (10, 7, 8) is output voxel (10-3, 7-1, 8-2), and tap a sits a-3 away
    cube = np.zeros((20, 15, 16))
    cube[10, 7, 8] = 1.0
    out = O.convolve3(cube, kz, ky, kx)
    ref = np.zeros_like(out)
    for a in range(7):
        for b in range(3):
            for c in range(5):
                ref[10 - 3 + a - 3, 7 - 1 + b - 1, 8 - 2 + c - 2] = kz[a] * ky[b] * kx[c]
    np.testing.assert_allclose(out, ref, rtol=1e-14, atol=1e-300)


# ---------------------------------------------------------------------------
# Pin (d): separable passes equal brute-force 3-D convolution
# ---------------------------------------------------------------------------

def test_convolve3_matches_bruteforce_loops(O):
    rng = np.random.default_rng(11)
    cube = rng.random((9, 8, 10))
    kz, ky, kx = rng.random(5), rng.random(3), rng.random(5)   # asymmetric on purpose
    out = O.convolve3(cube, kz, ky, kx)
    k3 = kz[:, None, None] * ky[None, :, None] * kx[None, None, :]
    oz, oy, ox = 9 - 4, 8 - 2, 10 - 4
    ref = np.zeros((oz, oy, ox))
    for z in range(oz):
        for y in range(oy):
            for x in range(ox):
                s = 0.0
                for a in range(5):
                    for b in range(3):
                        for c in range(5):
                            s += k3[a, b, c] * cube[z + 4 - a, y + 2 - b, x + 4 - c]
                ref[z, y, x] = s
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=0)


def test_convolve3_matches_scipy(O):
    rng = np.random.default_rng(12)
    cube = rng.random((20, 17, 15))
    kz, ky, kx = rng.random(9), rng.random(7), rng.random(3)
    out = O.convolve3(cube, kz, ky, kx)
    k3 = kz[:, None, None] * ky[None, :, None] * kx[None, None, :]
    ref = signal.convolve(cube, k3, mode="valid", method="direct")
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=0)


def test_model_cube_voxels(O):
    """Random voxels of the model cube equal I(r) times a unit-area normal
    density of the line-of-sight velocity, at the stated fine-grid positions."""
    d = O.Desc(12, 10, 16, 2, 25.0, v0=7.0, crpix=8.0, psf_fwhm=2.0, lsf_sigma=20.0)
    p = par(xo=5.5, yo=4.2, pa=100.0, inc=55.0, vsys=7.0, vt=140.0, rt=2.5, sig=33.0, r0=3.0,
            i0=1.7)
    cube = O.model_cube(d, p)
    nxe, nye, nze, hp, hl = O.cube_dims(d)
    assert cube.shape == (nze, nye, nxe)
    rng = np.random.default_rng(3)
    for _ in range(200):
        zz, yy, xx = rng.integers(nze), rng.integers(nye), rng.integers(nxe)
        x = ((xx - hp) + 0.5) / 2 - 0.5
        y = ((yy - hp) + 0.5) / 2 - 0.5
        v = 7.0 + (((zz - hl) + 0.5) / 2 - 0.5 - 8.0) * 25.0
        inten = 1.7 * math.exp(-deprojected_radius(p, x, y) / 3.0)
        ref = inten * stats.norm.pdf(v, loc=projected_velocity(0, p, x, y), scale=33.0)
        assert abs(cube[zz, yy, xx] - ref) <= 1e-12 * max(ref, 1e-300) + 1e-300


# ---------------------------------------------------------------------------
# Down-sampling and moments (Sec. 2.2.4, 2.2.5)
# ---------------------------------------------------------------------------

def test_downsample_is_block_mean(O):
    rng = np.random.default_rng(2)
    fine = rng.random((6, 8, 10))
    out = O.downsample(fine, 2)
    ref = fine.reshape(3, 2, 4, 2, 5, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(out, ref, rtol=1e-14)
    np.testing.assert_array_equal(O.downsample(fine, 1), fine)


def test_moments_spikes(O):
    nz, dv = 10, 15.0
    vel = 100.0 + (np.arange(nz) - 5) * dv
    cube = np.zeros((nz, 1, 4))
    cube[3, 0, 0] = 2.0                       # one spike
    cube[2, 0, 1] = cube[6, 0, 1] = 1.0       # two equal spikes
    cube[4, 0, 2], cube[5, 0, 2], cube[6, 0, 2] = 1.0, 2.0, 1.0
    m = O.moments(cube, vel, dv, vsys=42.0)   # column 3 is empty
    assert m[0, 0, 0] == 2.0 * dv and m[1, 0, 0] == vel[3] and m[2, 0, 0] == 0.0
    assert abs(m[1, 0, 1] - (vel[2] + vel[6]) / 2) < 1e-12
    assert abs(m[2, 0, 1] - 2 * dv) < 1e-12
    assert abs(m[1, 0, 2] - vel[5]) < 1e-12
    assert abs(m[2, 0, 2] - dv * math.sqrt(0.5)) < 1e-12
    assert (m[0, 0, 3], m[1, 0, 3], m[2, 0, 3]) == (0.0, 42.0, 0.0)


def test_lines_outside_the_band(O):
    """Reading of Sec. 2.2.2 for lines outside the band: a fine spaxel keeps its
    line only if the line rises above 2^-40 of its peak (|v - vlos| <= sigma
    sqrt(80 ln 2) = 7.45 sigma) at some channel of the model band (data
    channels plus the spectral halo); then the whole sampled Gaussian counts.
    One spaxel on the kinematic centre (vlos = Vsys), channels -100..100 km/s
    every 10 km/s, sigma 10 km/s, no PSF or LSF: a line 7 sigma above the
    band gives the moments of its sampled wing over the band (written out
    here from their definition); 8 and 30 sigma outside give no flux, i.e.
    (0, Vsys, 0).  With an LSF the band grows by its halo (4 channels of
    10 km/s here): a line 7 sigma beyond the halo still reaches it, 8 sigma
    beyond does not."""
    d = O.Desc(1, 1, 21, 1, 10.0, v0=0.0, crpix=10.0, psf_fwhm=0.0, lsf_sigma=0.0)
    v = (np.arange(21) - 10) * 10.0
    for vsys in (170.0, -170.0):
        m = O.evaluate(d, par(xo=0.0, yo=0.0, vsys=vsys, sig=10.0, i0=1.3))
        g = np.exp(-0.5 * ((v - vsys) / 10.0) ** 2)
        m0 = 10.0 * 1.3 * g.sum() / (math.sqrt(2 * math.pi) * 10.0)
        m1 = np.sum(v * g) / g.sum()
        m2 = math.sqrt(np.sum(g * (v - m1) ** 2) / g.sum())
        assert m[0, 0, 0] > 0.0
        assert abs(m[0, 0, 0] - m0) <= 1e-12 * m0
        assert abs(m[1, 0, 0] - m1) <= 1e-9 and abs(m[2, 0, 0] - m2) <= 1e-9
    for vsys in (180.0, -180.0, 400.0, -400.0):
        m = O.evaluate(d, par(xo=0.0, yo=0.0, vsys=vsys, sig=10.0))
        assert (m[0, 0, 0], m[1, 0, 0], m[2, 0, 0]) == (0.0, vsys, 0.0)
    dl = O.Desc(1, 1, 21, 1, 10.0, v0=0.0, crpix=10.0, psf_fwhm=0.0, lsf_sigma=10.0)
    assert O.cube_dims(dl)[4] == 4
    assert O.evaluate(dl, par(xo=0.0, yo=0.0, vsys=210.0, sig=10.0))[0, 0, 0] > 0.0
    m = O.evaluate(dl, par(xo=0.0, yo=0.0, vsys=220.0, sig=10.0))
    assert (m[0, 0, 0], m[1, 0, 0], m[2, 0, 0]) == (0.0, 220.0, 0.0)


# ---------------------------------------------------------------------------
# Goodness of fit (eq. 11): hand-computed fixture
# ---------------------------------------------------------------------------

def test_chi2_golden(O):
    with open(os.path.join(GOLDEN, "chi2_3x3.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        c, n = O.chi2(g["m1"], g["m2"], g["v_obs"], g["s_obs"], g["e_v"], g["e_s"], g["mask"],
                      case["W"])
        assert abs(c - case["chi2"]) < 1e-12 and n == case["n_valid"]
    c, n = O.chi2(g["m1"], g["m2"], g["v_obs"], g["s_obs"], g["e_v"], g["e_s"],
                  np.zeros((3, 3)), 1.0)
    assert (c, n) == (0.0, 0)


# ---------------------------------------------------------------------------
# Exact invariants of the full pipeline (PSF and LSF on)
# ---------------------------------------------------------------------------

def full_desc(O, u=1, nz=64):
    return O.Desc(33, 33, nz, u, 20.0, v0=9.0, crpix=(nz - 1) / 2.0, psf_fwhm=3.0,
                  lsf_sigma=25.0)


def test_i0_is_a_pure_scale(O):
    d = full_desc(O)
    p = par(pa=33.0, inc=52.0, vsys=9.0, vt=170.0, rt=3.0, sig=25.0, r0=5.0)
    a = O.evaluate(d, p)
    p[P["i0"]] = 3.7
    b = O.evaluate(d, p)
    np.testing.assert_allclose(b[0], 3.7 * a[0], rtol=1e-13)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b[2], a[2], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("u", [1, 2])
def test_no_rotation_gives_systemic_field(O, u):
    d = full_desc(O, u=u, nz=48)
    p = par(pa=33.0, inc=52.0, vsys=9.0, vt=0.0, rt=3.0, sig=25.0, r0=5.0)
    m = O.evaluate(d, p)
    np.testing.assert_allclose(m[1], 9.0, rtol=0, atol=1e-9)
    np.testing.assert_allclose(m[2], m[2][16, 16], rtol=1e-9)


@pytest.mark.parametrize("u", [1, 2])
def test_point_reflection_symmetry(O, u):
    """Centre on a pixel and a channel grid symmetric about Vsys: reflecting
    through the centre negates m1 - Vsys and leaves m0, m2 unchanged."""
    d = full_desc(O, u=u)
    p = par(xo=16.0, yo=16.0, pa=71.0, inc=48.0, vsys=9.0, vt=190.0, rt=2.5, sig=22.0, r0=4.0)
    m = O.evaluate(d, p)
    refl = m[:, ::-1, ::-1]
    np.testing.assert_allclose(m[0], refl[0], rtol=1e-9)
    np.testing.assert_allclose(m[1] - 9.0, -(refl[1] - 9.0), rtol=0, atol=1e-8)
    np.testing.assert_allclose(m[2], refl[2], rtol=1e-9)


def test_pa_half_turn_negates_rotation(O):
    d = full_desc(O)
    p = par(xo=15.3, yo=16.8, pa=20.0, inc=61.0, vsys=9.0, vt=150.0, rt=3.0, sig=30.0, r0=4.0)
    a = O.evaluate(d, p)
    p[P["pa"]] += 180.0
    b = O.evaluate(d, p)
    np.testing.assert_allclose(b[1] - 9.0, -(a[1] - 9.0), rtol=0, atol=1e-8)
    np.testing.assert_allclose(b[0], a[0], rtol=1e-9)
    np.testing.assert_allclose(b[2], a[2], rtol=1e-9)


# ---------------------------------------------------------------------------
# Domain
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("slot,val", [("inc", 90.0), ("inc", 0.0), ("sig", 0.0), ("r0", -1.0),
                                      ("rt", 0.0), ("i0", 0.0), ("vt", float("nan")),
                                      ("xo", float("inf"))])
def test_out_of_domain_rows(O, slot, val):
    d = O.Desc(8, 8, 16, 1, 30.0, psf_fwhm=2.0, lsf_sigma=30.0)
    p = par(xo=4.0, yo=4.0)
    p[P[slot]] = val
    assert not O.params_valid(d, p)
    assert np.isnan(O.evaluate(d, p)).all()
    ones = np.ones((8, 8))
    c, n = O.eval_chi2(d, p, ones, ones, ones, ones, ones, 1.0)
    assert c == math.inf and n == 0
