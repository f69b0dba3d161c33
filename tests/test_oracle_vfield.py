"""Pins of the oracle's velocity-field strategy (Bekiaris et al. 2016, Sec. 2.2.1).

The strategy evaluates the kinematic model of eq. 8 at every data pixel and
goes straight to the goodness of fit of eq. 11.  Its oracle is pinned here
against the polar-form restatement of a projected thin rotating disc, the
cube strategy's moments in the limit where they reduce to the same maps (no
PSF or LSF, channels much finer than the line), hand-computed chi-square
sums, and the special values of the rotation curves.
"""
import math

import numpy as np
import pytest

from test_oracle_pins import deprojected_radius, par, projected_velocity


def vf_desc(O, nx=29, ny=23, rc=0):
    return O.Desc(nx, ny, 1, 1, 10.0, rc=rc)


@pytest.mark.parametrize("rc,pa,inc", [(0, 0.0, 45.0), (0, 60.0, 30.0), (1, 137.0, 70.0),
                                       (2, 251.0, 55.0), (1, -20.0, 10.0), (2, 359.0, 85.0)])
def test_vfield_velocity_is_the_projected_disc(O, rc, pa, inc):
    p = par(pa=pa, inc=inc, vsys=1234.5, vt=180.0, rt=3.5, sig=25.0, r0=7.0,
            a=1.7 if rc == 1 else 1.0, g=0.6 if rc == 1 else 1.0, xo=13.4, yo=10.8)
    d = vf_desc(O, rc=rc)
    m = O.vfield(d, p)
    err = max(abs(m[1, y, x] - projected_velocity(rc, p, x, y))
              for y in range(d.ny) for x in range(d.nx))
    assert err < 1e-9


def test_vfield_brightness_and_dispersion_planes(O):
    p = par(xo=14.0, yo=11.0, pa=35.0, inc=60.0, sig=31.5, r0=4.0, i0=3.0)
    d = vf_desc(O)
    m = O.vfield(d, p)
    for (y, x) in [(11, 14), (0, 0), (22, 28), (5, 17)]:
        r = deprojected_radius(p, x, y)
        assert abs(m[0, y, x] - 3.0 * math.exp(-min(r / 4.0, 60.0))) < 1e-13 * 3.0
    assert np.all(m[2] == 31.5)
    # beyond 60 scale lengths the brightness is held at I0 exp(-60)
    p[8] = 0.1
    m = O.vfield(d, p)
    assert deprojected_radius(p, 0, 0) / 0.1 > 60
    assert abs(m[0, 0, 0] / (3.0 * math.exp(-60.0)) - 1) < 1e-12


def test_vfield_major_and_minor_axes(O):
    """Epinat curve at r = rt gives Vt / 2 for any slopes; PA = 0 puts the
    receding major axis on +y and the minor axis on x."""
    d = vf_desc(O, nx=21, ny=21, rc=1)
    p = par(xo=10.0, yo=10.0, pa=0.0, inc=40.0, vsys=-50.0, vt=240.0, rt=5.0, a=2.3, g=0.7)
    m1 = O.vfield(d, p)[1]
    s = math.sin(math.radians(40.0))
    assert abs(m1[15, 10] - (-50.0 + 120.0 * s)) < 1e-10
    assert abs(m1[5, 10] - (-50.0 - 120.0 * s)) < 1e-10
    assert np.all(np.abs(m1[10, :] + 50.0) < 1e-10)     # minor axis: systemic
    assert abs(m1[10, 10] + 50.0) < 1e-12                # the centre itself


@pytest.mark.parametrize("rc", [0, 1, 2])
def test_vfield_is_the_cube_strategy_without_beam_smearing(O, rc):
    """With no PSF and no LSF, and channels much finer than the line inside a
    wide band, the cube strategy's moments of each spaxel's sampled Gaussian
    are its area, centre and width: the two strategies give the same maps."""
    p = par(xo=7.3, yo=8.6, pa=70.0, inc=55.0, vsys=20.0, vt=150.0, rt=2.5, sig=30.0, r0=5.0,
            i0=2.0, a=1.2 if rc == 1 else 1.0, g=0.9 if rc == 1 else 1.0)
    nz, dv = 480, 2.0
    dc = O.Desc(15, 17, nz, 1, dv, v0=0.0, crpix=(nz - 1) / 2.0, rc=rc)
    cube = O.evaluate(dc, p)
    vf = O.vfield(O.Desc(15, 17, 1, rc=rc), p)
    assert np.max(np.abs(cube[1] - vf[1])) < 1e-8
    assert np.max(np.abs(cube[2] - vf[2])) < 1e-8
    assert np.max(np.abs(cube[0] - vf[0]) / vf[0]) < 1e-10


def test_vfield_chi2_hand_sums(O):
    """Observed maps = model + known offsets: chi2 is the sum of squared
    offsets over the unmasked pixels, divided by the errors; the dispersion
    term enters with weight W and is dropped at W = 0."""
    d = vf_desc(O, nx=4, ny=3)
    p = par(xo=1.5, yo=1.0, pa=20.0, inc=50.0, vsys=5.0, sig=22.0)
    m = O.vfield(d, p)
    dvel = np.array([[1.0, -2.0, 0.5, 0.0], [3.0, 0.0, -1.0, 2.0], [0.25, 4.0, 0.0, -3.0]])
    dsig = np.array([[0.0, 1.0, 0.0, 2.0], [-1.0, 0.0, 0.5, 0.0], [3.0, 0.0, 1.0, 0.0]])
    ev = np.full((3, 4), 2.0)
    es = np.full((3, 4), 0.5)
    mask = np.array([[1, 1, 0, 1], [1, 1, 1, 0], [0, 1, 1, 1]], dtype=np.uint8)
    vo, so = m[1] - dvel, m[2] - dsig
    c0, n0 = O.vfield_chi2(d, p, vo, so, ev, es, mask, 0.0)
    # velocity offsets on unmasked pixels: 1,-2,0 | 3,0,-1 | 4,0,-3 -> 40, / 2^2
    assert n0 == 9
    assert abs(c0 - 40.0 / 4.0) < 1e-9
    c1, n1 = O.vfield_chi2(d, p, vo, so, ev, es, mask, 0.3)
    # dispersion offsets on unmasked pixels: 0,1,2 | -1,0,0.5 | 0,1,0 -> 7.25, / 0.5^2
    assert n1 == 9
    assert abs(c1 - (10.0 + 0.3 * 7.25 / 0.25)) < 1e-9


def test_vfield_out_of_domain(O):
    d = vf_desc(O, nx=5, ny=4, rc=1)
    p = par(g=0.0)
    assert np.isnan(O.vfield(d, p)).all()
    ones = np.ones(20)
    c, n = O.vfield_chi2(d, p, ones, ones, ones, ones, np.ones(20, np.uint8), 0.0)
    assert c == math.inf and n == 0
