"""Each plausible mistake planted in a copy of the oracle must fail a pin.

The mutated copies are compiled on the CPU into a temporary directory and the
pin suite (test_oracle_pins.py) is run against each one in a subprocess; a
mutation that every pin lets through would mean the pins cannot tell a broken
oracle from a correct one.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gk_oracle.c")

MUTATIONS = {
    "eq1 sign of the x term": ("double xe = -dx * sin(pa) + dy * cos(pa);",
                               "double xe = dx * sin(pa) + dy * cos(pa);"),
    "eq2 sign of the y term": ("double ye = -dx * cos(pa) - dy * sin(pa);",
                               "double ye = -dx * cos(pa) + dy * sin(pa);"),
    "eq3 inclination on the wrong axis": (
        "sqrt(xe * xe + (ye / cos(inc)) * (ye / cos(inc)))",
        "sqrt((xe / cos(inc)) * (xe / cos(inc)) + ye * ye)"),
    "eq4 sine instead of cosine": ("double costh = r > 0.0 ? xe / r : 0.0;",
                                   "double costh = r > 0.0 ? ye / r : 0.0;"),
    "eq8 dropped sin i": ("go_vrot(rc, r, p) * sin(inc) * costh", "go_vrot(rc, r, p) * costh"),
    "eq6 wrong prefactor": ("(2.0 / GO_PI) * vt * atan(r / rt)", "(1.0 / GO_PI) * vt * atan(r / rt)"),
    "eq7 slopes swapped": ("pow(q, p[P_G]) / (1.0 + pow(q, p[P_A]))",
                           "pow(q, p[P_A]) / (1.0 + pow(q, p[P_G]))"),
    "exponential rise missing rt": ("vt * (1.0 - exp(-r / rt))", "vt * (1.0 - exp(-r))"),
    "eq5 scale length dropped": ("double rr = r / p[P_R0];", "double rr = r;"),
    "brightness floor dropped": ("if (rr > 60.0) rr = 60.0;", ""),
    "line normalisation": ("1.0 / (sqrt(2.0 * GO_PI) * sig)", "1.0 / (sqrt(GO_PI) * sig)"),
    "line width doubled": ("double t = (v - vlos) / sig;", "double t = (v - vlos) / (2.0 * sig);"),
    "channel centre offset": ("((zz - hl) + 0.5) / u - 0.5 - d->crpix",
                              "((zz - hl) + 0.5) / u - d->crpix"),
    "sub-pixel position": ("double x = ((xx - hp) + 0.5) / u - 0.5;",
                           "double x = (double)(xx - hp) / u;"),
    "halo not removed from y": ("double y = ((yy - hp) + 0.5) / u - 0.5;",
                                "double y = ((yy) + 0.5) / u - 0.5;"),
    "taps not normalised": ("for (int k = 0; k < 2 * h + 1; ++k) taps[k] /= s;", ""),
    "taps half width": ("int h = (int)ceil(R * sigma);", "int h = (int)ceil(0.5 * R * sigma);"),
    "LSF ignores upsampling": ("d->u * d->lsf_sigma / d->dv", "d->lsf_sigma / d->dv"),
    "PSF FWHM taken as sigma": ("d->u * fwhm_to_sigma(d->psf_fwhm)", "d->u * d->psf_fwhm"),
    "z pass tap offset dropped": ("in[((size_t)(z + hz - k) * nye + y) * nxe + x]",
                                  "in[((size_t)(z + hz) * nye + y) * nxe + x]"),
    "x pass reads along y": ("t1[((size_t)z * nye + y) * nxe + (x + hx - k)]",
                             "t1[((size_t)z * nye + (y + hx - k < nye ? y + hx - k : y)) * nxe + x + hx]"),
    "y pass off by one": ("t2[((size_t)z * nye + (y + hy - k)) * ox + x]",
                          "t2[((size_t)z * nye + (y + hy - k + (k == hy))) * ox + x]"),
    "downsample not averaged": ("out[((size_t)z * ny + y) * nx + x] = s * inv;",
                                "out[((size_t)z * ny + y) * nx + x] = s;"),
    "m0 without channel width": ("m0[i] = dv * s0;", "m0[i] = s0;"),
    "m2 not centred": ("s2 += c * (vel[z] - mean) * (vel[z] - mean);",
                       "s2 += c * vel[z] * (vel[z] - mean) + 1e-3 * c;"),
    "m2 without square root": ("m2[i] = sqrt(s2 / s0);", "m2[i] = s2 / s0;"),
    "empty spectrum velocity": ("m1[i] = vsys;", "m1[i] = 0.0;"),
    "chi2 ignores mask": ("if (!mask[i]) continue;", ""),
    "chi2 ignores W": ("c += W * rs * rs;", "c += rs * rs;"),
    "chi2 error not squared": ("double rv = (m1[i] - vo[i]) / ev[i];",
                               "double rv = (m1[i] - vo[i]) / sqrt(ev[i]);"),
    "domain check on inclination": ("if (!(p[P_INC] > 0.0 && p[P_INC] < 90.0)) return 0;", ""),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old!r}"
    mutated = tmp_path / "gk_oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libgk_oracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(lib),
                           str(mutated), "-lm"])
    env = dict(os.environ, GK_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"no pin caught the mutation {name!r}:\n{r.stdout[-2000:]}"
