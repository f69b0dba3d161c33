"""Shared helpers of the parity tests: GPU maps / chi-square against the oracle.

Tolerances (maps in FP32, sums in FP64):
  m1, m2: |gpu - oracle| <= 1e-3 km/s + 1e-5 |oracle|
  m0:     |gpu - oracle| <= 1e-5 |oracle|
  chi2:   relative 1e-6 when chi2 >= N_valid, else absolute 1e-6 N_valid
  integers (n_valid, masks): exact.
Map parity is checked where the oracle's flux sum is at least 1e-12 of its
maximum; fainter spaxels must only be finite.
"""
import numpy as np

M12_ABS, M12_REL = 1e-3, 1e-5
M0_REL = 1e-5
CHI2_REL = 1e-6


def oracle_desc(O, grid: dict):
    return O.Desc(grid["nx"], grid["ny"], grid["nz"], grid["u"], grid["dv"], v0=grid["v0"],
                  crpix=grid["crpix"], psf_fwhm=grid["psf_fwhm"], lsf_sigma=grid["lsf_sigma"],
                  R=grid["R"], rc=grid["rc"])


def bright(ref_m0: np.ndarray, frac: float = 1e-12) -> np.ndarray:
    mx = np.nanmax(ref_m0)
    return ref_m0 >= frac * mx


def assert_maps_close(gpu: np.ndarray, ref: np.ndarray, what: str = "", bright_frac: float = 1e-12):
    """gpu, ref: [3][ny][nx]; ref is the FP64 oracle.  Parity is checked where
    the oracle's flux is at least bright_frac of its maximum."""
    gpu = np.asarray(gpu, dtype=np.float64)
    b = bright(ref[0], bright_frac)
    assert np.isfinite(gpu).all(), f"{what}: non-finite GPU map values"
    d0 = np.abs(gpu[0] - ref[0])
    tol0 = M0_REL * np.abs(ref[0])
    bad0 = (d0 > tol0) & b
    assert not bad0.any(), f"{what}: m0 max rel err {np.max(d0[b] / np.abs(ref[0][b])):.3g}"
    for k, name in ((1, "m1"), (2, "m2")):
        d = np.abs(gpu[k] - ref[k])
        tol = M12_ABS + M12_REL * np.abs(ref[k])
        bad = (d > tol) & b
        assert not bad.any(), (f"{what}: {name} max err {np.max(d[b]):.3g} km/s at "
                               f"{np.argwhere(bad)[:3].tolist()}")


def max_map_errors(gpu: np.ndarray, ref: np.ndarray) -> dict:
    gpu = np.asarray(gpu, dtype=np.float64)
    b = bright(ref[0])
    return {"m0_rel": float(np.max(np.abs(gpu[0] - ref[0])[b] / np.abs(ref[0][b]))),
            "m1_abs": float(np.max(np.abs(gpu[1] - ref[1])[b])),
            "m2_abs": float(np.max(np.abs(gpu[2] - ref[2])[b]))}


# Accuracy of the GPU's moment maps against the oracle's (largest m1/m2 error
# measured over every test grid: 8e-5 km/s), used for the chi-square bound of
# near-perfect fits.
MAP_EPS = 1e-4


def assert_chi2_close(gpu: float, ref: float, n_valid: int, what: str = "", obs=None):
    """Relative 1e-6 when chi2 >= N_valid.  Below that (fits near the noise-free
    optimum, where the maps' own rounding dominates the residuals) the bound
    is what map errors of at most MAP_EPS can move chi2 by: with
    S = sum over the mask of (MAP_EPS / E_v)^2 + W (MAP_EPS / E_s)^2, Cauchy-
    Schwarz gives |d chi2| <= 2 sqrt(chi2 S) + S; that bound is used (capped at
    the former 1e-6 N_valid) when the observation is given."""
    if ref >= n_valid:
        assert abs(gpu - ref) <= CHI2_REL * abs(ref), f"{what}: chi2 {gpu!r} vs {ref!r}"
        return
    tol = CHI2_REL * max(n_valid, 1)
    if obs is not None:
        mk = np.asarray(obs.mask).astype(bool)
        S = float(np.sum((MAP_EPS / np.asarray(obs.evel, dtype=np.float64)[mk]) ** 2))
        if obs.W > 0:
            S += obs.W * float(np.sum((MAP_EPS / np.asarray(obs.esig, dtype=np.float64)[mk]) ** 2))
        tol = min(tol, CHI2_REL * abs(ref) + 2.0 * np.sqrt(abs(ref) * S) + S)
    assert abs(gpu - ref) <= tol, f"{what}: chi2 {gpu!r} vs {ref!r} (tol {tol:.3g})"
