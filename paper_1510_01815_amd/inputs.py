"""Seeded synthetic workloads: instrument grids, parameter draws, noise, masks.

This module holds no arithmetic of the method itself (no geometry, no line
profiles, no convolution, no moments, no chi-square).  It only describes the
workloads and draws random numbers, so both the GPU path and the CPU oracle
can be fed identical inputs.  An observation is built by the caller from model
maps that it computed itself, via ``make_observation``.

Workloads follow the shapes of the paper's data (Bekiaris et al. 2016, Sec. 3,
Tables 1-2): mock IFU cubes of 32-96 pixels a side at 10-60 km/s resolution,
Fabry-Perot-like high-resolution cubes and low-resolution beam-smeared cubes.
Parameter slots: x0, y0, PA [deg], i [deg], Vsys, Vt, rt, sigma, r0, I0, a, g.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NPAR = 12
XO, YO, PA, INC, VSYS, VT, RT, SIG, R0, I0, A, G = range(NPAR)
PARAM_NAMES = ("xo", "yo", "pa", "inc", "vsys", "vt", "rt", "sig", "r0", "i0", "a", "g")
RC_ARCTAN, RC_EPINAT, RC_BOISSIER = 0, 1, 2

FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))


@dataclass
class Grid:
    """Instrument/data grid of one observation."""
    nx: int
    ny: int
    nz: int
    dv: float
    psf_fwhm: float
    lsf_sigma: float
    u: int = 1
    v0: float = 0.0
    crpix: float | None = None
    R: float = 4.0
    rc: int = RC_ARCTAN
    strategy: int = 0   # 0: intensity cube, 1: velocity field (no spectral axis used)

    def as_dict(self) -> dict:
        crpix = self.nz / 2.0 if self.crpix is None else self.crpix
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, u=self.u, dv=self.dv, v0=self.v0,
                    crpix=crpix, psf_fwhm=self.psf_fwhm, lsf_sigma=self.lsf_sigma, R=self.R,
                    rc=self.rc, strategy=self.strategy)


def rng_for(config_id: int, galaxy: int = 0, purpose: int = 0) -> np.random.Generator:
    """Independent, reproducible stream per (workload, galaxy, purpose)."""
    return np.random.default_rng([config_id, galaxy, purpose])


# --------------------------------------------------------------------------
# Workload 1: single galaxy, 32 x 32 x 64, arctan curve, plain LM
# --------------------------------------------------------------------------

def c1_grid() -> Grid:
    return Grid(32, 32, 64, 30.0, psf_fwhm=2.5, lsf_sigma=30.0, rc=RC_ARCTAN)


def c1_truth() -> np.ndarray:
    p = np.zeros(NPAR)
    p[[XO, YO, PA, INC, VSYS, VT, RT, SIG, R0, I0, A, G]] = \
        [16.0, 16.0, 60.0, 45.0, 0.0, 200.0, 4.0, 40.0, 6.0, 1.0, 1.0, 1.0]
    return p


def c1_start(rng: np.random.Generator, free=(XO, YO, PA, INC, VSYS, VT, RT, SIG, R0),
             frac: float = 0.2) -> np.ndarray:
    """Truth perturbed by +/- 20% with a random sign per free slot (Vsys,
    whose truth is 0, by +/- 6 km/s)."""
    p = c1_truth()
    for k in free:
        s = 1.0 if rng.random() < 0.5 else -1.0
        p[k] = p[k] + s * 6.0 if k == VSYS else p[k] * (1.0 + s * frac)
    return p


# --------------------------------------------------------------------------
# Workload 2: Fabry-Perot-like, 128 x 128 x 48, exponential-rise curve, NS
# --------------------------------------------------------------------------

# the spectral resolution is not given for this workload; a 30 km/s FWHM
# (the Fabry-Perot survey resolution of Sec. 3.2) is used
C2_LSF_SIGMA = 30.0 / FWHM_PER_SIGMA


def c2_grid() -> Grid:
    return Grid(128, 128, 48, 16.0, psf_fwhm=3.0, lsf_sigma=C2_LSF_SIGMA, rc=RC_BOISSIER)


def c2_draw(rng: np.random.Generator, n: int = 1) -> np.ndarray:
    """Generative parameter draws for the 128 x 128 workload."""
    p = np.zeros((n, NPAR))
    p[:, XO] = rng.uniform(0.45, 0.55, n) * 128
    p[:, YO] = rng.uniform(0.45, 0.55, n) * 128
    p[:, PA] = rng.uniform(0.0, 360.0, n)
    p[:, INC] = rng.uniform(20.0, 70.0, n)
    p[:, VSYS] = rng.uniform(-20.0, 20.0, n)
    p[:, VT] = rng.uniform(100.0, 300.0, n)
    p[:, RT] = rng.uniform(5.0, 20.0, n)
    p[:, SIG] = rng.uniform(10.0, 40.0, n)
    p[:, R0] = 20.0
    p[:, I0] = 1.0
    p[:, A] = 1.0
    p[:, G] = 1.0
    return p


def c2_prior_box() -> tuple[np.ndarray, np.ndarray]:
    """Uniform prior box for nested sampling on the 128 x 128 workload: the
    generative ranges widened x1.5 about their centres (clipped to physical
    values), centre within 0.4-0.6 of the field, free Vsys, r0 and I0."""
    lo = np.array([0.4 * 128, 0.4 * 128, 0.0, 7.5, -50.0, 50.0, 1.25, 2.5, 10.0, 0.5, 1.0, 1.0])
    hi = np.array([0.6 * 128, 0.6 * 128, 360.0, 82.5, 50.0, 350.0, 23.75, 47.5, 40.0, 2.0, 1.0, 1.0])
    return lo, hi


# --------------------------------------------------------------------------
# Shared prior box of the single-galaxy workload (Table 2 of the paper with
# PA widened to a full turn), used by the survey / grid / surrogate workloads
# --------------------------------------------------------------------------

def c1_box_draw(rng: np.random.Generator, n: int, nxy, psf_fwhm) -> np.ndarray:
    nxy = np.broadcast_to(np.asarray(nxy, dtype=np.float64), (n,))
    fw = np.broadcast_to(np.asarray(psf_fwhm, dtype=np.float64), (n,))
    p = np.zeros((n, NPAR))
    p[:, XO] = rng.uniform(0.4, 0.6, n) * nxy
    p[:, YO] = rng.uniform(0.4, 0.6, n) * nxy
    p[:, PA] = rng.uniform(0.0, 360.0, n)
    p[:, INC] = rng.uniform(5.0, 85.0, n)
    p[:, VSYS] = 0.0
    p[:, VT] = rng.uniform(50.0, 300.0, n)
    p[:, RT] = rng.uniform(0.5, 2.0, n) * fw
    p[:, SIG] = rng.uniform(20.0, 100.0, n)
    p[:, R0] = rng.uniform(1.0, 3.0, n) * fw
    p[:, I0] = 1.0
    p[:, A] = 1.0
    p[:, G] = 1.0
    return p


# --------------------------------------------------------------------------
# Workload 3: survey of uneven cubes
# --------------------------------------------------------------------------

@dataclass
class SurveyGalaxy:
    grid: Grid
    truth: np.ndarray
    noise: float
    seed: tuple = field(default_factory=tuple)


def c3_survey(n: int = 2000, seed: int = 3) -> list[SurveyGalaxy]:
    rng = rng_for(3, 0, seed)
    out = []
    for k in range(n):
        side = int(rng.integers(16, 97))
        nz = int(rng.integers(32, 129))
        fw = float(rng.uniform(1.5, 4.0))
        g = Grid(side, side, nz, 30.0, psf_fwhm=fw, lsf_sigma=30.0, rc=RC_ARCTAN)
        truth = c1_box_draw(rng, 1, side, fw)[0]
        out.append(SurveyGalaxy(g, truth, float(rng.uniform(3.0, 15.0)), (3, k)))
    return out


# --------------------------------------------------------------------------
# Workload 4: low-resolution beam-smeared grid search
# --------------------------------------------------------------------------

def c4_galaxy(k: int) -> tuple[Grid, np.ndarray]:
    rng = rng_for(4, k, 0)
    fw = float(rng.uniform(3.0, 6.0))
    g = Grid(30, 30, 64, 30.0, psf_fwhm=fw, lsf_sigma=30.0, rc=RC_ARCTAN)
    p = c1_box_draw(rng, 1, 30, fw)[0]
    p[R0] = rng.uniform(2.0, 5.0)
    p[VT] = rng.uniform(50.0, 250.0)
    return g, p


# --------------------------------------------------------------------------
# Workload 5: surrogate instrument
# --------------------------------------------------------------------------

def c5_grid() -> Grid:
    return Grid(64, 64, 64, 30.0, psf_fwhm=2.5, lsf_sigma=30.0, rc=RC_ARCTAN)


def c5_box() -> tuple[np.ndarray, np.ndarray]:
    """Prior box of the surrogate workload (the single-galaxy box on a 64 px
    grid, PSF FWHM 2.5): the training range of the surrogate and the nested
    sampler's prior; a and g are fixed at 1 (arctan curve)."""
    lo = np.array([25.6, 25.6, 0.0, 5.0, -50.0, 50.0, 1.25, 20.0, 2.5, 0.5, 1.0, 1.0])
    hi = np.array([38.4, 38.4, 360.0, 85.0, 50.0, 300.0, 5.0, 100.0, 7.5, 2.0, 1.0, 1.0])
    return lo, hi


C5_FREE = (1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0)


def c5_galaxy(k: int) -> np.ndarray:
    """Truth of galaxy k: drawn in the box, with PA kept 20 deg away from the
    box ends so that no posterior straddles the 0/360 cut."""
    rng = rng_for(5, k, 0)
    lo, hi = c5_box()
    p = lo + rng.random(NPAR) * (hi - lo)
    p[PA] = rng.uniform(20.0, 340.0)
    p[VSYS] = rng.uniform(-20.0, 20.0)
    p[I0] = 1.0
    return p


# --------------------------------------------------------------------------
# Workload 6: velocity fields shaped like the GHASP Fabry-Perot sample
# (Sec. 4.2 of the paper): side x side maps (256 or 512), Epinat curve,
# velocity only, kinematic centre held fixed -> 7 free parameters
# --------------------------------------------------------------------------

STRATEGY_CUBE, STRATEGY_VFIELD = 0, 1
GHASP_FREE = (0, 0, 1, 1, 1, 1, 1, 0, 0, 0, 1, 1)


def ghasp_grid(side: int = 512) -> Grid:
    return Grid(side, side, 1, 1.0, psf_fwhm=0.0, lsf_sigma=0.0, rc=RC_EPINAT,
                strategy=STRATEGY_VFIELD)


def ghasp_box(side: int = 512) -> tuple[np.ndarray, np.ndarray]:
    """Fitting box of the velocity-field workload."""
    lo = np.array([0.0, 0.0, -180.0, 5.0, 0.0, 10.0, 0.005 * side, 1.0, 0.01 * side, 0.1,
                   0.2, 0.2])
    hi = np.array([side, side, 540.0, 85.0, 10000.0, 600.0, 0.5 * side, 200.0, side, 10.0,
                   4.0, 4.0])
    return lo, hi


def ghasp_draw(rng: np.random.Generator, n: int, side: int = 512) -> np.ndarray:
    """Nearby discs filling much of the field: systemic velocities of a few
    thousand km/s, turn-over radii of 3-15% of the field, inner slope g in
    [0.8, 1.6] and outer slope a >= g so that the curve stays bounded."""
    p = np.zeros((n, NPAR))
    p[:, XO] = rng.uniform(0.45, 0.55, n) * side
    p[:, YO] = rng.uniform(0.45, 0.55, n) * side
    p[:, PA] = rng.uniform(0.0, 360.0, n)
    p[:, INC] = rng.uniform(20.0, 75.0, n)
    p[:, VSYS] = rng.uniform(300.0, 6000.0, n)
    p[:, VT] = rng.uniform(80.0, 300.0, n)
    p[:, RT] = rng.uniform(0.03, 0.15, n) * side
    p[:, SIG] = 20.0
    p[:, R0] = rng.uniform(0.08, 0.2, n) * side
    p[:, I0] = 1.0
    p[:, G] = rng.uniform(0.8, 1.6, n)
    p[:, A] = p[:, G] + rng.uniform(0.0, 1.0, n)
    return p


def ghasp_start(rng: np.random.Generator, truth: np.ndarray, side: int = 512) -> np.ndarray:
    """Start of a fit: the free parameters perturbed about the truth."""
    p = truth.copy()
    p[PA] += rng.uniform(-10.0, 10.0)
    p[INC] = np.clip(p[INC] + rng.uniform(-10.0, 10.0), 10.0, 80.0)
    p[VSYS] += rng.uniform(-20.0, 20.0)
    p[VT] *= rng.uniform(0.8, 1.2)
    p[RT] *= rng.uniform(0.8, 1.2)
    p[A] *= rng.uniform(0.85, 1.15)
    p[G] *= rng.uniform(0.85, 1.15)
    return p


# coverage of a Fabry-Perot map: the disc out to ~3 scale lengths, with a
# patchy fraction of the pixels (no H-alpha) missing; velocity noise 3-10 km/s
GHASP_FLUX_FRAC = math.exp(-3.0)
GHASP_HOLES = 0.3


# --------------------------------------------------------------------------
# Random draws of the Monte-Carlo error estimates (Sec. 4.2, 4.3)
# --------------------------------------------------------------------------

def mc_permutations(rng: np.random.Generator, n_sim: int, n_valid: int) -> np.ndarray:
    """One permutation of 0..n_valid-1 per simulation, int32 [n_sim][n_valid]."""
    return np.stack([rng.permutation(n_valid) for _ in range(n_sim)]).astype(np.int32)


def mc_normals(rng: np.random.Generator, n_sim: int, ny: int, nx: int) -> np.ndarray:
    """Standard normal draws per simulation, map and pixel, float32 [n_sim][2][ny][nx]."""
    return rng.standard_normal((n_sim, 2, ny, nx)).astype(np.float32)


# --------------------------------------------------------------------------
# Observations from model maps computed by the caller
# --------------------------------------------------------------------------

@dataclass
class Observation:
    vel: np.ndarray
    sig: np.ndarray
    evel: np.ndarray
    esig: np.ndarray
    mask: np.ndarray
    W: float = 1.0


def make_observation(maps: np.ndarray, noise_v: float, rng: np.random.Generator,
                     noise_s: float | None = None, flux_frac: float = 0.01,
                     random_mask: float = 0.0, W: float = 1.0) -> Observation:
    """maps[3][ny][nx] = (m0, m1, m2) of the truth -> noisy observed maps.

    Gaussian noise of `noise_v` on the velocity map and `noise_s` (default:
    the same) on the dispersion map; error maps equal the noise levels (a
    noise-free observation uses unit errors).  Spaxels whose flux is below
    `flux_frac` of the peak are masked out, and a further random fraction
    `random_mask` is masked.
    """
    maps = np.asarray(maps, dtype=np.float64)
    ns = noise_v if noise_s is None else noise_s
    shape = maps.shape[1:]
    vel = maps[1] + noise_v * rng.standard_normal(shape)
    sig = maps[2] + ns * rng.standard_normal(shape)
    ev = np.full(shape, noise_v if noise_v > 0 else 1.0)
    es = np.full(shape, ns if ns > 0 else 1.0)
    mask = (maps[0] >= flux_frac * np.nanmax(maps[0])).astype(np.uint8)
    if random_mask > 0:
        mask &= (rng.random(shape) >= random_mask).astype(np.uint8)
    f32 = np.float32
    return Observation(vel.astype(f32), sig.astype(f32), ev.astype(f32), es.astype(f32), mask, W)
