"""Reference optimisers of the oracle (Sec. 2.3), plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle.py): used by tests/ to check the GPU
library's fitters.  Each follows a step-by-step rule that the library's
fitters follow too, stated in each function's docstring; the paper names the
algorithms but uses third-party implementations (mpfit, MultiNest), so the
details below are this project's reading.

levenberg_marquardt: Sec. 2.3.1 -- gradient/curvature local optimiser with box
constraints and a finite-difference Jacobian of absolute step ~0.1 (Sec. 4).
mc_errors: Monte-Carlo parameter errors by refits of simulated observations,
shuffled residuals (Sec. 4.2) or perturbations by the error maps (Sec. 4.3).
fit_gaussian_line(s): Gaussian fit of each spectrum of a cube, the alternative
to moments (Sec. 2.2.5, Sec. 5.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import oracle as O


@dataclass
class LMResult:
    p: np.ndarray
    chi2: float
    iterations: int
    n_evals: int
    errors: np.ndarray
    reason: str
    history: list = field(default_factory=list)


def _cholesky_solve(M: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solves M x = rhs for symmetric positive definite M by an explicit
    Cholesky factorisation M = L L^T (no library solver)."""
    n = M.shape[0]
    L = np.zeros_like(M)
    for i in range(n):
        for j in range(i + 1):
            s = M[i, j] - sum(L[i, k] * L[j, k] for k in range(j))
            if i == j:
                if s <= 0.0:
                    raise np.linalg.LinAlgError("matrix not positive definite")
                L[i, i] = math.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (rhs[i] - sum(L[i, k] * y[k] for k in range(i))) / L[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (y[i] - sum(L[k, i] * x[k] for k in range(i + 1, n))) / L[i, i]
    return x


def levenberg_marquardt(resid, p0, free, lo, hi, h=0.1, lam0=1e-3, max_iter=200,
                        ftol=1e-10, xtol=1e-10) -> LMResult:
    """Damped Gauss-Newton with box constraints.

    resid(p) -> residual vector r(p); chi2 = r.r.
    Jacobian column a (free slots): (r(p+) - r(p-)) / (p+ - p-), with
    p+- = p_a +- h clipped to the box.  A = J^T J, g = J^T r; free slots whose
    column is identically zero are frozen.  Step: (A + lam diag A) d = -g,
    trial = clip(p + d).  A trial that lowers chi2 is accepted (lam /= 10),
    otherwise lam *= 10.  Stops after an accepted step when the relative
    chi2 decrease <= ftol or max |d_a| / (|p_a| + 1e-10) <= xtol, or when
    lam > 1e10 or after max_iter trials.  Errors: sqrt(diag(A^-1)) at the end.
    """
    p = np.clip(np.asarray(p0, dtype=np.float64).copy(), lo, hi)
    free = [a for a in range(len(p)) if free[a] and hi[a] > lo[a]]
    n_evals = 0

    def jac(pc):
        nonlocal n_evals
        r0 = resid(pc)
        n_evals += 1
        cols = []
        for a in free:
            pp, pm = pc.copy(), pc.copy()
            pp[a] = min(pc[a] + h, hi[a])
            pm[a] = max(pc[a] - h, lo[a])
            cols.append((resid(pp) - resid(pm)) / (pp[a] - pm[a]))
            n_evals += 2
        J = np.stack(cols, axis=1) if cols else np.zeros((len(r0), 0))
        return r0, J

    r, J = jac(p)
    chi2 = float(r @ r)
    A, g = J.T @ J, J.T @ r
    lam, it, reason, hist = lam0, 0, "maxiter", []
    while it < max_iter:
        it += 1
        act = [k for k in range(len(free)) if A[k, k] > 0.0]
        d = np.zeros(len(free))
        if act:
            M = A[np.ix_(act, act)].copy()
            M[np.diag_indices_from(M)] *= (1.0 + lam)
            d[act] = _cholesky_solve(M, -g[act])
        pt = p.copy()
        for k, a in enumerate(free):
            pt[a] = min(max(p[a] + d[k], lo[a]), hi[a])
        rt, Jt = jac(pt)
        chi2t = float(rt @ rt)
        if chi2t < chi2:
            step = max((abs(pt[a] - p[a]) / (abs(p[a]) + 1e-10) for a in free), default=0.0)
            dec = (chi2 - chi2t) / chi2 if chi2 > 0 else 0.0
            p, r, J, chi2 = pt, rt, Jt, chi2t
            A, g = J.T @ J, J.T @ r
            lam = lam / 10.0
            hist.append(chi2)
            if chi2 == 0.0 or dec <= ftol:
                reason = "ftol"
                break
            if step <= xtol:
                reason = "xtol"
                break
        else:
            lam *= 10.0
            if lam > 1e10:
                reason = "lambda"
                break
    err = np.zeros(len(p))
    act = [k for k in range(len(free)) if A[k, k] > 0.0]
    if act:
        Ainv = np.linalg.inv(A[np.ix_(act, act)])
        for j, k in enumerate(act):
            err[free[k]] = math.sqrt(max(Ainv[j, j], 0.0))
    return LMResult(p, chi2, it, n_evals, err, reason, hist)


def model_residuals(d: "O.Desc", obs):
    """r(p) of the oracle model against an observation: (m1 - v_obs)/E_v then
    sqrt(W) (m2 - s_obs)/E_s over unmasked pixels (the terms of eq. 11)."""
    mk = np.asarray(obs.mask).astype(bool).ravel()
    vo = np.asarray(obs.vel, dtype=np.float64).ravel()[mk]
    so = np.asarray(obs.sig, dtype=np.float64).ravel()[mk]
    ev = np.asarray(obs.evel, dtype=np.float64).ravel()[mk]
    es = np.asarray(obs.esig, dtype=np.float64).ravel()[mk]
    sw = math.sqrt(obs.W)

    def resid(p):
        m = O.evaluate(d, p)
        rv = (m[1].ravel()[mk] - vo) / ev
        rs = sw * (m[2].ravel()[mk] - so) / es if obs.W > 0 else np.zeros_like(rv)
        return np.concatenate([rv, rs])
    return resid


def vfield_residuals(d: "O.Desc", obs):
    """r(p) of the velocity-field strategy (Sec. 2.2.1): the terms of eq. 11
    with the eq. 8 velocity field and sigma in place of m1 and m2."""
    mk = np.asarray(obs.mask).astype(bool).ravel()
    vo = np.asarray(obs.vel, dtype=np.float64).ravel()[mk]
    so = np.asarray(obs.sig, dtype=np.float64).ravel()[mk]
    ev = np.asarray(obs.evel, dtype=np.float64).ravel()[mk]
    es = np.asarray(obs.esig, dtype=np.float64).ravel()[mk]
    sw = math.sqrt(obs.W)

    def resid(p):
        m = O.vfield(d, p)
        rv = (m[1].ravel()[mk] - vo) / ev
        rs = sw * (m[2].ravel()[mk] - so) / es if obs.W > 0 else np.zeros_like(rv)
        return np.concatenate([rv, rs])
    return resid


def mc_simulations(best_maps: np.ndarray, obs, mode: str, perm=None, noise=None) -> list:
    """Simulated observations of the Monte-Carlo error estimates.

    shuffle (Sec. 4.2): the residual field of the best fit, observation minus
    model over the unmasked pixels, has its pixel positions shuffled and is
    added back to the best-fit model; the unmasked pixels are numbered in
    row-major order and simulation s puts residual perm[s][k] on pixel k.
    perturb (Sec. 4.3): each unmasked pixel of the observed maps is moved by
    its measurement error times noise[s].  The dispersion map changes only
    when the observation weighs it (W > 0).  Maps are returned as float32,
    like every observation.
    """
    mk = np.asarray(obs.mask).astype(bool)
    idx = np.flatnonzero(mk.ravel())
    vo = np.asarray(obs.vel, dtype=np.float64).ravel()
    so = np.asarray(obs.sig, dtype=np.float64).ravel()
    out = []
    n_sim = len(perm) if mode == "shuffle" else len(noise)
    for s in range(n_sim):
        v, g = vo.copy(), so.copy()
        if mode == "shuffle":
            bv = best_maps[1].ravel().astype(np.float64)
            bs = best_maps[2].ravel().astype(np.float64)
            src = idx[np.asarray(perm[s])]
            v[idx] = bv[idx] + (vo[src] - bv[src])
            if obs.W > 0:
                g[idx] = bs[idx] + (so[src] - bs[src])
        else:
            n = np.asarray(noise[s], dtype=np.float64)
            ev = np.asarray(obs.evel, dtype=np.float64).ravel()
            es = np.asarray(obs.esig, dtype=np.float64).ravel()
            v[idx] = vo[idx] + ev[idx] * n[0].ravel()[idx]
            if obs.W > 0:
                g[idx] = so[idx] + es[idx] * n[1].ravel()[idx]
        out.append(type(obs)(v.reshape(mk.shape).astype(np.float32),
                             g.reshape(mk.shape).astype(np.float32), obs.evel, obs.esig, obs.mask,
                             obs.W))
    return out


def mc_errors(residuals_of, best, best_maps, obs, free, lo, hi, mode, perm=None, noise=None,
              **lm):
    """Monte-Carlo parameter errors: every simulation refitted by LM from
    `best`; returns (fits [n_sim][12], sample SD of each free slot).
    residuals_of(obs) -> r(p) of the strategy in use."""
    sims = mc_simulations(best_maps, obs, mode, perm, noise)
    fits = np.array([levenberg_marquardt(residuals_of(o), best, free, lo, hi, **lm).p
                     for o in sims])
    sd = np.where(np.asarray(free, dtype=bool), fits.std(axis=0, ddof=1), 0.0)
    return fits, sd


@dataclass
class LineFit:
    amp: float
    vel: float
    disp: float
    chi2: float
    iterations: int
    status: int   # 0 no line, 1 converged, 2 damping limit, 3 iteration cap


def fit_gaussian_line(spec, v, dv, max_iter=100, lam0=1e-3, ftol=1e-12, xtol=1e-12) -> LineFit:
    """Gaussian line fit of one spectrum (the alternative to moments of
    Sec. 2.2.5, done on the CPU with mpfit in the paper, Sec. 5.2).

    Model A exp(-(v - mu)^2 / (2 s^2)) at the channel velocities v, residuals
    model - data, analytic Jacobian.  Start: the moments of the spectrum
    clipped at zero (noise makes raw wing moments meaningless): area S0 dv,
    centre, width, A = area / (s sqrt(2 pi)); no line (S0 <= 0 or a zero
    width) gives status 0.  Box: A >= 0, mu inside the band, s in
    [dv / 4, n dv].  Step rule as levenberg_marquardt: (M + lam diag M) d = -g,
    trial clipped to the box, accepted if chi2 drops (lam /= 10, stop when the
    relative decrease <= ftol or the largest relative step <= xtol), else
    lam *= 10 (stop above 1e10); at most max_iter trials.
    """
    spec = np.asarray(spec, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    pos = np.maximum(spec, 0.0)
    s0 = float(np.sum(pos))
    if not s0 > 0.0:
        return LineFit(0.0, math.nan, math.nan, math.nan, 0, 0)
    mu = float(np.sum(pos * v)) / s0
    var = float(np.sum(pos * (v - mu) ** 2)) / s0
    if not var > 0.0:
        return LineFit(0.0, math.nan, math.nan, math.nan, 0, 0)
    lo = np.array([0.0, min(v[0], v[-1]), 0.25 * dv])
    hi = np.array([math.inf, max(v[0], v[-1]), len(v) * dv])
    s = math.sqrt(var)
    p = np.clip(np.array([s0 * dv / (s * math.sqrt(2.0 * math.pi)), mu, s]), lo, hi)

    def system(q):
        A, m, w = q
        t = (v - m) / w
        e = np.exp(-0.5 * t * t)
        r = A * e - spec
        J = np.stack([e, A * e * t / w, A * e * t * t / w], axis=1)
        return float(r @ r), J.T @ J, J.T @ r

    chi2, M, g = system(p)
    lam, it, status = lam0, 0, 3
    while it < max_iter:
        it += 1
        K = M.copy()
        K[np.diag_indices_from(K)] *= (1.0 + lam)
        try:
            d = _cholesky_solve(K, -g)
        except np.linalg.LinAlgError:
            d = np.zeros(3)
        pt = np.clip(p + d, lo, hi)
        chi2t, Mt, gt = system(pt)
        if chi2t < chi2:
            step = float(np.max(np.abs(pt - p) / (np.abs(p) + 1e-10)))
            dec = (chi2 - chi2t) / chi2
            p, chi2, M, g = pt, chi2t, Mt, gt
            lam /= 10.0
            if chi2 == 0.0 or dec <= ftol or step <= xtol:
                status = 1
                break
        else:
            lam *= 10.0
            if lam > 1e10:
                status = 2
                break
    return LineFit(float(p[0]), float(p[1]), float(p[2]), chi2, it, status)


def fit_gaussian_lines(cube, v, dv, **kw) -> np.ndarray:
    """Every spectrum of cube [nz][ny][nx]: maps [3][ny][nx] = (line flux
    A s sqrt(2 pi), centre, width); NaN centre and width where there is no
    line.  Also returns the status map."""
    nz, ny, nx = cube.shape
    maps = np.zeros((3, ny, nx))
    st = np.zeros((ny, nx), dtype=np.int32)
    for y in range(ny):
        for x in range(nx):
            f = fit_gaussian_line(cube[:, y, x], v, dv, **kw)
            maps[:, y, x] = (f.amp * f.disp * math.sqrt(2.0 * math.pi) if f.status else 0.0,
                             f.vel, f.disp)
            st[y, x] = f.status
    return maps, st


@dataclass
class GridResult:
    best: np.ndarray
    chi2: float
    best_index: int
    levels: int
    n_evals: int
    spacing: np.ndarray


def nested_grid(chi2_fn, lo0, hi0, free, fixed, n=16, max_levels=3, accuracy=None) -> GridResult:
    """Nested grids (Sec. 2.3.3): a regular grid of n_k nodes along each free
    slot k (end points included; n an int for every slot, or one count per
    slot as the paper's per-parameter grids of Sec. 4) over the current box;
    the least-chi2 node (lowest linear index on ties; the index is mixed
    radix, first free slot varying slowest) centres the next box, node +- one
    spacing clipped to the initial box.  Stops after max_levels or when every
    spacing is below accuracy."""
    slots = [k for k in range(len(fixed)) if free[k]]
    nk = {k: (n if np.isscalar(n) else int(n[k])) for k in slots}
    lo = np.array(lo0, dtype=np.float64).copy()
    hi = np.array(hi0, dtype=np.float64).copy()
    best_p, best_v, best_i, n_evals, level = None, math.inf, -1, 0, 0
    spacing = np.zeros(len(fixed))
    total = 1
    for k in slots:
        total *= nk[k]
    for level in range(1, max_levels + 1):
        step = {k: (hi[k] - lo[k]) / (nk[k] - 1) for k in slots}
        best_v, best_i = math.inf, -1
        for L in range(total):
            p = np.array(fixed, dtype=np.float64).copy()
            rem = L
            for k in reversed(slots):
                p[k] = lo[k] + (rem % nk[k]) * step[k]
                rem //= nk[k]
            v = chi2_fn(p)
            n_evals += 1
            if v < best_v:
                best_v, best_i, best_p = v, L, p
        for k in slots:
            spacing[k] = step[k]
            lo[k] = max(best_p[k] - step[k], lo0[k])
            hi[k] = min(best_p[k] + step[k], hi0[k])
        if accuracy is not None and all(step[k] < accuracy[k] for k in slots):
            break
    return GridResult(best_p, best_v, best_i, level, n_evals, spacing)
