"""ctypes binding of libgbk.so (C ABI in include/gbk.h).

Argument marshalling only: every step of the evaluation runs in the HIP
library.  PyTorch provides device memory and streams (``data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``).  Importing this module does not
need a GPU; loading the library does, and a missing library raises at once
(there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgbk.so")

GK_OK, GK_PARTIAL, GK_EINVAL, GK_ENOMEM, GK_EDEVICE, GK_ENOTCONV, GK_ESTATE = 0, 1, -1, -2, -3, -4, -5
NPAR = 12
RC = {"arctan": 0, "epinat": 1, "boissier": 2}
CONV = {"auto": 0, "direct": 1, "fft": 2}
STRATEGY = {"cube": 0, "vfield": 1}

# exported symbols, kept in step with include/gbk.h
SYMBOLS = (
    "gk_create_model", "gk_destroy_model", "gk_set_observation", "gk_observation_count",
    "gk_evaluate_batch", "gk_chi2_batch", "gk_residual_batch", "gk_model_dims", "gk_last_error",
    "gk_set_profiling", "gk_read_profile", "gk_lm_default_opts", "gk_fit_lm",
    "gk_ns_default_opts", "gk_fit_nested", "gk_nested_sample", "gk_philox4x32", "gk_fit_grid",
    "gk_create_survey", "gk_destroy_survey", "gk_survey_chi2", "gk_fit_lm_survey",
    "gk_surrogate_default_opts", "gk_surrogate_create", "gk_surrogate_destroy",
    "gk_surrogate_train", "gk_surrogate_weight_count", "gk_surrogate_get_weights",
    "gk_surrogate_set_weights", "gk_surrogate_save", "gk_surrogate_load",
    "gk_surrogate_gradients", "gk_surrogate_predict",
    "gk_surrogate_chi2", "gk_fit_nested_screened", "gk_gemm_bf16", "gk_model_conv_path",
    "gk_set_launch_mode", "gk_graph_launches", "gk_autotune", "gk_set_conv_config",
    "gk_mc_errors", "gk_line_default_opts", "gk_fit_lines", "gk_surrogate_step",
    "gk_chi2_batch_noalloc",
)
MC = {"shuffle": 0, "perturb": 1}
LM_REASONS = {1: "ftol", 2: "xtol", 3: "lambda", 4: "maxiter"}
GK_PROF_TIMING, GK_PROF_COUNT = 1, 2


class GkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gbk status {status}: {msg}")
        self.status = status


class ModelDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("upsample", ctypes.c_int32), ("dv_kms", ctypes.c_double),
                ("v0_kms", ctypes.c_double), ("crpix", ctypes.c_double),
                ("psf_fwhm_pix", ctypes.c_double), ("lsf_sigma_kms", ctypes.c_double),
                ("kernel_radius_sigma", ctypes.c_double), ("rc", ctypes.c_int32),
                ("conv_mode", ctypes.c_int32), ("strategy", ctypes.c_int32)]


class ProfileStats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double * 4), ("launches", ctypes.c_int64 * 4),
                ("support_voxels", ctypes.c_int64), ("rows", ctypes.c_int64)]


class LMOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fd_step", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("ftol", ctypes.c_double), ("xtol", ctypes.c_double)]


class LineOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lambda0", ctypes.c_double), ("ftol", ctypes.c_double), ("xtol", ctypes.c_double)]


class LMResult(ctypes.Structure):
    _fields_ = [("chi2", ctypes.c_double), ("n_valid", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("reason", ctypes.c_int32),
                ("n_evals", ctypes.c_int64), ("errors", ctypes.c_double * NPAR)]


class NSOpts(ctypes.Structure):
    _fields_ = [("n_live", ctypes.c_int32), ("batch", ctypes.c_int32), ("max_iter", ctypes.c_int64),
                ("enlarge", ctypes.c_double), ("tol", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("max_ell", ctypes.c_int32), ("batch_max", ctypes.c_int32),
                ("accept_target", ctypes.c_int32), ("screen_cost", ctypes.c_double),
                ("screen_rows", ctypes.c_int32), ("separate_modes", ctypes.c_int32),
                ("max_wall_s", ctypes.c_double)]


NS_MAX_MODES = 8  # GK_NS_MAX_MODES


class NSMode(ctypes.Structure):
    _fields_ = [("logz", ctypes.c_double), ("logz_err", ctypes.c_double),
                ("info_h", ctypes.c_double), ("n_live", ctypes.c_int64),
                ("n_samples", ctypes.c_int64)] + [
                (n, ctypes.c_double * NPAR) for n in ("mean", "sd", "median", "q16", "q84")]


class NSResult(ctypes.Structure):
    _fields_ = [("logz", ctypes.c_double), ("logz_err", ctypes.c_double),
                ("info_h", ctypes.c_double), ("max_logl", ctypes.c_double),
                ("n_iter", ctypes.c_int64), ("n_evals", ctypes.c_int64),
                ("n_launches", ctypes.c_int64)] + [
                (n, ctypes.c_double * NPAR) for n in ("best", "mean", "sd", "median", "q16", "q84")] + [
                (n, ctypes.c_int64) for n in ("n_screened", "n_rejected", "n_audited", "n_audit_miss")] + [
                ("t_wall_s", ctypes.c_double), ("t_wait_s", ctypes.c_double),
                ("n_modes", ctypes.c_int32), ("reserved_modes", ctypes.c_int32),
                ("modes", NSMode * NS_MAX_MODES)]


class TuneResult(ctypes.Structure):
    _fields_ = [("conv_mode", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("ms_best", ctypes.c_double),
                ("ms", ctypes.c_double * 16)]


TUNE_CANDIDATES = (("fft", 0, 0), ("direct", 32, 32), ("direct", 64, 32), ("direct", 32, 16),
                   ("direct", 16, 16), ("direct", 32, 8), ("direct", 16, 8), ("direct", 8, 8),
                   ("direct", 64, 16))


class SurrogateOpts(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("layers", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lr", ctypes.c_double), ("lr_final", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class GridResult(ctypes.Structure):
    _fields_ = [("best", ctypes.c_double * NPAR), ("chi2", ctypes.c_double),
                ("best_index", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_evals", ctypes.c_int64),
                ("spacing", ctypes.c_double * NPAR)]


LOGLIKE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                              ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


def _ns_opts(L, **opts):
    o = NSOpts()
    _check(L.gk_ns_default_opts(ctypes.byref(o)))
    for k, v in opts.items():
        setattr(o, k, v)
    if "n_live" in opts and "batch" not in opts:
        o.batch = o.n_live
    return o


def _ns_dict(r: "NSResult", st: int, dim: int, samples=None) -> dict:
    out = {"logz": r.logz, "logz_err": r.logz_err, "info_h": r.info_h, "max_logl": r.max_logl,
           "n_iter": r.n_iter, "n_evals": r.n_evals, "n_launches": r.n_launches, "status": st,
           "n_screened": r.n_screened, "n_rejected": r.n_rejected, "n_audited": r.n_audited,
           "n_audit_miss": r.n_audit_miss, "t_wall_s": r.t_wall_s, "t_wait_s": r.t_wait_s}
    for n in ("best", "mean", "sd", "median", "q16", "q84"):
        out[n] = np.array(getattr(r, n)[:dim])
    out["modes"] = []
    for k in range(r.n_modes):
        md = r.modes[k]
        e = {"logz": md.logz, "logz_err": md.logz_err, "info_h": md.info_h,
             "n_live": md.n_live, "n_samples": md.n_samples}
        for n in ("mean", "sd", "median", "q16", "q84"):
            e[n] = np.array(getattr(md, n)[:dim])
        out["modes"].append(e)
    if samples is not None:
        out["samples"] = samples
    return out


def _grid_dict(r: "GridResult") -> dict:
    return {"best": np.array(r.best[:]), "chi2": r.chi2, "best_index": r.best_index,
            "levels": r.levels, "n_evals": r.n_evals, "spacing": np.array(r.spacing[:])}


def philox4x32(ctr, key):
    """Philox4x32-10 block of the library (gk_philox4x32)."""
    L = load()
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    _check(L.gk_philox4x32(c, k, o))
    return list(o)


def nested_sample(loglike, lo, hi, want_samples=0, **opts) -> dict:
    """gk_nested_sample with a Python batch log-likelihood loglike(theta[n, dim]) -> [n]."""
    L = load()
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    dim = lo.size

    def cb(theta, n, d, out, user):
        try:
            th = np.ctypeslib.as_array(theta, shape=(n, d)).copy()
            v = np.asarray(loglike(th), dtype=np.float64)
            np.ctypeslib.as_array(out, shape=(n,))[:] = v
            return 0
        except Exception:
            return 1
    fn = LOGLIKE_FN(cb)
    r = NSResult()
    o = _ns_opts(L, **opts)
    buf = np.zeros((max(want_samples, 1), NPAR + 1))
    ns = ctypes.c_int64(0)
    st = L.gk_nested_sample(dim, lo.ctypes.data, hi.ctypes.data, fn, None, ctypes.byref(o),
                            ctypes.byref(r), buf.ctypes.data if want_samples else None,
                            want_samples, ctypes.byref(ns))
    if st < 0 and st != GK_ENOTCONV:
        _check(st)
    smp = buf[: ns.value, list(range(dim)) + [NPAR]] if want_samples else None
    return _ns_dict(r, st, dim, smp)


KERNEL_NAMES = ("k_prep", "k_line_sums", "k_psf_moments", "k_reduce_chi2")

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libgbk.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with __graft_entry__.build() "
                                "(hipcc --offload-arch=gfx950)")
    L = ctypes.CDLL(path)
    vp, i32, i64p, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_double
    L.gk_create_model.argtypes = [ctypes.POINTER(ModelDesc), ctypes.c_int, ctypes.POINTER(vp)]
    L.gk_destroy_model.argtypes = [vp]
    L.gk_set_observation.argtypes = [vp, vp, vp, vp, vp, vp, dp]
    L.gk_observation_count.argtypes = [vp, i64p]
    L.gk_evaluate_batch.argtypes = [vp, vp, i32, vp, vp]
    L.gk_chi2_batch.argtypes = [vp, vp, i32, vp, vp, vp]
    L.gk_chi2_batch_noalloc.argtypes = [vp, vp, i32, vp, vp, vp]
    L.gk_residual_batch.argtypes = [vp, vp, i32, vp, vp]
    L.gk_model_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.gk_set_profiling.argtypes = [vp, ctypes.c_int]
    L.gk_read_profile.argtypes = [vp, ctypes.POINTER(ProfileStats)]
    L.gk_lm_default_opts.argtypes = [ctypes.POINTER(LMOpts)]
    L.gk_fit_lm.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(LMOpts), ctypes.POINTER(LMResult)]
    L.gk_ns_default_opts.argtypes = [ctypes.POINTER(NSOpts)]
    L.gk_fit_nested.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(NSOpts),
                                ctypes.POINTER(NSResult), vp, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64)]
    L.gk_nested_sample.argtypes = [ctypes.c_int32, vp, vp, LOGLIKE_FN, vp,
                                   ctypes.POINTER(NSOpts), ctypes.POINTER(NSResult), vp,
                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.gk_philox4x32.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(ctypes.c_uint32)]
    L.gk_fit_grid.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp,
                              ctypes.POINTER(GridResult)]
    L.gk_fit_grid_nd.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp,
                                 ctypes.POINTER(GridResult)]
    L.gk_fit_grid_survey.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int32, vp,
                                     ctypes.POINTER(GridResult)]
    L.gk_create_survey.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp)]
    L.gk_destroy_survey.argtypes = [vp]
    L.gk_survey_chi2.argtypes = [vp, vp, vp, i32, vp, vp]
    L.gk_fit_lm_survey.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(LMOpts),
                                   ctypes.POINTER(LMResult)]
    L.gk_line_default_opts.argtypes = [ctypes.POINTER(LineOpts)]
    L.gk_fit_lines.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.POINTER(LineOpts), vp, vp, vp, vp]
    L.gk_mc_errors.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(LMOpts), ctypes.c_int32,
                               ctypes.c_int32, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32)]
    L.gk_surrogate_default_opts.argtypes = [ctypes.POINTER(SurrogateOpts)]
    L.gk_surrogate_create.argtypes = [vp, vp, vp, ctypes.POINTER(SurrogateOpts), ctypes.POINTER(vp)]
    L.gk_surrogate_destroy.argtypes = [vp]
    L.gk_surrogate_train.argtypes = [vp, ctypes.c_int64, vp]
    L.gk_surrogate_weight_count.argtypes = [vp]
    L.gk_surrogate_get_weights.argtypes = [vp, vp, ctypes.c_int64]
    L.gk_surrogate_set_weights.argtypes = [vp, vp, ctypes.c_int64]
    L.gk_surrogate_save.argtypes = [vp, ctypes.c_char_p]
    L.gk_surrogate_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
    L.gk_surrogate_gradients.argtypes = [vp, vp, i32, vp, ctypes.POINTER(ctypes.c_double)]
    L.gk_surrogate_predict.argtypes = [vp, vp, i32, vp, vp]
    L.gk_surrogate_step.argtypes = [vp, vp, i32, dp, ctypes.POINTER(ctypes.c_double)]
    L.gk_surrogate_chi2.argtypes = [vp, vp, vp, i32, vp, vp]
    L.gk_fit_nested_screened.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(NSOpts), dp, dp,
                                         ctypes.POINTER(NSResult), vp, ctypes.c_int64, i64p]
    L.gk_gemm_bf16.argtypes = [i32, i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, vp]
    L.gk_model_conv_path.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.gk_set_launch_mode.argtypes = [vp, ctypes.c_int32]
    L.gk_autotune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(TuneResult)]
    L.gk_set_conv_config.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.gk_graph_launches.argtypes = [vp, i64p]
    L.gk_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS:
        if name == "gk_surrogate_weight_count":
            L.gk_surrogate_weight_count.restype = ctypes.c_int64
        elif name != "gk_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int, allow_partial: bool = True) -> int:
    if st < 0:
        raise GkError(st, load().gk_last_error().decode())
    if st == GK_PARTIAL and not allow_partial:
        raise GkError(st, "rows out of domain")
    return st


def _stream_ptr(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _params_arg(params):
    """(pointer, B, keepalive) for a [B][12] float64 host array or CUDA tensor."""
    try:
        import torch
        if isinstance(params, torch.Tensor):
            if params.dtype != torch.float64 or params.dim() != 2 or params.shape[1] != NPAR:
                raise ValueError("params must be a [B][12] float64 tensor")
            params = params.contiguous()
            return params.data_ptr(), params.shape[0], params
    except ImportError:
        pass
    a = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, NPAR)
    return a.ctypes.data, a.shape[0], a


class Model:
    """One instrument grid on one device; see gk_create_model."""

    def __init__(self, nx, ny, nz, dv, psf_fwhm=0.0, lsf_sigma=0.0, u=1, v0=0.0, crpix=None,
                 R=4.0, rc=0, device=0, conv="auto", strategy=0):
        L = load()
        if isinstance(rc, str):
            rc = RC[rc]
        if isinstance(conv, str):
            conv = CONV[conv]
        if isinstance(strategy, str):
            strategy = STRATEGY[strategy]
        self.desc = ModelDesc(nx, ny, nz, u, dv, v0, nz / 2.0 if crpix is None else crpix,
                              psf_fwhm, lsf_sigma, R, rc, conv, strategy)
        self.strategy = strategy
        self.nx, self.ny, self.nz, self.device = nx, ny, nz, device
        h = ctypes.c_void_p()
        _check(L.gk_create_model(ctypes.byref(self.desc), device, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_grid(cls, grid, device=0, conv="auto"):
        d = grid.as_dict() if hasattr(grid, "as_dict") else dict(grid)
        return cls(d["nx"], d["ny"], d["nz"], d["dv"], d["psf_fwhm"], d["lsf_sigma"], d["u"],
                   d["v0"], d["crpix"], d["R"], d["rc"], device, conv, d.get("strategy", 0))

    @classmethod
    def velocity_field(cls, nx, ny, rc=0, device=0):
        """A velocity-field strategy model (Sec. 2.2.1) of an nx x ny map."""
        return cls(nx, ny, 1, 1.0, rc=rc, device=device, strategy=STRATEGY["vfield"])

    def close(self):
        if getattr(self, "_h", None):
            load().gk_destroy_model(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self):
        d = (ctypes.c_int32 * 5)()
        _check(load().gk_model_dims(self._h, d))
        return tuple(d)

    def set_observation(self, vel, sig, evel, esig, mask, W=1.0):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        vel, evel = f(vel), f(evel)
        sig = None if sig is None else f(sig)
        esig = None if esig is None else f(esig)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self._obs = (vel, sig, evel, esig, mask)
        ptr = lambda a: None if a is None else a.ctypes.data
        _check(load().gk_set_observation(self._h, ptr(vel), ptr(sig), ptr(evel), ptr(esig),
                                         ptr(mask), float(W)))

    def set_obs(self, obs):
        self.set_observation(obs.vel, obs.sig, obs.evel, obs.esig, obs.mask, obs.W)

    def set_launch_mode(self, mode: str) -> None:
        """"graph" (default: repeated device-row calls replay a HIP graph) or "eager"."""
        _check(load().gk_set_launch_mode(self._h, {"eager": 0, "graph": 1}[mode]))

    def graph_launches(self) -> int:
        n = ctypes.c_int64()
        _check(load().gk_graph_launches(self._h, ctypes.byref(n)))
        return n.value

    def autotune(self, batch: int) -> dict:
        """Times the convolution configurations and keeps the fastest (gk_autotune)."""
        r = TuneResult()
        _check(load().gk_autotune(self._h, batch, ctypes.byref(r)))
        return {"conv": {1: "direct", 2: "fft"}[r.conv_mode], "tile": (r.tile_x, r.tile_y),
                "ms_best": r.ms_best, "n_candidates": r.n_candidates,
                "ms": {c: r.ms[k] for k, c in enumerate(TUNE_CANDIDATES) if r.ms[k] >= 0}}

    def set_conv_config(self, conv: str, tile_x: int = 0, tile_y: int = 0) -> None:
        _check(load().gk_set_conv_config(self._h, CONV[conv], tile_x, tile_y))

    def conv_path(self) -> str:
        """"direct" or "fft": the spatial convolution the model runs."""
        c = ctypes.c_int32()
        _check(load().gk_model_conv_path(self._h, ctypes.byref(c)))
        return {1: "direct", 2: "fft"}[c.value]

    def n_valid(self) -> int:
        n = ctypes.c_int64()
        _check(load().gk_observation_count(self._h, ctypes.byref(n)))
        return n.value

    def evaluate(self, params, out=None, stream=None):
        """maps [B][3][ny][nx] float32 CUDA tensor (m0, m1, m2)."""
        import torch
        p, B, keep = _params_arg(params)
        if out is None:
            out = torch.empty((B, 3, self.ny, self.nx), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        self.last_status = _check(load().gk_evaluate_batch(self._h, p, B, out.data_ptr(),
                                                           _stream_ptr(stream)))
        return out

    def chi2(self, params, out=None, n_valid=None, stream=None):
        """(chi2 [B] float64, n_valid [B] int64) CUDA tensors."""
        import torch
        p, B, keep = _params_arg(params)
        dev = f"cuda:{self.device}"
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=dev)
        if n_valid is None:
            n_valid = torch.empty(B, dtype=torch.int64, device=dev)
        self.last_status = _check(load().gk_chi2_batch(self._h, p, B, out.data_ptr(),
                                                       n_valid.data_ptr(), _stream_ptr(stream)))
        return out, n_valid

    def chi2_noalloc(self, params, out, n_valid=None, stream=None):
        """gk_chi2_batch_noalloc: chi2 of device rows into the caller's device
        tensors out [B] float64 and n_valid [B] int64 (optional), with the
        library's fixed scratch array (nothing is allocated)."""
        p, B, keep = _params_arg(params)
        self.last_status = _check(load().gk_chi2_batch_noalloc(
            self._h, p, B, out.data_ptr(),
            None if n_valid is None else n_valid.data_ptr(), _stream_ptr(stream)))
        return out, n_valid

    def set_profiling(self, flags: int):
        _check(load().gk_set_profiling(self._h, flags))

    def read_profile(self) -> dict:
        st = ProfileStats()
        _check(load().gk_read_profile(self._h, ctypes.byref(st)))
        return {"kernel_ms": dict(zip(KERNEL_NAMES, st.kernel_ms)),
                "launches": dict(zip(KERNEL_NAMES, st.launches)),
                "support_voxels": st.support_voxels, "rows": st.rows}

    def fit_lm(self, p0, free, lo=None, hi=None, **opts) -> dict:
        """Levenberg-Marquardt fit (gk_fit_lm); returns the fitted row and diagnostics."""
        L = load()
        o = LMOpts()
        _check(L.gk_lm_default_opts(ctypes.byref(o)))
        for k, v in opts.items():
            setattr(o, k, v)
        p = np.ascontiguousarray(p0, dtype=np.float64).copy()
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
        hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
        r = LMResult()
        st = L.gk_fit_lm(self._h, p.ctypes.data, fm.ctypes.data,
                         None if lo_a is None else lo_a.ctypes.data,
                         None if hi_a is None else hi_a.ctypes.data, ctypes.byref(o), ctypes.byref(r))
        if st < 0 and st != GK_ENOTCONV:
            _check(st)
        return {"p": p, "chi2": r.chi2, "n_valid": r.n_valid, "iterations": r.iterations,
                "reason": LM_REASONS.get(r.reason, str(r.reason)), "n_evals": r.n_evals,
                "errors": np.array(r.errors[:]), "status": st}

    def mc_errors(self, best, free, lo=None, hi=None, mode="shuffle", perm=None, noise=None,
                  **opts) -> dict:
        """Monte-Carlo parameter errors (gk_mc_errors): every simulation's fit and the
        standard deviation over them."""
        L = load()
        o = LMOpts()
        _check(L.gk_lm_default_opts(ctypes.byref(o)))
        for k, v in opts.items():
            setattr(o, k, v)
        b = np.ascontiguousarray(best, dtype=np.float64)
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64)
        hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64)
        md = MC[mode] if isinstance(mode, str) else int(mode)
        pa = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        na = None if noise is None else np.ascontiguousarray(noise, dtype=np.float32)
        n_sim = len(pa) if pa is not None else (len(na) if na is not None else 0)
        fits = np.zeros((max(n_sim, 1), NPAR))
        sd = np.zeros(NPAR)
        capped = ctypes.c_int32(0)
        ptr = lambda a: None if a is None else a.ctypes.data
        _check(L.gk_mc_errors(self._h, b.ctypes.data, fm.ctypes.data, ptr(lo_a), ptr(hi_a),
                              ctypes.byref(o), md, n_sim, ptr(pa), ptr(na), fits.ctypes.data,
                              sd.ctypes.data, ctypes.byref(capped)))
        return {"fits": fits[:n_sim], "sd": sd, "n_capped": capped.value}

    def fit_nested(self, lo, hi, free, fixed, want_samples=0, **opts) -> dict:
        """Nested sampling of the model's posterior (gk_fit_nested)."""
        L = load()
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        fx = np.ascontiguousarray(fixed, dtype=np.float64)
        r = NSResult()
        o = _ns_opts(L, **opts)
        buf = np.zeros((max(want_samples, 1), NPAR + 1))
        ns = ctypes.c_int64(0)
        st = L.gk_fit_nested(self._h, lo.ctypes.data, hi.ctypes.data, fm.ctypes.data,
                             fx.ctypes.data, ctypes.byref(o), ctypes.byref(r),
                             buf.ctypes.data if want_samples else None, want_samples,
                             ctypes.byref(ns))
        if st < 0 and st != GK_ENOTCONV:
            _check(st)
        return _ns_dict(r, st, NPAR, buf[: ns.value] if want_samples else None)

    def fit_grid(self, lo, hi, free, fixed, n_per_dim=16, max_levels=3, accuracy=None) -> dict:
        """Nested-grid search: gk_fit_grid for one node count, gk_fit_grid_nd for a
        count per slot (a sequence of 12)."""
        L = load()
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (lo, hi, fixed)]
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        acc = None if accuracy is None else np.ascontiguousarray(accuracy, dtype=np.float64)
        r = GridResult()
        if np.isscalar(n_per_dim):
            _check(L.gk_fit_grid(self._h, a[0].ctypes.data, a[1].ctypes.data, fm.ctypes.data,
                                 a[2].ctypes.data, int(n_per_dim), max_levels,
                                 None if acc is None else acc.ctypes.data, ctypes.byref(r)))
        else:
            ns = np.ascontiguousarray(n_per_dim, dtype=np.int32)
            _check(L.gk_fit_grid_nd(self._h, a[0].ctypes.data, a[1].ctypes.data, fm.ctypes.data,
                                    a[2].ctypes.data, ns.ctypes.data, max_levels,
                                    None if acc is None else acc.ctypes.data, ctypes.byref(r)))
        return _grid_dict(r)

    def residuals(self, params, out=None, stream=None):
        """resid [B][2][ny][nx] float64 CUDA tensor."""
        import torch
        p, B, keep = _params_arg(params)
        if out is None:
            out = torch.empty((B, 2, self.ny, self.nx), dtype=torch.float64,
                              device=f"cuda:{self.device}")
        self.last_status = _check(load().gk_residual_batch(self._h, p, B, out.data_ptr(),
                                                           _stream_ptr(stream)))
        return out


def fit_lines(cube, v0, dv, crpix, stream=None, **opts):
    """Gaussian fit of every spectrum of a channel-major float32 CUDA tensor
    cube [nz, ...] (gk_fit_lines): (maps [3, ...] float32, status, iterations)."""
    import torch
    L = load()
    o = LineOpts()
    _check(L.gk_line_default_opts(ctypes.byref(o)))
    for k, v in opts.items():
        setattr(o, k, v)
    assert cube.dtype == torch.float32 and cube.is_cuda and cube.is_contiguous()
    nz = cube.shape[0]
    nspec = cube.numel() // nz
    maps = torch.empty((3,) + tuple(cube.shape[1:]), dtype=torch.float32, device=cube.device)
    st = torch.empty(tuple(cube.shape[1:]), dtype=torch.int32, device=cube.device)
    it = torch.empty(tuple(cube.shape[1:]), dtype=torch.int32, device=cube.device)
    _check(L.gk_fit_lines(cube.data_ptr(), nz, nspec, v0, dv, crpix, ctypes.byref(o),
                          maps.data_ptr(), st.data_ptr(), it.data_ptr(), _stream_ptr(stream)))
    return maps, st, it


class Survey:
    """A set of models on one device evaluated in ragged batches (gk_create_survey)."""

    def __init__(self, models):
        L = load()
        self.models = list(models)
        arr = (ctypes.c_void_p * len(self.models))(*[m._h.value for m in self.models])
        h = ctypes.c_void_p()
        _check(L.gk_create_survey(arr, len(self.models), ctypes.byref(h)))
        self._h = h
        self.device = self.models[0].device

    def close(self):
        if getattr(self, "_h", None):
            load().gk_destroy_survey(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def chi2(self, model_idx, params, out=None, stream=None):
        """chi2 [B] float64 CUDA tensor of rows params [B][12] of models model_idx [B]."""
        import torch
        idx = np.ascontiguousarray(model_idx, dtype=np.int32)
        p, B, keep = _params_arg(params)
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=f"cuda:{self.device}")
        _check(load().gk_survey_chi2(self._h, idx.ctypes.data, p, B, out.data_ptr(),
                                     _stream_ptr(stream)))
        return out

    def fit_grid(self, lo, hi, free, fixed, n_per_dim=16, max_levels=3, accuracy=None):
        """Nested grids of every galaxy at once (gk_fit_grid_survey): lo, hi, fixed
        [n][12]; n_per_dim one count or 12; returns a list of result dicts."""
        L = load()
        G = len(self.models)
        a = [np.ascontiguousarray(np.broadcast_to(v, (G, NPAR)), dtype=np.float64)
             for v in (lo, hi, fixed)]
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        ns = np.ascontiguousarray(np.broadcast_to(n_per_dim, (NPAR,)), dtype=np.int32)
        acc = None if accuracy is None else np.ascontiguousarray(accuracy, dtype=np.float64)
        res = (GridResult * G)()
        _check(L.gk_fit_grid_survey(self._h, a[0].ctypes.data, a[1].ctypes.data, fm.ctypes.data,
                                    a[2].ctypes.data, ns.ctypes.data, max_levels,
                                    None if acc is None else acc.ctypes.data, res))
        return [_grid_dict(r) for r in res]

    def fit_lm(self, p0, free, lo=None, hi=None, **opts):
        """Levenberg-Marquardt of every galaxy at once (gk_fit_lm_survey)."""
        L = load()
        o = LMOpts()
        _check(L.gk_lm_default_opts(ctypes.byref(o)))
        for k, v in opts.items():
            setattr(o, k, v)
        n = len(self.models)
        p = np.ascontiguousarray(p0, dtype=np.float64).reshape(n, NPAR).copy()
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        lo_a = None if lo is None else np.ascontiguousarray(lo, dtype=np.float64).reshape(n, NPAR)
        hi_a = None if hi is None else np.ascontiguousarray(hi, dtype=np.float64).reshape(n, NPAR)
        res = (LMResult * n)()
        st = L.gk_fit_lm_survey(self._h, p.ctypes.data, fm.ctypes.data,
                                None if lo_a is None else lo_a.ctypes.data,
                                None if hi_a is None else hi_a.ctypes.data, ctypes.byref(o), res)
        if st < 0 and st != GK_ENOTCONV:
            _check(st)
        return {"p": p, "chi2": np.array([r.chi2 for r in res]),
                "iterations": np.array([r.iterations for r in res]),
                "reason": [LM_REASONS.get(r.reason, str(r.reason)) for r in res],
                "n_evals": np.array([r.n_evals for r in res]),
                "errors": np.array([r.errors[:] for r in res]), "status": st}


def gemm_bf16(A, B, trans_a=False, trans_b=False, M=None, N=None, K=None, C=None, stream=None):
    """C [M][N] float32 = sum_k A(m, k) B(n, k) on the surrogate's BF16 GEMM
    (gk_gemm_bf16).  A, B: 2-D bfloat16 CUDA tensors in the stored layout."""
    import torch
    if A.dtype != torch.bfloat16 or B.dtype != torch.bfloat16:
        raise ValueError("A and B must be bfloat16")
    M = M if M is not None else (A.shape[1] if trans_a else A.shape[0])
    K = K if K is not None else (A.shape[0] if trans_a else A.shape[1])
    N = N if N is not None else (B.shape[1] if trans_b else B.shape[0])
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(load().gk_gemm_bf16(int(trans_a), int(trans_b), M, N, K, A.data_ptr(), A.stride(0),
                               B.data_ptr(), B.stride(0), C.data_ptr(), C.stride(0),
                               _stream_ptr(stream)))
    return C


class Surrogate:
    """MLP emulator of the moment maps of one instrument (gk_surrogate_create)."""

    def __init__(self, model: "Model", lo, hi, **opts):
        L = load()
        o = SurrogateOpts()
        _check(L.gk_surrogate_default_opts(ctypes.byref(o)))
        for k, v in opts.items():
            setattr(o, k, v)
        self.opts = o
        self.model = model  # the model must outlive the surrogate
        self.lo = np.ascontiguousarray(lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(hi, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(L.gk_surrogate_create(model._h, self.lo.ctypes.data, self.hi.ctypes.data,
                                     ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.device = model.device
        self.nx, self.ny = model.nx, model.ny

    def save(self, path: str) -> None:
        """Writes options, box, instrument and weights to `path` (gk_surrogate_save)."""
        _check(load().gk_surrogate_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, model: "Model", path: str) -> "Surrogate":
        """A surrogate for `model`'s instrument from a file written by save()."""
        L = load()
        h = ctypes.c_void_p()
        _check(L.gk_surrogate_load(model._h, os.fsencode(path), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.model = model  # the model must outlive the surrogate
        self.device = model.device
        self.nx, self.ny = model.nx, model.ny
        self.opts = None
        self.lo = self.hi = None
        return self

    def close(self):
        if getattr(self, "_h", None):
            load().gk_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train(self, steps: int) -> np.ndarray:
        """Runs `steps` Adam steps; returns each step's loss."""
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        _check(load().gk_surrogate_train(self._h, steps, losses.ctypes.data))
        return losses[:steps]

    def weight_count(self) -> int:
        return int(load().gk_surrogate_weight_count(self._h))

    def get_weights(self) -> np.ndarray:
        w = np.zeros(self.weight_count(), dtype=np.float32)
        _check(load().gk_surrogate_get_weights(self._h, w.ctypes.data, w.size))
        return w

    def set_weights(self, w) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(load().gk_surrogate_set_weights(self._h, w.ctypes.data, w.size))

    def gradients(self, params):
        """(loss, gradient vector) on rows params [B][12] (B a multiple of 32)."""
        p, B, keep = _params_arg(params)
        g = np.zeros(self.weight_count(), dtype=np.float32)
        loss = ctypes.c_double(0.0)
        _check(load().gk_surrogate_gradients(self._h, p, B, g.ctypes.data, ctypes.byref(loss)))
        return loss.value, g

    def step(self, params, lr: float) -> float:
        """One Adam step on rows params [B][12] (gk_surrogate_step); returns the loss
        before the update."""
        p, B, keep = _params_arg(params)
        loss = ctypes.c_double(0.0)
        _check(load().gk_surrogate_step(self._h, p, B, float(lr), ctypes.byref(loss)))
        return loss.value

    def predict(self, params, out=None, stream=None):
        """maps [B][2][ny][nx] float32 CUDA tensor (m1, m2 in km/s)."""
        import torch
        p, B, keep = _params_arg(params)
        if out is None:
            out = torch.empty((B, 2, self.ny, self.nx), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        _check(load().gk_surrogate_predict(self._h, p, B, out.data_ptr(), _stream_ptr(stream)))
        return out

    def chi2(self, model: "Model", params, out=None, stream=None):
        """Surrogate chi2 [B] float64 CUDA tensor against model's observation."""
        import torch
        p, B, keep = _params_arg(params)
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=f"cuda:{self.device}")
        _check(load().gk_surrogate_chi2(self._h, model._h, p, B, out.data_ptr(), _stream_ptr(stream)))
        return out

    def fit_nested(self, model: "Model", lo, hi, free, fixed, margin=25.0, audit=0.0,
                   want_samples=0, **opts) -> dict:
        """Surrogate-screened nested sampling (gk_fit_nested_screened)."""
        L = load()
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        fm = np.ascontiguousarray(free, dtype=np.uint8)
        fx = np.ascontiguousarray(fixed, dtype=np.float64)
        r = NSResult()
        o = _ns_opts(L, **opts)
        buf = np.zeros((max(want_samples, 1), NPAR + 1))
        ns = ctypes.c_int64(0)
        st = L.gk_fit_nested_screened(model._h, self._h, lo.ctypes.data, hi.ctypes.data,
                                      fm.ctypes.data, fx.ctypes.data, ctypes.byref(o), margin,
                                      audit, ctypes.byref(r),
                                      buf.ctypes.data if want_samples else None, want_samples,
                                      ctypes.byref(ns))
        if st < 0 and st != GK_ENOTCONV:
            _check(st)
        return _ns_dict(r, st, NPAR, buf[: ns.value] if want_samples else None)
