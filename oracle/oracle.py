"""ctypes binding of the FP64 CPU oracle (gk_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports
it.  Nothing here is shared with the GPU library: the descriptor struct and
every signature are declared independently.

Each function follows a step of the paper's evaluation (Bekiaris et al. 2016):
model cube (Sec. 2.1, eqs. 1-8; Sec. 2.2.2), PSF/LSF convolution (eq. 9,
Sec. 2.2.3), down-sampling (Sec. 2.2.4), moments (Sec. 2.2.5), chi-square
(eq. 11, Sec. 2.2.6); the velocity-field strategy (Sec. 2.2.1) evaluates eq. 8
per data pixel and skips the cube, convolution and moment steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gk_oracle.c")
# GK_ORACLE_LIB lets the mutation test load a deliberately broken copy.
LIB = os.environ.get("GK_ORACLE_LIB") or os.path.join(HERE, "libgk_oracle.so")

RC_ARCTAN, RC_EPINAT, RC_BOISSIER = 0, 1, 2
NPAR = 12


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (plain C, no intrinsics)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("u", ctypes.c_int32), ("dv", ctypes.c_double), ("v0", ctypes.c_double),
                ("crpix", ctypes.c_double), ("psf_fwhm", ctypes.c_double),
                ("lsf_sigma", ctypes.c_double), ("R", ctypes.c_double),
                ("rc", ctypes.c_int32), ("pad_", ctypes.c_int32)]


@dataclass
class Desc:
    """Observation/model grid: data size, upsampling, channel grid, PSF/LSF."""
    nx: int
    ny: int
    nz: int
    u: int = 1
    dv: float = 30.0
    v0: float = 0.0
    crpix: float | None = None      # default nz/2
    psf_fwhm: float = 0.0           # data pixels
    lsf_sigma: float = 0.0          # km/s
    R: float = 4.0
    rc: int = RC_ARCTAN

    def c(self) -> _Desc:
        crpix = self.nz / 2.0 if self.crpix is None else self.crpix
        return _Desc(self.nx, self.ny, self.nz, self.u, self.dv, self.v0, crpix,
                     self.psf_fwhm, self.lsf_sigma, self.R, self.rc, 0)

    def velocities(self) -> np.ndarray:
        crpix = self.nz / 2.0 if self.crpix is None else self.crpix
        return self.v0 + (np.arange(self.nz) - crpix) * self.dv


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        D, I, P = ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(_Desc)
        L.go_kernel_taps.argtypes = [ctypes.c_double, ctypes.c_double, D, I]
        L.go_kernel_taps.restype = I
        L.go_cube_dims.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.go_params_valid.argtypes = [P, D]
        L.go_vrot.argtypes = [I, ctypes.c_double, D]
        L.go_vrot.restype = ctypes.c_double
        L.go_sky_point.argtypes = [I, D, ctypes.c_double, ctypes.c_double, D, D]
        L.go_model_cube.argtypes = [P, D, D]
        L.go_convolve3.argtypes = [D, I, I, I, D, I, D, I, D, I, D]
        L.go_downsample.argtypes = [D, I, I, I, I, D]
        L.go_moments.argtypes = [D, I, I, I, D, ctypes.c_double, ctypes.c_double, D, D, D]
        L.go_evaluate.argtypes = [P, D, D]
        U8 = ctypes.POINTER(ctypes.c_uint8)
        L.go_chi2.argtypes = [I, D, D, D, D, D, D, U8, ctypes.c_double, D,
                              ctypes.POINTER(ctypes.c_int64)]
        L.go_eval_chi2.argtypes = [P, D, D, D, D, D, U8, ctypes.c_double, D,
                                   ctypes.POINTER(ctypes.c_int64)]
        L.go_vfield.argtypes = [P, D, D]
        L.go_vfield_chi2.argtypes = [P, D, D, D, D, D, U8, ctypes.c_double, D,
                                     ctypes.POINTER(ctypes.c_int64)]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def kernel_taps(sigma: float, R: float = 4.0) -> np.ndarray:
    buf = np.zeros(4097)
    h = lib().go_kernel_taps(sigma, R, _ptr(buf), buf.size)
    if h < 0:
        raise ValueError("kernel too wide")
    return buf[: 2 * h + 1].copy()


def cube_dims(d: Desc):
    dims = (ctypes.c_int32 * 5)()
    lib().go_cube_dims(ctypes.byref(d.c()), dims)
    return tuple(dims)  # nxe, nye, nze, hp, hl


def params_valid(d: Desc, p) -> bool:
    p = _f64(p)
    return bool(lib().go_params_valid(ctypes.byref(d.c()), _ptr(p)))


def vrot(rc: int, r: float, p) -> float:
    p = _f64(p)
    return lib().go_vrot(rc, r, _ptr(p))


def sky_point(rc: int, p, x: float, y: float):
    p = _f64(p)
    v, i = ctypes.c_double(), ctypes.c_double()
    lib().go_sky_point(rc, _ptr(p), x, y, ctypes.byref(v), ctypes.byref(i))
    return v.value, i.value


def model_cube(d: Desc, p) -> np.ndarray:
    nxe, nye, nze, _, _ = cube_dims(d)
    out = np.zeros((nze, nye, nxe))
    p = _f64(p)
    if lib().go_model_cube(ctypes.byref(d.c()), _ptr(p), _ptr(out)) != 0:
        raise ValueError("parameters outside the model domain")
    return out


def convolve3(cube, kz, ky, kx) -> np.ndarray:
    cube, kz, ky, kx = _f64(cube), _f64(kz), _f64(ky), _f64(kx)
    nze, nye, nxe = cube.shape
    hz, hy, hx = (len(kz) - 1) // 2, (len(ky) - 1) // 2, (len(kx) - 1) // 2
    out = np.zeros((nze - 2 * hz, nye - 2 * hy, nxe - 2 * hx))
    rc = lib().go_convolve3(_ptr(cube), nze, nye, nxe, _ptr(kz), hz, _ptr(ky), hy,
                            _ptr(kx), hx, _ptr(out))
    if rc != 0:
        raise ValueError("convolve3 failed")
    return out


def downsample(cube, u: int) -> np.ndarray:
    cube = _f64(cube)
    NZ, NY, NX = cube.shape
    out = np.zeros((NZ // u, NY // u, NX // u))
    lib().go_downsample(_ptr(cube), NZ // u, NY // u, NX // u, u, _ptr(out))
    return out


def moments(cube, vel, dv: float, vsys: float = 0.0):
    cube, vel = _f64(cube), _f64(vel)
    nz, ny, nx = cube.shape
    m = np.zeros((3, ny, nx))
    lib().go_moments(_ptr(cube), nz, ny, nx, _ptr(vel), dv, vsys,
                     _ptr(m[0]), _ptr(m[1]), _ptr(m[2]))
    return m


def evaluate(d: Desc, p) -> np.ndarray:
    """maps[3][ny][nx] = (m0, m1, m2); NaN maps for out-of-domain parameters."""
    out = np.zeros((3, d.ny, d.nx))
    p = _f64(p)
    rc = lib().go_evaluate(ctypes.byref(d.c()), _ptr(p), _ptr(out))
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    return out


def chi2(m1, m2, vo, so, ev, es, mask, W: float):
    m1, m2, vo, so, ev, es = (_f64(a).ravel() for a in (m1, m2, vo, so, ev, es))
    mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    c, n = ctypes.c_double(), ctypes.c_int64()
    lib().go_chi2(m1.size, _ptr(m1), _ptr(m2), _ptr(vo), _ptr(so), _ptr(ev), _ptr(es),
                  mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), W,
                  ctypes.byref(c), ctypes.byref(n))
    return c.value, n.value


def eval_chi2(d: Desc, p, vo, so, ev, es, mask, W: float):
    """(chi2, n_valid) of one parameter vector; chi2 = +inf out of domain."""
    vo, so, ev, es = (_f64(a).ravel() for a in (vo, so, ev, es))
    mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    p = _f64(p)
    c, n = ctypes.c_double(), ctypes.c_int64()
    rc = lib().go_eval_chi2(ctypes.byref(d.c()), _ptr(p), _ptr(vo), _ptr(so), _ptr(ev),
                            _ptr(es), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            W, ctypes.byref(c), ctypes.byref(n))
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    return c.value, n.value


def vfield(d: Desc, p) -> np.ndarray:
    """Velocity-field strategy (Sec. 2.2.1): maps[3][ny][nx] = (surface
    brightness, eq. 8 velocity, sigma) at the data pixel centres; NaN maps for
    out-of-domain parameters.  Only nx, ny and rc of the descriptor are used."""
    out = np.zeros((3, d.ny, d.nx))
    p = _f64(p)
    lib().go_vfield(ctypes.byref(d.c()), _ptr(p), _ptr(out))
    return out


def vfield_chi2(d: Desc, p, vo, so, ev, es, mask, W: float):
    """(chi2, n_valid) of the velocity-field strategy; chi2 = +inf out of domain."""
    vo, so, ev, es = (_f64(a).ravel() for a in (vo, so, ev, es))
    mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    p = _f64(p)
    c, n = ctypes.c_double(), ctypes.c_int64()
    rc = lib().go_vfield_chi2(ctypes.byref(d.c()), _ptr(p), _ptr(vo), _ptr(so), _ptr(ev),
                              _ptr(es), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                              W, ctypes.byref(c), ctypes.byref(n))
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    return c.value, n.value
