"""FP64 reference oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
shares no code with the GPU path.  The arithmetic lives in ``gabor_oracle.c``
(plain direct sums of Eq. (1) and Eq. (17), double precision); this module only
compiles it with gcc and marshals numpy arrays through ctypes.

Functions:
  gabor_bank(img, omegas, sigmas, thetas, radius_sigmas, boundary)
      -> complex128 [O][N][H][W], Eq. (1)-(2) evaluated directly.
  gabor_bank_points(img, ..., xs, ys) -> complex128 [P][O][N].
  lsdft(img, my, mx, sigma, boundary) -> complex128 [My][Mx][H][W], Eq. (17)-(18).
  lsdft_points(img, my, mx, sigma, boundary, xs, ys) -> complex128 [P][My][Mx].
  gabor_grad_points(img, ..., xs, ys) -> float64 [P], gradient of
      mean |F|^2 over all bank outputs (zero boundary).
  gabor_bank_iir(img, omegas, sigmas, thetas, boundary) -> complex128
      [O][N][H][W], the recursive-smoother variant (modulate, third-order
      recursive Gaussian forward and backward, demodulate), FP64.
  iir_coeffs(sigma) -> (a0, a1, a2, a3) of that recursive Gaussian.
  gaussian_taps(sigma, R) -> float64 [2R+1], the normalised sampled Gaussian.
  radius(sigma, radius_sigmas) -> R = floor(radius_sigmas * sigma + 0.5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gabor_oracle.c")
_LIB = os.path.join(_HERE, "libgabor_oracle.so")

ZERO = 0
MIRROR = 1
_BOUNDARY = {"zero": ZERO, "mirror": MIRROR, ZERO: ZERO, MIRROR: MIRROR}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (OpenMP, no arch tuning)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oracle_radius.argtypes = [f64, f64]
    lib.oracle_radius.restype = ctypes.c_int
    lib.oracle_gaussian_taps.argtypes = [f64, ctypes.c_int, P]
    lib.oracle_gabor_bank.argtypes = [P, i32, i32, i64, i32, P, P, i32, P, f64, i32, P, i32]
    lib.oracle_gabor_bank_points.argtypes = [P, i32, i32, i64, i32, P, P, i32, P, f64, i32,
                                             i64, P, P, P, i32]
    lib.oracle_lsdft.argtypes = [P, i32, i32, i64, i32, i32, f64, i32, P, i32]
    lib.oracle_lsdft_points.argtypes = [P, i32, i32, i64, i32, i32, f64, i32, i64, P, P, P, i32]
    lib.oracle_gabor_grad_points.argtypes = [P, i32, i32, i64, i32, P, P, i32, P, f64,
                                             i64, P, P, P, i32]
    lib.oracle_gabor_bank_iir.argtypes = [P, i32, i32, i64, i32, P, P, i32, P, i32, P, i32]
    lib.oracle_iir_coeffs.argtypes = [f64, P]
    lib.oracle_iir_extension.argtypes = [f64]
    lib.oracle_iir_extension.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _img(img) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(img, dtype=np.float32))
    if a.ndim != 2:
        raise ValueError("image must be 2-D")
    return a


def _params(omegas, sigmas, thetas):
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, dtype=np.float64)))
    sg = np.ascontiguousarray(np.atleast_1d(np.asarray(sigmas, dtype=np.float64)))
    if om.shape != sg.shape:
        raise ValueError("omegas and sigmas must have the same length")
    th = np.ascontiguousarray(np.atleast_1d(np.asarray(thetas, dtype=np.float64)))
    return om, sg, th


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def radius(sigma: float, radius_sigmas: float = 3.0) -> int:
    return int(_load().oracle_radius(float(sigma), float(radius_sigmas)))


def gaussian_taps(sigma: float, R: int) -> np.ndarray:
    out = np.empty(2 * R + 1, dtype=np.float64)
    _check(_load().oracle_gaussian_taps(float(sigma), int(R), _ptr(out)), "taps")
    return out


def gabor_bank(img, omegas, sigmas, thetas, radius_sigmas=3.0, boundary="zero",
               n_threads: int = 0) -> np.ndarray:
    a = _img(img)
    om, sg, th = _params(omegas, sigmas, thetas)
    H, W = a.shape
    out = np.empty((om.size, th.size, H, W, 2), dtype=np.float64)
    rc = _load().oracle_gabor_bank(_ptr(a), H, W, W, om.size, _ptr(om), _ptr(sg), th.size,
                                   _ptr(th), float(radius_sigmas), _BOUNDARY[boundary],
                                   _ptr(out), int(n_threads))
    _check(rc, "gabor_bank")
    return out[..., 0] + 1j * out[..., 1]


def gabor_bank_points(img, omegas, sigmas, thetas, xs, ys, radius_sigmas=3.0,
                      boundary="zero", n_threads: int = 0) -> np.ndarray:
    a = _img(img)
    om, sg, th = _params(omegas, sigmas, thetas)
    H, W = a.shape
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.int32))
    if xs.shape != ys.shape or xs.ndim != 1:
        raise ValueError("xs and ys must be 1-D of equal length")
    out = np.empty((xs.size, om.size, th.size, 2), dtype=np.float64)
    rc = _load().oracle_gabor_bank_points(_ptr(a), H, W, W, om.size, _ptr(om), _ptr(sg),
                                          th.size, _ptr(th), float(radius_sigmas),
                                          _BOUNDARY[boundary], xs.size, _ptr(xs), _ptr(ys),
                                          _ptr(out), int(n_threads))
    _check(rc, "gabor_bank_points")
    return out[..., 0] + 1j * out[..., 1]


def lsdft(img, my: int, mx: int, sigma: float, boundary="zero", n_threads: int = 0):
    a = _img(img)
    H, W = a.shape
    out = np.empty((my, mx, H, W, 2), dtype=np.float64)
    rc = _load().oracle_lsdft(_ptr(a), H, W, W, int(my), int(mx), float(sigma),
                              _BOUNDARY[boundary], _ptr(out), int(n_threads))
    _check(rc, "lsdft")
    return out[..., 0] + 1j * out[..., 1]


def lsdft_points(img, my: int, mx: int, sigma: float, xs, ys, boundary="zero",
                 n_threads: int = 0):
    a = _img(img)
    H, W = a.shape
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.int32))
    out = np.empty((xs.size, my, mx, 2), dtype=np.float64)
    rc = _load().oracle_lsdft_points(_ptr(a), H, W, W, int(my), int(mx), float(sigma),
                                     _BOUNDARY[boundary], xs.size, _ptr(xs), _ptr(ys),
                                     _ptr(out), int(n_threads))
    _check(rc, "lsdft_points")
    return out[..., 0] + 1j * out[..., 1]


def gabor_grad_points(img, omegas, sigmas, thetas, xs, ys, radius_sigmas=3.0,
                      n_threads: int = 0) -> np.ndarray:
    a = _img(img)
    om, sg, th = _params(omegas, sigmas, thetas)
    H, W = a.shape
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int32))
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.int32))
    out = np.empty(xs.size, dtype=np.float64)
    rc = _load().oracle_gabor_grad_points(_ptr(a), H, W, W, om.size, _ptr(om), _ptr(sg),
                                          th.size, _ptr(th), float(radius_sigmas), xs.size,
                                          _ptr(xs), _ptr(ys), _ptr(out), int(n_threads))
    _check(rc, "gabor_grad_points")
    return out


def iir_coeffs(sigma: float):
    """(a0, a1, a2, a3) of the recursive Gaussian: w[n] = a0 u[n] - a1 w[n-1] - ..."""
    a = np.zeros(4)
    _check(_load().oracle_iir_coeffs(float(sigma), _ptr(a)), "iir_coeffs")
    return tuple(float(v) for v in a)


def iir_extension(sigma: float) -> int:
    return int(_load().oracle_iir_extension(float(sigma)))


def gabor_bank_iir(img, omegas, sigmas, thetas, boundary="zero", n_threads: int = 0):
    a = _img(img)
    om, sg, th = _params(omegas, sigmas, thetas)
    H, W = a.shape
    out = np.empty((om.size, th.size, H, W, 2), dtype=np.float64)
    rc = _load().oracle_gabor_bank_iir(_ptr(a), H, W, W, om.size, _ptr(om), _ptr(sg), th.size, _ptr(th),
                                       _BOUNDARY[boundary], _ptr(out), int(n_threads))
    _check(rc, "gabor_bank_iir")
    return out[..., 0] + 1j * out[..., 1]
