"""CPU oracle for P-HGRMS (Section 2 of the paper: Algorithms 1 and 2 and the
pass loop), as a plain single-threaded C library behind ctypes.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product package never imports this
module, and this module imports nothing from the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "phgrms_oracle.c")
_LIB = os.path.join(_HERE, "libphgrms_oracle.so")


def compile_oracle(src: str, out: str) -> str:
    """gcc -O2, single-threaded, no OpenMP, no intrinsics."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
         "-I", _HERE, "-o", tmp, src])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        compile_oracle(SOURCE, _LIB)
    return _LIB


def _u8(img: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(img)
    if a.dtype != np.uint8 or a.ndim != 2:
        raise ValueError("oracle images are 2-D uint8 arrays")
    return a


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Oracle:
    """ctypes front end of one build of the oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32 = ctypes.c_int32
        lib.phgrms_oracle_cardinality.argtypes = [
            u8p, i32, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_uint16)]
        lib.phgrms_oracle_cardinality.restype = ctypes.c_int
        lib.phgrms_oracle_pass.argtypes = [u8p, u8p, i32, i32, i32, i32]
        lib.phgrms_oracle_pass.restype = ctypes.c_int64
        lib.phgrms_oracle_denoise.argtypes = [
            u8p, u8p, i32, i32, i32, i32, i32,
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
        lib.phgrms_oracle_denoise.restype = ctypes.c_int
        lib.phgrms_oracle_denoise_cycle.argtypes = [
            u8p, u8p, i32, i32, i32, i32, i32,
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
        lib.phgrms_oracle_denoise_cycle.restype = ctypes.c_int
        lib.phgrms_oracle_isqrt.argtypes = [ctypes.c_uint32]
        lib.phgrms_oracle_isqrt.restype = ctypes.c_uint32
        lib.phgrms_oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_int64,
                                                 ctypes.POINTER(ctypes.c_uint64)]
        lib.phgrms_oracle_splitmix64.restype = None
        lib.phgrms_oracle_salt_pepper.argtypes = [u8p, u8p, ctypes.c_int64, ctypes.c_uint64,
                                                  ctypes.c_uint32, ctypes.c_uint32]
        lib.phgrms_oracle_salt_pepper.restype = ctypes.c_int
        lib.phgrms_oracle_sq_diff_sum.argtypes = [u8p, u8p, ctypes.c_int64]
        lib.phgrms_oracle_sq_diff_sum.restype = ctypes.c_int64
        self.lib = lib
        self.path = path

    def isqrt(self, q: int) -> int:
        return int(self.lib.phgrms_oracle_isqrt(ctypes.c_uint32(q)))

    def cardinality(self, img: np.ndarray, alpha: int, beta: int,
                    scatter: bool = True) -> np.ndarray:
        """Algorithm 1: the cardinality matrix C of one image (uint16)."""
        a = _u8(img)
        rows, cols = a.shape
        card = np.zeros((rows, cols), dtype=np.uint16)
        rc = self.lib.phgrms_oracle_cardinality(
            _ptr(a, ctypes.c_uint8), rows, cols, alpha, beta,
            1 if scatter else 0, _ptr(card, ctypes.c_uint16))
        if rc != 0:
            raise ValueError("invalid oracle arguments")
        return card

    def one_pass(self, img: np.ndarray, alpha: int, beta: int):
        """One pass (Algorithm 1 then Algorithm 2): (image, changed)."""
        a = _u8(img)
        rows, cols = a.shape
        out = np.empty_like(a)
        ch = self.lib.phgrms_oracle_pass(
            _ptr(a, ctypes.c_uint8), _ptr(out, ctypes.c_uint8), rows, cols,
            alpha, beta)
        if ch < 0:
            raise ValueError("invalid oracle arguments")
        return out, int(ch)

    def denoise(self, img: np.ndarray, alpha: int, beta: int, k: int):
        """The full pass loop: (image, iterations, changed list)."""
        a = _u8(img)
        rows, cols = a.shape
        out = np.empty_like(a)
        changed = np.zeros(max(k, 1), dtype=np.int64)
        it = ctypes.c_int32(0)
        rc = self.lib.phgrms_oracle_denoise(
            _ptr(a, ctypes.c_uint8), _ptr(out, ctypes.c_uint8), rows, cols,
            alpha, beta, k, _ptr(changed, ctypes.c_int64), ctypes.byref(it))
        if rc != 0:
            raise ValueError("invalid oracle arguments")
        n = it.value
        return out, n, [int(v) for v in changed[:n]]

    def denoise_cycle(self, img: np.ndarray, alpha: int, beta: int, k: int):
        """The pass loop with the opt-in period-2 stop: (image, iterations,
        changed list)."""
        a = _u8(img)
        rows, cols = a.shape
        out = np.empty_like(a)
        changed = np.zeros(max(k, 1), dtype=np.int64)
        it = ctypes.c_int32(0)
        rc = self.lib.phgrms_oracle_denoise_cycle(
            _ptr(a, ctypes.c_uint8), _ptr(out, ctypes.c_uint8), rows, cols,
            alpha, beta, k, _ptr(changed, ctypes.c_int64), ctypes.byref(it))
        if rc != 0:
            raise ValueError("invalid oracle arguments")
        n = it.value
        return out, n, [int(v) for v in changed[:n]]

    def denoise_window(self, img: np.ndarray, alpha: int, beta: int, k: int,
                       r: int, c: int) -> int:
        """Output pixel (r, c) of denoise(img, alpha, beta, k), computed on a
        crop.

        A pass changes a pixel using only its beta-window, so after t passes
        a pixel depends only on the input within Chebyshev radius t*beta.
        The crop of radius k*beta around (r, c), clipped to the image, run for
        k passes without early stop, therefore yields the value at (r, c) of
        k unconditional passes over the whole image.  That equals the
        method's output: once a pass changes nothing, the image is a fixed
        point and later passes are no-ops.  Crop borders that coincide with
        image borders are real borders; the others are k*beta away from
        (r, c), and the error they cause moves inward beta per pass."""
        a = _u8(img)
        rows, cols = a.shape
        rad = k * beta
        r0, r1 = max(0, r - rad), min(rows, r + rad + 1)
        c0, c1 = max(0, c - rad), min(cols, c + rad + 1)
        out = np.ascontiguousarray(a[r0:r1, c0:c1])
        for _ in range(k):
            out, _ch = self.one_pass(out, alpha, beta)
        return int(out[r - r0, c - c0])


    # ---- noise and quality measure of the experiments (Section 3) -------

    def splitmix64(self, seed: int, n: int) -> list:
        """The first n outputs of SplitMix64 seeded with `seed`."""
        out = (ctypes.c_uint64 * max(n, 1))()
        self.lib.phgrms_oracle_splitmix64(ctypes.c_uint64(seed), n, out)
        return [int(out[i]) for i in range(n)]

    def salt_pepper(self, img: np.ndarray, seed: int, t_pepper: int, t_salt: int) -> np.ndarray:
        """Salt-and-pepper noise with the given 32-bit thresholds."""
        a = _u8(img)
        out = np.empty_like(a)
        rc = self.lib.phgrms_oracle_salt_pepper(
            _ptr(a, ctypes.c_uint8), _ptr(out, ctypes.c_uint8), a.size,
            ctypes.c_uint64(seed), ctypes.c_uint32(t_pepper), ctypes.c_uint32(t_salt))
        if rc != 0:
            raise ValueError("invalid oracle arguments")
        return out

    def sq_diff_sum(self, a: np.ndarray, b: np.ndarray) -> int:
        """Sum of squared differences of two equal-shape uint8 images."""
        x, y = _u8(a), _u8(b)
        if x.shape != y.shape:
            raise ValueError("shapes differ")
        return int(self.lib.phgrms_oracle_sq_diff_sum(
            _ptr(x, ctypes.c_uint8), _ptr(y, ctypes.c_uint8), x.size))


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _default = Oracle(_LIB)
    return _default


def isqrt(q: int) -> int:
    return get().isqrt(q)


def cardinality(img, alpha, beta, scatter=True):
    return get().cardinality(img, alpha, beta, scatter)


def one_pass(img, alpha, beta):
    return get().one_pass(img, alpha, beta)


def denoise(img, alpha, beta, k):
    return get().denoise(img, alpha, beta, k)


def denoise_window(img, alpha, beta, k, r, c):
    return get().denoise_window(img, alpha, beta, k, r, c)


def denoise_cycle(img, alpha, beta, k):
    return get().denoise_cycle(img, alpha, beta, k)


def splitmix64(seed, n):
    return get().splitmix64(seed, n)


def salt_pepper(img, seed, t_pepper, t_salt):
    return get().salt_pepper(img, seed, t_pepper, t_salt)


def sq_diff_sum(a, b):
    return get().sq_diff_sum(a, b)
