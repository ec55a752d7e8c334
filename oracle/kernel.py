"""RBF kernel blocks in FP64 for the oracle (test infrastructure only).

The kernel is the one of section 2 of the paper: k(x, z) = exp(-gamma * ||x - z||^2). The squared distance
is summed from explicit coordinate differences, never from the expansion |x|^2 + |z|^2 - 2 x.z.

Two implementations of the same formula: a small C routine (``rbf.c``, built next to this file with gcc and
OpenMP) for speed on large inputs, and a NumPy one used when the C library is not built. Tests check that
they agree.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librbf_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``rbf.c`` into ``librbf_oracle.so`` with gcc (no GPU code involved)."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", os.path.join(_HERE, "rbf.c"),
                               "-o", _LIB_PATH, "-lm"])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None and os.path.exists(_LIB_PATH):
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_rbf_block.restype = None
        lib.oracle_rbf_block.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_double, ctypes.c_void_p]
        _lib = lib
    return _lib


def have_c_kernel() -> bool:
    return _load() is not None


def rbf_block_numpy(X: np.ndarray, Z: np.ndarray, gamma: float, rows_per_chunk: int = 256) -> np.ndarray:
    """out[i, k] = exp(-gamma * sum_t (X[i, t] - Z[k, t])^2) by explicit differences (NumPy)."""
    X = np.asarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    out = np.empty((X.shape[0], Z.shape[0]))
    for lo in range(0, X.shape[0], rows_per_chunk):
        diff = X[lo:lo + rows_per_chunk, None, :] - Z[None, :, :]
        out[lo:lo + rows_per_chunk] = np.exp(-gamma * np.einsum("ikt,ikt->ik", diff, diff))
    return out


def rbf_block(X: np.ndarray, Z: np.ndarray, gamma: float, use_c: bool = True) -> np.ndarray:
    """K[i, k] = k(x_i, z_k) for the RBF kernel of section 2, FP64, explicit differences."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if X.ndim != 2 or Z.ndim != 2 or X.shape[1] != Z.shape[1]:
        raise ValueError("X and Z must be 2-D with the same number of columns")
    lib = _load() if use_c else None
    if lib is None:
        return rbf_block_numpy(X, Z, gamma)
    out = np.empty((X.shape[0], Z.shape[0]))
    if out.size:
        lib.oracle_rbf_block(X.ctypes.data, X.shape[0], X.shape[1], Z.ctypes.data, Z.shape[0], float(gamma),
                             out.ctypes.data)
    return out


def rbf_column(X: np.ndarray, z: np.ndarray, gamma: float) -> np.ndarray:
    """The kernel column k(x_i, z) for every row x_i of X."""
    return rbf_block(X, np.asarray(z, dtype=np.float64).reshape(1, -1), gamma)[:, 0]
