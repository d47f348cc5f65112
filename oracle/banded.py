"""Band storage, band LU with partial pivoting and band solves (oracle).

Test infrastructure only.  The arithmetic lives in ``oracle/csrc/band.c``
(plain column-by-column loops); this module converts sparse matrices to band
storage and calls it.  It is the "pre-factorize K_i" step of Alg. composite
(Sec. 3.2) and the solves K_i^{-1} of eq. linearsolve2.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import scipy.sparse as sp

from . import build_oracle

_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_oracle.build())
        _lib.oracle_band_lu.restype = ctypes.c_int
        _lib.oracle_band_lu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p]
        _lib.oracle_band_solve.restype = None
        _lib.oracle_band_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_int64]
    return _lib


def bandwidths(M) -> tuple[int, int]:
    """(kl, ku) of a sparse matrix: largest i-j and j-i over its entries."""
    C = sp.coo_matrix(M)
    if C.nnz == 0:
        return 0, 0
    d = C.row.astype(np.int64) - C.col.astype(np.int64)
    return int(max(d.max(), 0)), int(max((-d).max(), 0))


@dataclasses.dataclass
class BandLU:
    n: int
    kl: int
    ku: int
    ab: np.ndarray      # (2kl+ku+1, n) complex128, Fortran order
    ipiv: np.ndarray    # int32, 0-based
    info: int

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        """Return K^{-1} rhs for a vector or an n x m block."""
        lib = _load()
        vec = rhs.ndim == 1
        X = np.array(rhs.reshape(self.n, -1), dtype=np.complex128, order="F", copy=True)
        lib.oracle_band_solve(self.n, self.kl, self.ku,
                              self.ab.ctypes.data, self.ipiv.ctypes.data,
                              X.shape[1], X.ctypes.data, X.shape[0])
        return X[:, 0] if vec else X


def to_band(M, kl: int, ku: int) -> np.ndarray:
    """Copy a sparse n x n matrix into band storage with kl rows of fill room.

    Entry (i, j) goes to ab[kl + ku + i - j, j]; ldab = 2 kl + ku + 1.
    """
    C = sp.coo_matrix(M)
    n = C.shape[0]
    ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128, order="F")
    np.add.at(ab, (kl + ku + C.row - C.col, C.col), C.data.astype(np.complex128))
    return ab


def band_lu(M, kl: int | None = None, ku: int | None = None) -> BandLU:
    """Band LU with partial pivoting of the sparse matrix M."""
    if kl is None or ku is None:
        kl, ku = bandwidths(M)
    n = M.shape[0]
    ab = to_band(M, kl, ku)
    ipiv = np.zeros(n, dtype=np.int32)
    info = _load().oracle_band_lu(n, kl, ku, ab.ctypes.data, ipiv.ctypes.data)
    return BandLU(n, kl, ku, ab, ipiv, int(info))
