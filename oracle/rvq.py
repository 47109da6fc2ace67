"""ctypes front end of the R-VQ oracle (rvq.c).  Test infrastructure only.

Sec. 3.4 eqs. (14)-(15): L cascaded stages of nearest-code search on the
residual, the reconstruction as the sum of the picked codes, the
codebook loss with the residual under a stop-gradient and its gradient to
the codes.  The nearest-code decision is taken in binary32 (see rvq.c);
loss and gradient are binary64.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB_RVQ):
            _build.build()
        _lib = ctypes.CDLL(_build.LIB_RVQ)
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def rvq(books, x):
    """books (L, P, D) and x (n, D), both taken as binary32.  Returns dict with
    idx (L, n) int32, recon (n, D) float32, loss (float), dbooks (L, P, D) float64."""
    books = np.ascontiguousarray(books, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    L, P, D = books.shape
    n = x.shape[0]
    assert x.shape == (n, D) and 1 <= D <= 64
    idx = np.empty((L, n), np.int32)
    recon = np.empty((n, D), np.float32)
    loss = ctypes.c_double()
    db = np.empty((L, P, D), np.float64)
    lib().orc_rvq(ctypes.c_int64(n), ctypes.c_int(D), ctypes.c_int(L), ctypes.c_int(P), _p(books), _p(x), _p(idx),
                  _p(recon), ctypes.byref(loss), _p(db))
    return dict(idx=idx, recon=recon, loss=loss.value, dbooks=db)
