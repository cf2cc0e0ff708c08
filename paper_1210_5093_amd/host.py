"""ctypes binding of libdfahost.so, the host multicore speculative matcher.

Argument marshalling only: the partition, the per-chunk set walks and the
merge all run in the C++ library.  This is a CPU yardstick beside the GPU
library, not a fallback for it."""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB_PATH = os.path.join(HERE, "libdfahost.so")
DFA_E_SYMBOL = -4

_lib = None


class HostError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what}: status {rc}")
        self.rc = rc


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(HOST_LIB_PATH):
        raise RuntimeError(f"{HOST_LIB_PATH} is not built (run paper_1210_5093_amd/build.py)")
    L = ctypes.CDLL(HOST_LIB_PATH)
    P, I, U32, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
    D = ctypes.POINTER(ctypes.c_double)
    L.dfa_host_create.restype = I
    L.dfa_host_create.argtypes = [P, U32, U32, U32, P, U32, P, ctypes.POINTER(P)]
    L.dfa_host_destroy.restype = None
    L.dfa_host_destroy.argtypes = [P]
    L.dfa_host_imax.restype = U32
    L.dfa_host_imax.argtypes = [P]
    L.dfa_host_partition.restype = I
    L.dfa_host_partition.argtypes = [U64, ctypes.c_double, D, U32, ctypes.POINTER(U64)]
    L.dfa_host_profile.restype = I
    L.dfa_host_profile.argtypes = [P, P, ctypes.c_size_t, U32, D]
    L.dfa_host_match.restype = I
    L.dfa_host_match.argtypes = [P, P, ctypes.c_size_t, U32, D, U32, ctypes.POINTER(U32),
                                 ctypes.POINTER(I)]
    _lib = L
    return L


def _doubles(xs: Optional[Sequence[float]]):
    if xs is None:
        return None
    return (ctypes.c_double * len(xs))(*[float(x) for x in xs])


class HostDFA:
    """A DFA copied into the host matcher."""

    def __init__(self, delta: np.ndarray, q0: int, accepting: Sequence[int],
                 byte_to_symbol: Optional[np.ndarray] = None):
        d = np.ascontiguousarray(delta, dtype=np.uint32)
        acc = np.ascontiguousarray(np.asarray(list(accepting), dtype=np.uint32))
        bmap = None if byte_to_symbol is None else \
            np.ascontiguousarray(byte_to_symbol, dtype=np.uint8)
        h = ctypes.c_void_p()
        rc = lib().dfa_host_create(d.ctypes.data, d.shape[0], d.shape[1], int(q0),
                                   acc.ctypes.data if acc.size else None, acc.size,
                                   bmap.ctypes.data if bmap is not None else None,
                                   ctypes.byref(h))
        if rc:
            raise HostError(rc, "dfa_host_create")
        self._h = h

    @classmethod
    def from_workload(cls, w) -> "HostDFA":
        return cls(w.delta, w.q0, w.accepting, w.byte_to_symbol)

    @property
    def imax(self) -> int:
        return int(lib().dfa_host_imax(self._h))

    def profile(self, sample: np.ndarray, threads: int) -> List[float]:
        x = np.ascontiguousarray(sample, dtype=np.uint8)
        out = (ctypes.c_double * threads)()
        rc = lib().dfa_host_profile(self._h, x.ctypes.data if x.size else None, x.size, threads,
                                    out)
        if rc:
            raise HostError(rc, "dfa_host_profile")
        return list(out)

    def match(self, x: np.ndarray, threads: int = 0, capacities=None,
              start: Optional[int] = None) -> Tuple[int, bool]:
        x = np.ascontiguousarray(x, dtype=np.uint8)
        fin, acc = ctypes.c_uint32(), ctypes.c_int()
        rc = lib().dfa_host_match(self._h, x.ctypes.data if x.size else None, x.size, threads,
                                  _doubles(capacities), 0xFFFFFFFF if start is None else start,
                                  ctypes.byref(fin), ctypes.byref(acc))
        if rc:
            raise HostError(rc, "dfa_host_match")
        return int(fin.value), bool(acc.value)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().dfa_host_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def partition(n: int, m: float, P: int, capacities=None) -> List[int]:
    """Half-open chunk boundaries (P + 1 values) of Eqs. (1)-(7)/(10)."""
    out = (ctypes.c_uint64 * (P + 1))()
    rc = lib().dfa_host_partition(int(n), float(m), _doubles(capacities), int(P), out)
    if rc:
        raise HostError(rc, "dfa_host_partition")
    return [int(v) for v in out]
