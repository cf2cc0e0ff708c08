"""ORACLE -- test infrastructure only.

Plain CPU statement of the DFA membership test of Ko, Jung, Han, Burgstaller
(arXiv 1210.5093).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the GPU library (``paper_1210_5093_amd``) and imports nothing from it.

Bulk work goes through ``oracle.c`` (compiled with gcc, its own translation
unit); the ``*_py`` functions restate the same definitions in pure Python for
tiny inputs.  Sources:

* ``walk`` / ``walk_py``: Algorithm 1 and delta* (Section 2.1).  The result is
  the plain definition final = delta*(q0, w), accept = final in F.
* ``absorbing``: the error/sink state q_e (Section 2.1), read as every state
  with a self-loop on all symbols.
* ``isets`` / ``isets_py``: Eq. (11) and the first loop of Algorithm 3.
* ``iset_word``: Eq. (13) (multi-symbol reverse lookahead).
* ``chunk_map``: the state-map vector L_i (Section 4.1).
* ``compose``: the map combination of Eq. (9).
* ``partition``: Eqs. (1), (5)-(7) and (10) (processor weights and chunk
  ranges), in pure Python.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib: Optional[ctypes.CDLL] = None

OK, BAD_SYMBOL, BAD_ARG = 0, 1, -1


class InvalidSymbol(ValueError):
    def __init__(self, index: int):
        super().__init__(f"byte at position {index} is not in the alphabet")
        self.index = index


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_walk.restype = ctypes.c_int
        lib.oracle_walk.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, ctypes.c_uint32,
                                    P, ctypes.c_uint64, P, ctypes.c_uint64, P, P, P]
        lib.oracle_accepts.restype = ctypes.c_int
        lib.oracle_accepts.argtypes = [ctypes.c_uint32, P, ctypes.c_uint32]
        lib.oracle_absorbing.restype = None
        lib.oracle_absorbing.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.oracle_isets.restype = None
        lib.oracle_isets.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, P]
        lib.oracle_iset_word.restype = None
        lib.oracle_iset_word.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, P,
                                         ctypes.c_uint32, P]
        lib.oracle_chunk_map.restype = ctypes.c_int
        lib.oracle_chunk_map.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, P,
                                         ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_uint32, P]
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


# ---------------------------------------------------------------------------
# Algorithm 1: sequential walk
# ---------------------------------------------------------------------------
def walk(delta, byte_to_symbol, start: int, w, probes: Optional[Sequence[int]] = None
         ) -> Tuple[int, Optional[np.ndarray]]:
    """Return (delta*(start, w), prefix states at ``probes``) via oracle.c.

    ``probes`` must be ascending positions in [0, len(w)]; the prefix state at
    p is delta*(start, w[0:p]).  Raises ``InvalidSymbol`` for a byte outside
    Sigma."""
    d = _u32(delta)
    nq, nsym = d.shape
    b2s = _u8(byte_to_symbol)
    assert b2s.size == 256
    wa = _u8(w)
    pr = None if probes is None else np.ascontiguousarray(probes, dtype=np.uint64)
    ps = None if pr is None else np.zeros(pr.size, dtype=np.uint32)
    fin = np.zeros(1, dtype=np.uint32)
    bad = np.zeros(1, dtype=np.uint64)
    rc = _load().oracle_walk(d.ctypes.data, nq, nsym, b2s.ctypes.data, int(start),
                             wa.ctypes.data if wa.size else None, int(wa.size),
                             pr.ctypes.data if pr is not None else None,
                             0 if pr is None else int(pr.size),
                             ps.ctypes.data if ps is not None else None,
                             fin.ctypes.data, bad.ctypes.data)
    if rc == BAD_SYMBOL:
        raise InvalidSymbol(int(bad[0]))
    if rc != OK:
        raise ValueError("oracle_walk: bad arguments")
    return int(fin[0]), ps


def accepts(final_state: int, accepting) -> bool:
    acc = _u32(accepting)
    return bool(_load().oracle_accepts(int(final_state), acc.ctypes.data if acc.size else None,
                                       int(acc.size)))


def membership(delta, byte_to_symbol, q0: int, accepting, w) -> Tuple[int, bool]:
    """Algorithm 1 end to end: (final state, w in L(A))."""
    fin, _ = walk(delta, byte_to_symbol, q0, w)
    return fin, accepts(fin, accepting)


def walk_py(delta, byte_to_symbol, start: int, w) -> int:
    """Pure-Python Algorithm 1 for tiny inputs."""
    state = int(start)
    for byte in bytes(w):
        a = int(byte_to_symbol[byte])
        if a >= len(delta[0]):
            raise InvalidSymbol(-1)
        state = int(delta[state][a])
    return state


# ---------------------------------------------------------------------------
# Error / sink states and initial-state sets
# ---------------------------------------------------------------------------
def absorbing(delta) -> np.ndarray:
    d = _u32(delta)
    nq, nsym = d.shape
    m = np.zeros(nq, dtype=np.uint8)
    _load().oracle_absorbing(d.ctypes.data, nq, nsym, m.ctypes.data)
    return m.astype(bool)


def isets(delta, excluded=None) -> np.ndarray:
    """bool [nsym][Q]: row a is I_a = {delta(x, a) : x in Q} minus excluded."""
    d = _u32(delta)
    nq, nsym = d.shape
    ex = None if excluded is None else _u8(np.asarray(excluded, dtype=bool))
    out = np.zeros((nsym, nq), dtype=np.uint8)
    _load().oracle_isets(d.ctypes.data, nq, nsym, ex.ctypes.data if ex is not None else None,
                         out.ctypes.data)
    return out.astype(bool)


def isets_py(delta, excluded=()) -> List[set]:
    nq, nsym = len(delta), len(delta[0])
    ex = set(excluded)
    return [{int(delta[x][a]) for x in range(nq)} - ex for a in range(nsym)]


def imax(delta, excluded=None) -> int:
    """Eq. (12): the largest |I_a| over the alphabet."""
    return int(isets(delta, excluded).sum(axis=1).max())


def iset_word(delta, symbols: Sequence[int], excluded=None) -> np.ndarray:
    """Eq. (13): bool [Q], I_{sigma_1..sigma_k} for the symbols in matching order."""
    d = _u32(delta)
    nq, nsym = d.shape
    ex = None if excluded is None else _u8(np.asarray(excluded, dtype=bool))
    sy = _u32(symbols)
    out = np.zeros(nq, dtype=np.uint8)
    _load().oracle_iset_word(d.ctypes.data, nq, nsym, ex.ctypes.data if ex is not None else None,
                             sy.ctypes.data if sy.size else None, int(sy.size), out.ctypes.data)
    return out.astype(bool)


def imax_r(delta, r: int, excluded=None) -> int:
    """I_max,r: the largest |I_{sigma_1..sigma_r}| over all r-symbol strings."""
    d = _u32(delta)
    nsym = d.shape[1]
    best = 0
    for idx in range(nsym ** r):
        syms, v = [], idx
        for _ in range(r):
            syms.append(v % nsym)
            v //= nsym
        best = max(best, int(iset_word(d, syms[::-1], excluded).sum()))
    return best


# ---------------------------------------------------------------------------
# State maps and their combination
# ---------------------------------------------------------------------------
def chunk_map(delta, byte_to_symbol, w, begin: int, end: int, starts) -> np.ndarray:
    """L[j] = delta*(starts[j], w[begin:end]) (state-map vector, Section 4.1)."""
    d = _u32(delta)
    nq, nsym = d.shape
    b2s = _u8(byte_to_symbol)
    wa = _u8(w)
    st = _u32(starts)
    out = np.zeros(st.size, dtype=np.uint32)
    rc = _load().oracle_chunk_map(d.ctypes.data, nq, nsym, b2s.ctypes.data,
                                  wa.ctypes.data if wa.size else None, int(begin), int(end),
                                  st.ctypes.data if st.size else None, int(st.size),
                                  out.ctypes.data)
    if rc == BAD_SYMBOL:
        raise InvalidSymbol(-1)
    if rc != OK:
        raise ValueError("oracle_chunk_map: bad arguments")
    return out


def compose(Li: Sequence[int], Lj: Sequence[int]) -> List[int]:
    """Eq. (9): L_{i,j}[k] = L_j[L_i[k]] for full maps over Q."""
    return [int(Lj[int(v)]) for v in Li]


def sequential_merge(maps: Sequence[Sequence[int]], start_index: int = 0) -> int:
    """Eq. (8): L_{P-1}[ ... L_1[L_0[start_index]] ... ] for full maps over Q."""
    s = int(start_index)
    for L in maps:
        s = int(L[s])
    return s


# ---------------------------------------------------------------------------
# Processor weights and input partition (Eqs. 1, 5-7, 10)
# ---------------------------------------------------------------------------
def weights(capacities: Sequence[float]) -> List[float]:
    """Eq. (1): w_k = m_k / mean(m)."""
    mean = sum(capacities) / len(capacities)
    return [m / mean for m in capacities]


def first_chunk_length(n: int, m: float, w: Sequence[float]) -> float:
    """Eq. (5) (m = |Q|) or Eq. (10) (m = I_max): L_0 = n m / (w_0 m + sum_{i>=1} w_i)."""
    return n * m / (w[0] * m + sum(w[1:]))


def partition(n: int, m: float, w: Sequence[float]) -> List[Tuple[int, int]]:
    """Eqs. (6)-(7): inclusive (StartPos, EndPos) per processor, with floors."""
    P = len(w)
    L0 = first_chunk_length(n, m, w)
    out = []
    for k in range(P):
        if k == 0:
            start = 0
        else:
            start = math.floor(L0 * w[0] + sum(L0 * w[i] for i in range(1, k)) / m)
        if k == P - 1:
            end = n - 1
        else:
            end = math.floor(L0 * w[0] + sum(L0 * w[i] for i in range(1, k + 1)) / m) - 1
        out.append((start, end))
    return out


# ---------------------------------------------------------------------------
# Timing helper for the CPU baseline
# ---------------------------------------------------------------------------
def time_walk(delta, byte_to_symbol, start: int, w, repeats: int = 1) -> Tuple[float, int]:
    """Wall time (s) of the fastest of ``repeats`` walks over ``w``, and the final state."""
    best, fin = float("inf"), -1
    for _ in range(repeats):
        t0 = time.perf_counter()
        fin, _ = walk(delta, byte_to_symbol, start, w)
        best = min(best, time.perf_counter() - t0)
    return best, fin
