"""Seeded, counter-based synthetic input streams (see ``csrc/streams.c``).

Word i of stream ``seed`` is SplitMix64's output function applied to
``key(seed) + (i + 1) * 0x9E3779B97F4A7C15``; bytes and residues are cut from
those words, so every byte range can be regenerated on its own (a 10 GiB
stream is produced block by block).  The C library does the bulk work; the
numpy functions ``*_np`` restate the same definition for cross-checks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from .patterns import AMINO

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwlstreams.so")
_lib: Optional[ctypes.CDLL] = None

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1

# A fixed, synthetic, non-uniform residue frequency vector (integer weights in
# the order of AMINO).  It is made up for these workloads (the paper publishes
# none) and is not taken from any sequence database.
AMINO_WEIGHTS = [3 + (7 * i) % 13 for i in range(len(AMINO))]


def build(force: bool = True) -> str:
    """Compile the stream generator with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "csrc", "streams.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.wl_stream_key.restype = ctypes.c_uint64
        lib.wl_stream_key.argtypes = [ctypes.c_uint64]
        lib.wl_uniform_bytes.restype = None
        lib.wl_uniform_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_void_p]
        lib.wl_residues.restype = None
        lib.wl_residues.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p]
        _lib = lib
    return _lib


def residue_cdf(weights=None) -> np.ndarray:
    w = np.asarray(AMINO_WEIGHTS if weights is None else weights, dtype=np.uint64)
    cum = np.cumsum(w)
    cdf = (cum.astype(object) * (1 << 32)) // int(cum[-1])
    return np.asarray([int(c) for c in cdf], dtype=np.uint64)


def uniform_bytes(seed: int, n: int, first: int = 0, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Bytes ``first .. first+n`` of the uniform stream ``seed``."""
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    assert out.dtype == np.uint8 and out.size >= n and out.flags.c_contiguous
    if n:
        _load().wl_uniform_bytes(seed, first, n, out.ctypes.data)
    return out[:n]


def residues(seed: int, n: int, first: int = 0, letters: str = AMINO, weights=None,
             out: Optional[np.ndarray] = None) -> np.ndarray:
    """Residue letters ``first .. first+n`` of stream ``seed`` (ASCII bytes)."""
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    assert out.dtype == np.uint8 and out.size >= n and out.flags.c_contiguous
    cdf = residue_cdf(weights)
    let = np.frombuffer(letters.encode("ascii"), dtype=np.uint8).copy()
    assert let.size == cdf.size
    if n:
        _load().wl_residues(seed, first, n, cdf.ctypes.data, int(cdf.size), let.ctypes.data,
                            out.ctypes.data)
    return out[:n]


# ---- numpy restatement of the same definition (for cross-checks) ----------
def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _words_np(seed: int, first_word: int, n_words: int) -> np.ndarray:
    key = int(_mix64_np(np.array([(seed + GAMMA) & M64], dtype=np.uint64))[0])
    i = np.arange(first_word, first_word + n_words, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + (i + np.uint64(1)) * np.uint64(GAMMA)
        return _mix64_np(z)


def uniform_bytes_np(seed: int, n: int, first: int = 0) -> np.ndarray:
    w0, w1 = first // 8, (first + n + 7) // 8
    with np.errstate(over="ignore"):
        b = _words_np(seed, w0, w1 - w0).view(np.uint8)
    return b[first - 8 * w0: first - 8 * w0 + n].copy()


def residues_np(seed: int, n: int, first: int = 0, letters: str = AMINO, weights=None) -> np.ndarray:
    w0, w1 = first // 2, (first + n + 1) // 2
    with np.errstate(over="ignore"):
        halves = _words_np(seed, w0, w1 - w0).view(np.uint32).astype(np.uint64)
    u = halves[first - 2 * w0: first - 2 * w0 + n]
    cdf = residue_cdf(weights)
    r = np.searchsorted(cdf, u, side="right")
    let = np.frombuffer(letters.encode("ascii"), dtype=np.uint8)
    return let[np.minimum(r, cdf.size - 1)]
