"""Seeded synthetic DFAs shaped like the paper's workloads.

A DFA here is the tuple (Q, Sigma, delta, q0, F) of the paper's background
section, given as a complete table ``delta[q][a]`` (uint32, caller numbering),
plus a 256-entry ``byte_to_symbol`` map from input bytes to symbol indices
(an entry >= |Sigma| marks a byte not in Sigma; 0xFF is used for that).  These are inputs for both the oracle and the GPU
library; nothing here evaluates the membership test.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class DFA:
    delta: np.ndarray            # uint32 [Q][nsym]
    q0: int
    accepting: np.ndarray        # uint32 state ids
    byte_to_symbol: np.ndarray   # uint8 [256]; 0xFF = not in Sigma
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_states(self) -> int:
        return int(self.delta.shape[0])

    @property
    def num_symbols(self) -> int:
        return int(self.delta.shape[1])

    def accept_mask(self) -> np.ndarray:
        m = np.zeros(self.num_states, dtype=bool)
        m[self.accepting] = True
        return m


def identity_byte_map() -> np.ndarray:
    return np.arange(256, dtype=np.uint8)


def random_dfa(seed: int, num_states: int = 16, num_symbols: int = 256, num_accepting: int = 4,
               name: str = "") -> DFA:
    """Uniformly random complete DFA: delta = rng.integers(0, Q, (Q, nsym)),
    F = rng.choice(Q, |F|, replace=False), q0 = 0, rng = default_rng(seed)."""
    rng = np.random.default_rng(seed)
    delta = rng.integers(0, num_states, (num_states, num_symbols)).astype(np.uint32)
    acc = np.sort(rng.choice(num_states, num_accepting, replace=False)).astype(np.uint32)
    if num_symbols == 256:
        b2s = identity_byte_map()
    else:
        b2s = np.full(256, 0xFF, dtype=np.uint8)
        b2s[:num_symbols] = np.arange(num_symbols, dtype=np.uint8)
    return DFA(delta, 0, acc, b2s, name or f"random{num_states}x{num_symbols}s{seed}",
               {"seed": seed})


def column_dfa(col_seed: int, map_seed: int, num_states: int = 512, num_columns: int = 64,
               accept_fraction: float = 0.125, name: str = "") -> DFA:
    """Byte-alphabet DFA whose 256 delta-columns are drawn from ``num_columns``
    distinct random columns: columns = default_rng(col_seed).integers(0, Q,
    (num_columns, Q)); the byte -> column map (default_rng(map_seed)) uses every
    column at least once; F = every state with a seeded coin below
    ``accept_fraction``; q0 = 0."""
    rng = np.random.default_rng(col_seed)
    while True:
        cols = rng.integers(0, num_states, (num_columns, num_states)).astype(np.uint32)
        if len({c.tobytes() for c in cols}) == num_columns:
            break
    acc = np.nonzero(rng.random(num_states) < accept_fraction)[0].astype(np.uint32)
    mrng = np.random.default_rng(map_seed)
    cmap = np.concatenate([np.arange(num_columns),
                           mrng.integers(0, num_columns, 256 - num_columns)])
    mrng.shuffle(cmap)
    delta = cols[cmap].T.copy()            # delta[s][b] = cols[cmap[b]][s]
    return DFA(delta.astype(np.uint32), 0, acc, identity_byte_map(),
               name or f"column{num_states}x{num_columns}s{col_seed}",
               {"col_seed": col_seed, "map_seed": map_seed, "num_columns": num_columns})


def from_pattern(pd) -> DFA:
    """Wrap a ``patterns.PatternDFA`` (20-letter amino-acid alphabet)."""
    return DFA(pd.delta.astype(np.uint32), pd.q0, pd.accepting.astype(np.uint32),
               pd.byte_to_symbol.copy(), f"prosite-like s{pd.seed} Q={pd.num_states}",
               {"seed": pd.seed, "pattern": pd.pattern.text(), "contains": pd.contains})
