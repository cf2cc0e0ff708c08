"""The five benchmark configurations as concrete synthetic inputs.

C1 plain:    one random complete DFA, 16 states over the 256-byte alphabet,
             q0 = 0, 4 accepting states (default_rng(1)); 1 MiB of uniform
             bytes from stream seed 2.
C2 protein:  minimal DFA for Sigma* P Sigma* of a seeded PROSITE-like pattern
             P over the 20 amino-acid letters, 270..330 states (seed search
             from 3); 256 MiB of residues from stream seed 4.
C3 large:    (i) protein DFA with 1288 states (seed search from 3; the first
             seed within +2% is used when no exact hit is found) and
             (ii) a 512-state byte DFA built from 64 distinct random columns
             (columns seed 5, byte->column map seed 6); 10 GiB inputs
             (residues, stream seed 10; uniform bytes, stream seed 11);
             chunk lengths 4 KiB .. 1 MiB.
C4 batched / C5 served: see ``batch_workload`` / ``served_workload``.

The seed searches are deterministic; their results are recorded below so the
DFAs are rebuilt directly (``tests/test_workloads.py`` re-runs the cheap
search).
"""
from __future__ import annotations

import numpy as np

from .dfas import DFA, random_dfa, column_dfa, from_pattern
from . import patterns, streams

MiB = 1 << 20
GiB = 1 << 30

# Recorded results of patterns.search_pattern_dfa(first_seed, lo, hi).
C2_SEARCH = (3, 270, 330)
C2_PATTERN_SEED = 32          # 284 states
C3_SEARCH = (3, 1288, 1313)
C3_PATTERN_SEED = 5825        # 1297 states (first seed within +2% of 1288)

C1_INPUT_SEED = 2
C2_INPUT_SEED = 4
C3_PROTEIN_INPUT_SEED = 10
C3_BYTE_INPUT_SEED = 11

C1_BYTES = 1 * MiB
C2_BYTES = 256 * MiB
C3_BYTES = 10 * GiB
C3_CHUNKS = [4096 << k for k in range(9)]   # 4 KiB .. 1 MiB


def c1_dfa(seed: int = 1) -> DFA:
    return random_dfa(seed, 16, 256, 4, name=f"C1 random 16x256 seed {seed}")


def c1_input(n: int = C1_BYTES, seed: int = C1_INPUT_SEED, first: int = 0) -> np.ndarray:
    return streams.uniform_bytes(seed, n, first)


def c2_dfa() -> DFA:
    d = from_pattern(patterns.pattern_dfa(C2_PATTERN_SEED))
    d.name = f"C2 prosite-like seed {C2_PATTERN_SEED} Q={d.num_states}"
    return d


def c2_input(n: int = C2_BYTES, seed: int = C2_INPUT_SEED, first: int = 0, out=None) -> np.ndarray:
    return streams.residues(seed, n, first, out=out)


def c3_protein_dfa() -> DFA:
    d = from_pattern(patterns.pattern_dfa(C3_PATTERN_SEED))
    d.name = f"C3 prosite-like seed {C3_PATTERN_SEED} Q={d.num_states}"
    return d


def c3_byte_dfa() -> DFA:
    d = column_dfa(5, 6, 512, 64)
    d.name = "C3 byte 512 states, 64 columns (seeds 5, 6)"
    return d


def c3_protein_input(n: int, first: int = 0, out=None) -> np.ndarray:
    return streams.residues(C3_PROTEIN_INPUT_SEED, n, first, out=out)


def c3_byte_input(n: int, first: int = 0, out=None) -> np.ndarray:
    return streams.uniform_bytes(C3_BYTE_INPUT_SEED, n, first, out=out)
