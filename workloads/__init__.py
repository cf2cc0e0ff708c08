"""Seeded synthetic workloads (DFAs and input streams) shared by the tests,
the oracle checks and the benchmark.  This package only produces inputs: it
holds none of the membership test's arithmetic."""
from .dfas import DFA, random_dfa, column_dfa, from_pattern, identity_byte_map  # noqa: F401
from . import patterns, streams, configs  # noqa: F401


def build(force: bool = True) -> None:
    streams.build(force)
