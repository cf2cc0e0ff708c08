"""Writes large_finals.json: the oracle's final state and accept bit
(Algorithm 1, one sequential walk) for the full-size protein-style and
large-DFA inputs, and the state after their first GiB.  The benchmark checks
its GPU results against these values; they come from oracle/ alone.

Run from the repository root: python tests/golden/make_large_finals.py"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                      # noqa: E402
from workloads import configs     # noqa: E402

GiB = 1 << 30
BLOCK = 256 << 20


def walk_stream(w, gen, n):
    """Sequential walk over n bytes generated block by block; returns the
    final state and the state after the first GiB (or the final one)."""
    state, at_gib = int(w.q0), None
    buf = np.empty(BLOCK, dtype=np.uint8)
    for off in range(0, n, BLOCK):
        m = min(BLOCK, n - off)
        x = gen(m, first=off, out=buf)
        state, _ = oracle.walk(w.delta, w.byte_to_symbol, state, x[:m])
        if off + m == GiB:
            at_gib = state
    return state, (state if at_gib is None else at_gib)


def main():
    out = {}
    cases = [
        ("c2", configs.c2_dfa(), lambda m, first, out: configs.c2_input(m, first=first, out=out),
         configs.C2_BYTES, f"protein-style, pattern seed {configs.C2_PATTERN_SEED}, stream "
         f"{configs.C2_INPUT_SEED}"),
        ("c3_protein", configs.c3_protein_dfa(), configs.c3_protein_input, configs.C3_BYTES,
         f"large protein DFA, pattern seed {configs.C3_PATTERN_SEED}, stream "
         f"{configs.C3_PROTEIN_INPUT_SEED}"),
        ("c3_byte", configs.c3_byte_dfa(), configs.c3_byte_input, configs.C3_BYTES,
         f"byte DFA 512 states (seeds 5, 6), stream {configs.C3_BYTE_INPUT_SEED}"),
    ]
    for key, w, gen, n, desc in cases:
        fin, at_gib = walk_stream(w, gen, n)
        out[key] = {"what": desc, "bytes": n, "states": w.num_states, "final_state": fin,
                    "accepted": bool(oracle.accepts(fin, w.accepting)),
                    "state_after_1GiB": at_gib}
        print(key, out[key], flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "large_finals.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
