"""Record (seed, states) of PROSITE-like pattern DFAs for seeds 0..N-1.

The batched and served workloads need pattern DFAs of given sizes; scanning
seeds is slow, so the scan is done once and its result kept in
prosite_pool.json (inputs only: pattern seeds and their minimal DFA sizes).
Usage: python -m workloads.make_prosite_pool [N]
"""
import json
import os
import sys

from .patterns import TooLarge, pattern_dfa

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "prosite_pool.json")


def main(n: int = 4000, max_states: int = 1400) -> None:
    pool = []
    for s in range(n):
        try:
            d = pattern_dfa(s, max_states=max_states)
        except TooLarge:
            continue
        pool.append([s, d.num_states])
    with open(OUT, "w") as f:
        json.dump({"seeds_scanned": n, "max_states": max_states,
                   "contains_language": True, "pool": pool}, f)
    print(f"{len(pool)} pattern DFAs written to {OUT}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4000)
