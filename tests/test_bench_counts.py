"""bench.py's work counts (the roofline numerators) against brute force on
small inputs: Algorithm 3's lookups (every start state of a chunk walked over
the whole chunk), the least work of early exit at absorbing states, and the
table reads and covered bytes of merged walks.  The brute force walks each
(chunk, start state) one symbol at a time in plain Python."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import configs, from_pattern, patterns, random_dfa, streams  # noqa: E402


def cases():
    pat = from_pattern(patterns.pattern_dfa(7, contains=True))      # accepting sink
    anch = from_pattern(patterns.pattern_dfa(7, contains=False))    # rejecting sink
    rnd = random_dfa(3, num_states=12, num_symbols=256)             # no absorbing state
    prot = configs.c2_input(5000, seed=11)
    return [("pattern", pat, prot), ("anchored", anch, prot),
            ("random", rnd, streams.uniform_bytes(12, 4000))]


def brute_sets(w, x, chunk, r):
    delta = w.delta.astype(np.int64)
    sym = w.byte_to_symbol.astype(np.int64)
    nq = delta.shape[0]
    absorbing = [bool(np.all(delta[q] == q)) for q in range(nq)]
    nch = (x.size + chunk - 1) // chunk
    sets = [[int(w.q0)]]
    for i in range(1, nch):
        p = i * chunk
        S = set(range(nq))
        for t in range(p - (min(r, p) if r > 0 else 0), p):
            S = {int(delta[q, sym[x[t]]]) for q in S}
        sets.append(sorted(q for q in S if not absorbing[q]))
    return sets, absorbing


@pytest.mark.parametrize("case", ["pattern", "anchored", "random"])
@pytest.mark.parametrize("chunk,r", [(64, 0), (100, 1), (256, 3), (333, 5)])
@pytest.mark.parametrize("step", [1, 2, 3])
def test_algorithmic_and_early_exit_counts(case, chunk, r, step):
    _, w, x = next(c for c in cases() if c[0] == case)
    sets, absorbing = brute_sets(w, x, chunk, r)
    delta = w.delta.astype(np.int64)
    sym = w.byte_to_symbol.astype(np.int64)
    n = x.size
    algo = exit_work = 0
    for i, S in enumerate(sets):
        ln = min(chunk, n - i * chunk)
        algo += len(S) * math.ceil(ln / step)
        for s in S:
            for t in range(ln):
                s = int(delta[s, sym[x[i * chunk + t]]])
                if t % step == 0:
                    exit_work += 1
                if absorbing[s]:
                    break
    assert bench.algorithmic_lookups(w, x, chunk, r, step) == algo
    assert bench.early_exit_lookups(w, x, chunk, r, int(w.q0), step) == exit_work


@pytest.mark.parametrize("case", ["pattern", "anchored", "random"])
@pytest.mark.parametrize("chunk,r,rounds", [(300, 1, 2), (700, 3, 3), (1000, 5, 4), (90, 1, 2)])
@pytest.mark.parametrize("step", [1, 2])
def test_merged_counts(case, chunk, r, rounds, step):
    _, w, x = next(c for c in cases() if c[0] == case)
    sets, absorbing = brute_sets(w, x, chunk, r)
    delta = w.delta.astype(np.int64)
    sym = w.byte_to_symbol.astype(np.int64)
    n = x.size
    reads = covered = 0
    for i, S in enumerate(sets):
        ln = min(chunk, n - i * chunk)
        walks, ext, t0 = list(S), 0, 0
        for k in range(rounds):
            t1 = 32 << (2 * k)
            if k + 1 == rounds:
                for s in walks:
                    if absorbing[s] or ln <= t0:
                        continue
                    t = t0
                    while True:
                        reads += 1
                        ext = max(ext, min(ln, t + step))
                        for j in range(step):
                            if t + j < ln:
                                s = int(delta[s, sym[x[i * chunk + t + j]]])
                        t += step
                        if t >= ln or absorbing[s]:
                            break
                break
            end = min(ln, t1)
            nxt = set()
            for s in walks:
                if end > t0:
                    reads += math.ceil((end - t0) / step)
                    ext = max(ext, end)
                for t in range(t0, end):
                    s = int(delta[s, sym[x[i * chunk + t]]])
                if ln > t1 and not absorbing[s]:
                    nxt.add(s)
            walks, t0 = sorted(nxt), t1
        covered += ext
    assert bench.merged_lookups(w, x, chunk, r, rounds, step) == (reads, covered)


def test_stored_traffic_lines_parse():
    """Every committed traffic line names a kernel the way the bench does
    (template arguments with spaces included) and parses back."""
    import glob
    import re
    lines = []
    for path in glob.glob(os.path.join(bench.ROOT, "profiles", "*.md")):
        with open(path) as fh:
            lines += [ln for ln in fh if ln.startswith("traffic:")]
    assert lines, "no traffic lines in profiles/"
    for ln in lines:
        m = re.match(r"traffic: kernel=(.+?) workload=(\S+) lookahead=(\d+) chunk=(\d+) "
                     r"bytes=(\d+) sources=([0-9a-f]+)", ln)
        assert m, ln
        if m.group(6) != bench.kernel_source_digest():
            continue
        got, src = bench.stored_traffic(m.group(1), m.group(2), int(m.group(3)), int(m.group(4)))
        assert got == int(m.group(5)) and src, ln
