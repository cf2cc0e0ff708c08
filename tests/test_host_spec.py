"""Host multicore speculative matcher (Algorithm 3 on CPU threads) and the
capacity-weighted partition of Eqs. (1)-(7)/(10).

The partition is pinned to the values the paper prints (Table 1 ranges; the
18-symbol first chunk of Section 4.2 and its 24-symbol counterpart without
lookahead) and compared with the oracle's partition (itself pinned to the
same values) on random cases.  Every match result must equal the oracle's
sequential walk (tolerance 0), for any thread count and capacity vector."""
import numpy as np
import pytest

import oracle
from conftest import load_golden
from workloads import configs, from_pattern, patterns, random_dfa, column_dfa

host = pytest.importorskip("paper_1210_5093_amd.host")


@pytest.fixture(scope="module", autouse=True)
def built():
    import os
    if not os.path.exists(host.HOST_LIB_PATH):
        from paper_1210_5093_amd import build
        build.build_host()


def golden_dfa(name):
    g = load_golden(name)
    delta = np.asarray(g["delta"], dtype=np.uint32)
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    for i, ch in enumerate(g["symbols"]):
        b2s[ord(ch)] = i
    return g, delta, b2s


def enc(s):
    return np.frombuffer(s.encode("ascii"), dtype=np.uint8)


def ranges(starts):
    return [(starts[k], starts[k + 1] - 1) for k in range(len(starts) - 1)]


# ---------------------------------------------------------------------------
# Partition
# ---------------------------------------------------------------------------
def test_partition_table1_ranges():
    g, _, _ = golden_dfa("example_dfa.json")
    p = g["printed"]
    starts = host.partition(36, 4, 3, p["table1_capacities"])
    assert ranges(starts) == [tuple(r) for r in p["table1_ranges"]]


def test_partition_first_chunk_with_and_without_lookahead():
    g, delta, b2s = golden_dfa("example_dfa.json")
    p = g["printed"]
    s = host.partition(36, p["imax"], 3)
    assert s[1] - s[0] == p["first_chunk_len_imax"]
    chunks = [g["input36"][s[k]:s[k + 1]] for k in range(3)]
    assert chunks == p["lookahead_chunks"]
    s = host.partition(36, len(delta) - 1, 3)    # |Q| = 4 without the error state
    assert s[1] - s[0] == p["first_chunk_len_allstates"]


@pytest.mark.parametrize("seed", range(40))
def test_partition_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 20))
    n = int(rng.integers(0, 1 << 30)) if seed % 3 else int(rng.integers(0, 100))
    m = float(rng.integers(1, 1300))
    caps = None if seed % 2 else list(rng.uniform(1.0, 100.0, size=P))
    w = oracle.weights(caps) if caps is not None else [1.0] * P
    starts = host.partition(n, m, P, caps)
    assert starts[0] == 0 and starts[-1] == n
    assert all(a <= b for a, b in zip(starts, starts[1:]))
    if n >= 4 * P * m:   # no clamping: the ranges are exactly Eqs. (6)-(7)
        assert ranges(starts) == oracle.partition(n, m, w)


def test_partition_rejects_bad_arguments():
    with pytest.raises(host.HostError):
        host.partition(10, 0, 3)
    with pytest.raises(host.HostError):
        host.partition(10, 2, 2, [1.0, 0.0])


# ---------------------------------------------------------------------------
# Matcher
# ---------------------------------------------------------------------------
def test_example_dfa_input36():
    g, delta, b2s = golden_dfa("example_dfa.json")
    h = host.HostDFA(delta, g["q0"], g["accepting"], b2s)
    assert h.imax == g["printed"]["imax"]
    for threads in (1, 2, 3, 5, 36, 40):
        assert h.match(enc(g["input36"]), threads) == (g["derived"]["final_state_input36"],
                                                       g["derived"]["accepted_input36"])
    assert h.match(enc(g["input36"]), 3, g["printed"]["table1_capacities"]) == (4, False)


def test_motivating_example():
    g, delta, b2s = golden_dfa("motivating_dfa.json")
    h = host.HostDFA(delta, g["q0"], g["accepting"], b2s)
    for threads in (1, 2, 3, 4, 12, 20):
        assert h.match(enc(g["input"]), threads) == (g["printed"]["final_state"],
                                                     g["printed"]["accepted"])


@pytest.mark.parametrize("threads", [1, 2, 7, 16])
def test_c1_full_input(threads):
    w = configs.c1_dfa(1)
    x = configs.c1_input(1 << 20)
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    assert host.HostDFA.from_workload(w).match(x, threads) == (fin, acc)


def test_protein_prefix_with_unequal_capacities():
    w = configs.c2_dfa()
    x = configs.c2_input(4 << 20)
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    h = host.HostDFA.from_workload(w)
    assert h.match(x, 8) == (fin, acc)
    assert h.match(x, 4, [3.0, 1.0, 0.5, 2.0]) == (fin, acc)


@pytest.mark.parametrize("seed", range(12))
def test_random_dfas_and_lengths(seed):
    rng = np.random.default_rng(100 + seed)
    kind = seed % 3
    if kind == 0:
        w = random_dfa(seed, int(rng.integers(1, 40)), int(rng.integers(1, 257)), 3)
    elif kind == 1:
        w = column_dfa(seed, seed + 1, int(rng.integers(2, 200)), int(rng.integers(1, 65)))
    else:
        w = from_pattern(patterns.pattern_dfa(seed, contains=bool(seed % 2)))
    n = int(rng.integers(0, 200000))
    valid = np.flatnonzero(w.byte_to_symbol < w.delta.shape[1]).astype(np.uint8)
    x = valid[rng.integers(0, valid.size, size=n)]
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    h = host.HostDFA.from_workload(w)
    for threads in (1, 3, 9):
        assert h.match(x, threads) == (fin, acc), threads
    if n:
        start = int(rng.integers(0, w.delta.shape[0]))
        fs, _ = oracle.walk(w.delta, w.byte_to_symbol, start, x)
        assert h.match(x, 5, start=start)[0] == fs


def test_edge_cases():
    w = configs.c1_dfa(2)
    h = host.HostDFA.from_workload(w)
    empty = np.zeros(0, dtype=np.uint8)
    assert h.match(empty, 4) == (w.q0, bool(np.isin(w.q0, w.accepting)))
    x = configs.c1_input(3)
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    assert h.match(x, 16) == (fin, acc)          # fewer bytes than threads


def test_invalid_symbol_is_an_error():
    w = configs.c2_dfa()
    x = configs.c2_input(1 << 16).copy()
    h = host.HostDFA.from_workload(w)
    for pos in (0, 5, 40000, (1 << 16) - 1):
        y = x.copy()
        y[pos] = ord("#")
        with pytest.raises(host.HostError) as e:
            h.match(y, 6)
        assert e.value.rc == host.DFA_E_SYMBOL


def test_profile_capacities():
    w = configs.c1_dfa(1)
    h = host.HostDFA.from_workload(w)
    caps = h.profile(configs.c1_input(1 << 18), 3)
    assert len(caps) == 3 and all(c > 0 for c in caps)
    x = configs.c1_input(1 << 16)
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    assert h.match(x, 3, caps) == (fin, acc)
