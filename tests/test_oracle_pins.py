"""Pins of the CPU oracle against values the paper prints, closed forms,
library routines (Python ``re``, numpy matrix products) and invariants.

None of these checks compares the oracle with itself: every expected value is
either printed in the paper (golden fixtures, cited there), computed by a
different route (boolean transition-matrix products, regular-expression
matching), or an invariant stated by the paper (Lemma of Section 4.3,
composition of Eq. 9, prefix states lying in the initial-state sets of
Eq. 11)."""
import itertools
import re

import numpy as np
import pytest

import oracle
from conftest import load_golden
from workloads import random_dfa, column_dfa, from_pattern, patterns


def golden_dfa(name):
    g = load_golden(name)
    delta = np.asarray(g["delta"], dtype=np.uint32)
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    for i, ch in enumerate(g["symbols"]):
        b2s[ord(ch)] = i
    return g, delta, b2s


def enc(s):
    return np.frombuffer(s.encode("ascii"), dtype=np.uint8)


# ---------------------------------------------------------------------------
# Printed worked examples
# ---------------------------------------------------------------------------
def test_motivating_example_final_state_and_accept():
    g, delta, b2s = golden_dfa("motivating_dfa.json")
    fin, acc = oracle.membership(delta, b2s, g["q0"], g["accepting"], enc(g["input"]))
    assert fin == g["printed"]["final_state"]
    assert acc == g["printed"]["accepted"]


def test_motivating_example_boundary_states():
    g, delta, b2s = golden_dfa("motivating_dfa.json")
    w = enc(g["input"])
    _, ps = oracle.walk(delta, b2s, g["q0"], w, probes=[0, 4, 8, 12])
    assert ps.tolist() == g["printed"]["boundary_states"]
    assert "".join(g["printed"]["chunks"]) == g["input"]


def test_motivating_example_state_map_of_chunk2():
    g, delta, b2s = golden_dfa("motivating_dfa.json")
    w = enc(g["input"])
    L2 = oracle.chunk_map(delta, b2s, w, 8, 12, [0, 1])
    assert L2.tolist() == g["printed"]["chunk2_map_from_q0_q1"]


def test_motivating_example_isets():
    g, delta, b2s = golden_dfa("motivating_dfa.json")
    ex = np.zeros(delta.shape[0], dtype=bool)
    ex[g["error_state"]] = True
    I = oracle.isets(delta, ex)
    for k, ch in enumerate(g["symbols"]):
        assert np.nonzero(I[k])[0].tolist() == g["printed"]["iset"][ch]
    assert oracle.imax(delta, ex) == g["printed"]["imax"]
    # the error state is the only absorbing state
    assert np.nonzero(oracle.absorbing(delta))[0].tolist() == [g["error_state"]]


def test_motivating_example_work_counts():
    """Section 3: 12 sequential steps; 8 per processor with equal chunks and two
    start states (1.5x); 6 with the balanced partition (2x); 4 with one-symbol
    reverse lookahead (3x).  The balanced lengths follow Eq. (5)/(10)."""
    g, _, _ = golden_dfa("motivating_dfa.json")
    seq, equal, balanced, lookahead = g["printed"]["work_units_seq_equal_chunks_lookahead"]
    n, P = 12, 3
    assert seq == n
    assert equal == 2 * (n // P)
    assert oracle.first_chunk_length(n, 2, [1, 1, 1]) == balanced
    assert oracle.first_chunk_length(n, 1, [1, 1, 1]) == lookahead


def test_example_dfa_isets_and_imax():
    g, delta, b2s = golden_dfa("example_dfa.json")
    ex = np.zeros(delta.shape[0], dtype=bool)
    ex[g["error_state"]] = True
    I = oracle.isets(delta, ex)
    for k, ch in enumerate(g["symbols"]):
        assert np.nonzero(I[k])[0].tolist() == g["printed"]["iset"][ch]
    assert oracle.imax(delta, ex) == g["printed"]["imax"]


def test_example_dfa_sbase_and_ibase():
    """Fig. 8: the flattened row-major table with plain state ids, and the
    symbol encoding of the 20-symbol input."""
    g, delta, b2s = golden_dfa("example_dfa.json")
    assert delta.reshape(-1).tolist() == g["printed"]["sbase_plain"]
    assert b2s[enc(g["input20"])].tolist() == g["printed"]["ibase_input20"]


def test_example_dfa_lookahead_partition():
    """Fig. 7 / Eq. (10): n = 36, I_max = 2, three equal processors -> chunks
    18 + 9 + 9, lookahead symbols a and b, initial-state sets {q1,q3}, {q2,q3}."""
    g, delta, b2s = golden_dfa("example_dfa.json")
    w = g["input36"]
    p = g["printed"]
    assert oracle.first_chunk_length(36, p["imax"], [1, 1, 1]) == p["first_chunk_len_imax"]
    assert oracle.first_chunk_length(36, 4, [1, 1, 1]) == p["first_chunk_len_allstates"]
    ranges = oracle.partition(36, p["imax"], [1, 1, 1])
    assert [w[a:b + 1] for a, b in ranges] == p["lookahead_chunks"]
    looks = [w[a - 1] for a, _ in ranges[1:]]
    assert looks == p["lookahead_symbols"]
    ex = np.zeros(delta.shape[0], dtype=bool)
    ex[g["error_state"]] = True
    I = oracle.isets(delta, ex)
    assert [np.nonzero(I[g["symbols"].index(c)])[0].tolist() for c in looks] == \
        p["lookahead_chunk_isets"]


def test_table1_weights_and_ranges():
    g, _, _ = golden_dfa("example_dfa.json")
    p = g["printed"]
    w = oracle.weights(p["table1_capacities"])
    assert w == pytest.approx(p["table1_weights"])
    L0 = oracle.first_chunk_length(36, 4, w)
    assert L0 == pytest.approx(p["table1_first_chunk_len"])
    Lk = [L0] + [L0 / 4] * 2
    assert [a * b for a, b in zip(Lk, w)] == pytest.approx(p["table1_weighted_lengths"])
    assert [list(r) for r in oracle.partition(36, 4, w)] == p["table1_ranges"]


def test_example_dfa_final_state_by_matrix_product():
    """Derived value, pinned by a different route: the one-hot start vector
    times the boolean transition matrices of the input symbols."""
    g, delta, b2s = golden_dfa("example_dfa.json")
    for key in ("input36", "input20"):
        w = enc(g[key])
        fin, acc = oracle.membership(delta, b2s, g["q0"], g["accepting"], w)
        assert fin == matrix_walk(delta, b2s, g["q0"], w)
        assert fin == g["derived"]["final_state_" + key]
        assert acc == g["derived"]["accepted_" + key]
    _, ps = oracle.walk(delta, b2s, 0, enc(g["input36"]), probes=list(range(37)))
    first_err = int(np.argmax(ps == g["error_state"]))
    assert first_err == g["derived"]["error_reached_after_symbols_input36"]


# ---------------------------------------------------------------------------
# Library routines: regular expressions and matrix products
# ---------------------------------------------------------------------------
def matrix_walk(delta, b2s, start, w):
    """delta*(start, w) as argmax of e_start * M_{w_0} * M_{w_1} * ... with
    M_a[s, t] = [delta(s, a) = t] (numpy matmul)."""
    nq, nsym = delta.shape
    M = np.zeros((nsym, nq, nq), dtype=np.int64)
    for a in range(nsym):
        M[a, np.arange(nq), delta[:, a].astype(np.int64)] = 1
    v = np.zeros(nq, dtype=np.int64)
    v[start] = 1
    for byte in w:
        v = v @ M[b2s[byte]]
    assert v.sum() == 1
    return int(np.argmax(v))


@pytest.mark.parametrize("name,regex", [("motivating_dfa.json", "a*bc*"),
                                        ("example_dfa.json", "(ab|bab|bb)a*")])
def test_small_dfa_languages_against_re(name, regex):
    """All strings up to length 7: Algorithm 1's accept bit equals Python's
    ``re.fullmatch`` for the language of the figure (a*bc* is stated in
    Section 3; the example DFA's language is read off Fig. 6)."""
    g, delta, b2s = golden_dfa(name)
    rx = re.compile(regex)
    for L in range(8):
        for tup in itertools.product(g["symbols"], repeat=L):
            s = "".join(tup)
            _, acc = oracle.membership(delta, b2s, g["q0"], g["accepting"], enc(s))
            assert acc == (rx.fullmatch(s) is not None), s


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_dfa_walk_against_matrix_product(seed):
    d = random_dfa(seed, 16, 256, 4)
    rng = np.random.default_rng(100 + seed)
    for n in (0, 1, 2, 17, 200):
        w = rng.integers(0, 256, n).astype(np.uint8)
        fin, ps = oracle.walk(d.delta, d.byte_to_symbol, d.q0, w, probes=list(range(n + 1)))
        assert fin == matrix_walk(d.delta, d.byte_to_symbol, d.q0, w)
        for p in range(0, n + 1, max(1, n // 5)):
            assert ps[p] == matrix_walk(d.delta, d.byte_to_symbol, d.q0, w[:p])


def test_nonsquare_random_dfa_walk_against_matrix_product():
    """Non-square table (Q != |Sigma|) so a transposed index cannot pass."""
    d = random_dfa(9, 37, 5, 3)
    rng = np.random.default_rng(9)
    w = rng.integers(0, 5, 300).astype(np.uint8)
    for start in (0, 5, 36):
        fin, _ = oracle.walk(d.delta, d.byte_to_symbol, start, w)
        assert fin == matrix_walk(d.delta, d.byte_to_symbol, start, w)


def test_invalid_symbol_is_reported():
    d = random_dfa(4, 8, 5, 2)
    w = np.array([0, 1, 2, 7, 1], dtype=np.uint8)   # byte 7 maps to 0xFF
    with pytest.raises(oracle.InvalidSymbol) as ei:
        oracle.walk(d.delta, d.byte_to_symbol, 0, w)
    assert ei.value.index == 3
    fin, _ = oracle.walk(d.delta, d.byte_to_symbol, 3, np.zeros(0, dtype=np.uint8))
    assert fin == 3   # empty input: the loop of Algorithm 1 does not run


# ---------------------------------------------------------------------------
# Closed forms and invariants
# ---------------------------------------------------------------------------
def test_random_dfa_expected_iset_size_closed_form():
    """For delta uniform, |I_a| has mean Q (1 - (1 - 1/Q)^Q); C1 has 256 columns."""
    Q = 16
    d = random_dfa(1, Q, 256, 4)
    sizes = oracle.isets(d.delta).sum(axis=1)
    expect = Q * (1 - (1 - 1 / Q) ** Q)
    assert abs(sizes.mean() - expect) < 0.5
    # a direct count of the distinct entries of each column (numpy unique)
    assert sizes.tolist() == [len(np.unique(d.delta[:, a])) for a in range(256)]


@pytest.mark.parametrize("kind", ["random", "column", "pattern", "pattern_anchored"])
def test_prefix_states_lie_in_lookahead_isets(kind):
    """For every position p >= 1, delta*(q0, w[0:p]) is in I_{w[p-1]} or is an
    absorbing state (Section 4.2: the state after the lookahead symbol)."""
    if kind == "random":
        d = random_dfa(3, 40, 256, 5)
        w = np.random.default_rng(3).integers(0, 256, 3000).astype(np.uint8)
    elif kind == "column":
        d = column_dfa(7, 8, 64, 8)
        w = np.random.default_rng(4).integers(0, 256, 3000).astype(np.uint8)
    else:
        d = from_pattern(patterns.pattern_dfa(5, contains=(kind == "pattern")))
        rng = np.random.default_rng(5)
        w = np.frombuffer(patterns.AMINO.encode(), dtype=np.uint8)[rng.integers(0, 20, 3000)]
    ab = oracle.absorbing(d.delta)
    I = oracle.isets(d.delta, ab)
    _, ps = oracle.walk(d.delta, d.byte_to_symbol, d.q0, w, probes=list(range(len(w) + 1)))
    for p in range(1, len(w) + 1):
        s = ps[p]
        assert ab[s] or I[d.byte_to_symbol[w[p - 1]], s]


@pytest.mark.parametrize("seed", [0, 5, 9])
def test_lemma_more_lookahead_never_grows(seed):
    """Lemma (Section 4.3): I_{sigma' sigma} is a subset of I_sigma, hence
    I_max,1 >= I_max,2 >= I_max,3."""
    d = from_pattern(patterns.pattern_dfa(seed))
    ab = oracle.absorbing(d.delta)
    nsym = d.num_symbols
    I1 = oracle.isets(d.delta, ab)
    for s1 in range(nsym):
        for s2 in range(nsym):
            I2 = oracle.iset_word(d.delta, [s1, s2], ab)
            assert not np.any(I2 & ~I1[s2])
    small = random_dfa(seed, 12, 3, 2)
    ab2 = oracle.absorbing(small.delta)
    m1, m2, m3 = (oracle.imax_r(small.delta, r, ab2) for r in (1, 2, 3))
    assert m1 == oracle.imax(small.delta, ab2)
    assert m1 >= m2 >= m3


def test_composition_equals_walk_over_concatenation():
    """Eq. (9): L_{i,j}[k] = L_j[L_i[k]] equals the state map of c_i c_j."""
    d = random_dfa(11, 23, 256, 4)
    rng = np.random.default_rng(11)
    w = rng.integers(0, 256, 90).astype(np.uint8)
    allq = np.arange(23)
    Li = oracle.chunk_map(d.delta, d.byte_to_symbol, w, 0, 40, allq)
    Lj = oracle.chunk_map(d.delta, d.byte_to_symbol, w, 40, 90, allq)
    Lij = oracle.chunk_map(d.delta, d.byte_to_symbol, w, 0, 90, allq)
    assert oracle.compose(Li, Lj) == Lij.tolist()
    # Eq. (8): sequential merge of three maps from q0 equals the final state
    L0 = oracle.chunk_map(d.delta, d.byte_to_symbol, w, 0, 30, allq)
    L1 = oracle.chunk_map(d.delta, d.byte_to_symbol, w, 30, 60, allq)
    L2 = oracle.chunk_map(d.delta, d.byte_to_symbol, w, 60, 90, allq)
    fin, _ = oracle.walk(d.delta, d.byte_to_symbol, 0, w)
    assert oracle.sequential_merge([L0, L1, L2], 0) == fin == matrix_walk(
        d.delta, d.byte_to_symbol, 0, w)


def test_pure_python_walk_agrees_on_tiny_inputs():
    g, delta, b2s = golden_dfa("example_dfa.json")
    for s in ("", "a", "ab", "bab", "bba", g["input20"]):
        assert oracle.walk_py(delta.tolist(), b2s, 0, s.encode()) == \
            matrix_walk(delta, b2s, 0, enc(s))
    I = oracle.isets_py(delta.tolist(), [g["error_state"]])
    assert [sorted(x) for x in I] == [g["printed"]["iset"]["a"], g["printed"]["iset"]["b"]]
