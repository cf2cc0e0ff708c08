"""Checks of the seeded workload generators (inputs shared by oracle and GPU
tests): the stream generator against SplitMix64's published sequence and a
numpy restatement; the pattern -> DFA pipeline against a direct NFA
simulation and Python ``re``; minimality by Moore refinement."""
import itertools

import numpy as np
import pytest

import oracle
from workloads import column_dfa, configs, from_pattern, patterns, random_dfa, streams


def test_splitmix64_published_sequence():
    """SplitMix64 with state 1234567: the first five outputs as published with
    the generator (Steele, Lea, Flood 2014 reference code)."""
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    s = 1234567
    out = []
    for _ in range(5):
        s = (s + streams.GAMMA) & streams.M64
        out.append(int(streams._mix64_np(np.array([s], dtype=np.uint64))[0]))
    assert out == expect


@pytest.mark.parametrize("first,n", [(0, 1), (0, 1000), (5, 3), (12345, 4099), (7, 0)])
def test_uniform_stream_c_matches_numpy(first, n):
    a = streams.uniform_bytes(77, n, first)
    b = streams.uniform_bytes_np(77, n, first)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("first,n", [(0, 1), (0, 1000), (3, 5), (4097, 2051)])
def test_residue_stream_c_matches_numpy(first, n):
    a = streams.residues(9, n, first)
    b = streams.residues_np(9, n, first)
    assert np.array_equal(a, b)


def test_streams_are_block_addressable():
    whole = streams.residues(4, 1 << 16)
    part = streams.residues(4, 1000, 30001)
    assert np.array_equal(whole[30001:31001], part)
    wb = streams.uniform_bytes(2, 1 << 16)
    assert np.array_equal(wb[999:2000], streams.uniform_bytes(2, 1001, 999))


def test_residue_frequencies_follow_weights():
    x = streams.residues(4, 1 << 20)
    counts = np.array([(x == ord(c)).sum() for c in patterns.AMINO])
    w = np.asarray(streams.AMINO_WEIGHTS, dtype=float)
    expect = w / w.sum() * x.size
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert counts.sum() == x.size
    assert chi2 < 60   # 19 degrees of freedom; p ~ 1e-6 at 60


def moore_classes(delta, acc):
    """Moore's partition refinement (not Hopcroft): number of equivalence classes."""
    cls = acc.astype(np.int64)
    while True:
        sig = np.concatenate([cls[:, None], cls[delta.astype(np.int64)]], axis=1)
        _, new = np.unique(sig, axis=0, return_inverse=True)
        new = new.reshape(-1)
        if len(np.unique(new)) == len(np.unique(cls)):
            return len(np.unique(new))
        cls = new


@pytest.mark.parametrize("seed", list(range(0, 12)))
@pytest.mark.parametrize("contains", [True, False])
def test_pattern_dfa_language(seed, contains):
    pd = patterns.pattern_dfa(seed, contains=contains)
    d = from_pattern(pd)
    nfa = patterns.thompson(pd.pattern, contains)
    rx = patterns.to_python_regex(pd.pattern, contains)
    import re
    crx = re.compile(rx)
    # reduced alphabet: letters named in the pattern plus one letter outside it
    named = sorted({a for e in pd.pattern.elements for a in e.residues})
    other = [a for a in range(20) if a not in named][:1]
    alpha = (named + other)[:4]
    letters = [patterns.AMINO[a] for a in alpha]
    words = ["".join(t) for L in range(6) for t in itertools.product(letters, repeat=L)]
    rng = np.random.default_rng(seed)
    for _ in range(150):
        L = int(rng.integers(1, 40))
        words.append("".join(patterns.AMINO[a] for a in rng.integers(0, 20, L)))
    for s in words:
        _, acc = oracle.membership(d.delta, d.byte_to_symbol, d.q0, d.accepting, s.encode())
        syms = [patterns.AMINO.index(c) for c in s]
        assert acc == patterns.nfa_accepts(nfa, syms), (pd.pattern.text(), s)
        assert acc == (crx.fullmatch(s) is not None), (pd.pattern.text(), s)


@pytest.mark.parametrize("seed", [0, 2, 5, 9, 15])
def test_pattern_dfa_is_minimal_and_complete(seed):
    d = from_pattern(patterns.pattern_dfa(seed))
    assert d.delta.max() < d.num_states
    assert moore_classes(d.delta, d.accept_mask()) == d.num_states
    seen, todo = {0}, [0]
    while todo:
        s = todo.pop()
        for t in d.delta[s]:
            if int(t) not in seen:
                seen.add(int(t))
                todo.append(int(t))
    assert len(seen) == d.num_states


def test_contains_language_has_one_accepting_sink():
    d = from_pattern(patterns.pattern_dfa(32))
    ab = oracle.absorbing(d.delta)
    assert ab.sum() == 1 and d.accept_mask()[ab].all()
    anch = from_pattern(patterns.pattern_dfa(32, contains=False))
    ab2 = oracle.absorbing(anch.delta)
    assert ab2.sum() == 1 and not anch.accept_mask()[ab2].any()


def test_recorded_c2_seed_search():
    first, lo, hi = configs.C2_SEARCH
    d = patterns.search_pattern_dfa(first, lo, hi)
    assert d.seed == configs.C2_PATTERN_SEED
    assert lo <= configs.c2_dfa().num_states <= hi


@pytest.mark.slow
def test_recorded_c3_seed_search():
    first, lo, hi = configs.C3_SEARCH
    assert patterns.search_pattern_dfa(first, lo, hi).seed == configs.C3_PATTERN_SEED


def test_c3_protein_size_and_c3_byte_columns():
    assert configs.C3_SEARCH[1] <= configs.c3_protein_dfa().num_states <= configs.C3_SEARCH[2]
    d = configs.c3_byte_dfa()
    assert d.num_states == 512
    assert len({d.delta[:, b].tobytes() for b in range(256)}) == 64


def test_random_dfa_recipe():
    d = random_dfa(1, 16, 256, 4)
    rng = np.random.default_rng(1)
    assert np.array_equal(d.delta, rng.integers(0, 16, (16, 256)))
    assert sorted(d.accepting.tolist()) == sorted(rng.choice(16, 4, replace=False).tolist())
    c = column_dfa(5, 6, 32, 8)
    assert len({c.delta[:, b].tobytes() for b in range(256)}) == 8
