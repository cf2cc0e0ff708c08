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
    d = configs.pattern_search(configs.C2_SEARCH)
    assert d.seed == configs.C2_PATTERN_SEED
    assert configs.C2_SEARCH[1] <= configs.c2_dfa().num_states <= configs.C2_SEARCH[2]


def _first_hit(args):
    first, lo, hi, tries, n = args
    try:
        return configs.pattern_search((first, lo, hi, tries, n)).seed
    except RuntimeError:
        return None


def test_recorded_c3_seed_search():
    """The whole C3 search (seeds 3 .. 67824), split into ranges over a
    process pool: the first hit of the lowest range with one is the search's."""
    from concurrent.futures import ProcessPoolExecutor
    first, lo, hi, _, n = configs.C3_SEARCH
    end = configs.C3_PATTERN_SEED + 1
    step = (end - first + 31) // 32
    ranges = [(a, lo, hi, min(step, end - a), n) for a in range(first, end, step)]
    with ProcessPoolExecutor(max_workers=8) as ex:
        hits = [h for h in ex.map(_first_hit, ranges) if h is not None]
    assert hits and hits[0] == configs.C3_PATTERN_SEED


def test_recorded_seeds_are_rare_in_their_inputs():
    """Expected occurrences of the pattern in the configured input length stay
    below the search's threshold, and the early-sink seeds are far above it."""
    wts = streams.AMINO_WEIGHTS
    for seed, n in [(configs.C2_PATTERN_SEED, configs.C2_BYTES),
                    (configs.C3_PATTERN_SEED, configs.C3_BYTES)]:
        assert n * patterns.occurrence_bound(patterns.random_pattern(seed), wts) <= 0.05
    for seed, n in [(configs.C2_EARLY_SINK_SEED, configs.C2_BYTES),
                    (configs.C3_EARLY_SINK_SEED, configs.C3_BYTES)]:
        assert n * patterns.occurrence_bound(patterns.random_pattern(seed), wts) > 1


def test_occurrence_bound_matches_counts():
    """The union bound against counted occurrences of short patterns in a
    residue stream: equal for a single-residue pattern, an upper bound (and
    within a factor of ~2) for a two-element one."""
    x = streams.residues(4, 1 << 20)
    text = x.tobytes().decode("ascii")
    import re
    wts = streams.AMINO_WEIGHTS
    one = patterns.Pattern((patterns.Element("res", (3,), 1, 1),))
    cnt = text.count(patterns.AMINO[3])
    exp = x.size * patterns.occurrence_bound(one, wts)
    assert abs(cnt - exp) < 5 * exp ** 0.5
    two = patterns.Pattern((patterns.Element("set", (0, 5), 1, 1),
                            patterns.Element("res", (9,), 1, 2)))
    starts = len(re.findall("(?=[%s%s]%s)" % (patterns.AMINO[0], patterns.AMINO[5],
                                              patterns.AMINO[9]), text))
    bound = x.size * patterns.occurrence_bound(two, wts)
    assert starts <= bound and bound < 2.2 * starts


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
