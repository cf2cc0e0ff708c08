"""The one-chunk-per-lane last round of merged walks (dfa_plan_info_t::tail_lanes).

With interleaved one-symbol codes, merged rounds and an aligned input, the
round before the last hands each chunk's remaining walks to one lane, which
walks them over the raw input to the chunk's end (Section 4.1's L_i[j] for
every handed-over start state).  Checked against the oracle: every boundary
state and accept bit, and the state maps themselves; chunks with more walks
than a lane keeps (a permutation automaton: walks never meet) through the
overflow list; bytes outside Sigma that only the last round reads; chunks
whose walks all ended early (absorbing states) and the ragged last chunk;
two chunks per lane (forced with DFA_TAIL_K=2: the second chunk of the
last wavefront past the end, chunks left with different byte counts after
their multi-chain segments); and the same results with the last round kept
on wave-tiles (DFA_TAIL=0).  Tolerance 0."""
import sys

import numpy as np
import pytest

import oracle
from test_gpu_maps import check_maps
from workloads import column_dfa, configs, from_pattern, patterns, streams
from workloads.dfas import DFA as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def dfa_mod():
    import torch
    import paper_1210_5093_amd as dfa
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dfa.lib()
    return dfa


def permutation_dfa(seed, nq=40, nsym=3):
    """Every symbol permutes Q: distinct walks never meet, so each chunk keeps
    all |Q| walks to its end."""
    rng = np.random.default_rng(seed)
    delta = np.stack([rng.permutation(nq) for _ in range(nsym)], axis=1).astype(np.uint32)
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    b2s[ord("a"):ord("a") + nsym] = np.arange(nsym, dtype=np.uint8)
    return W(delta, 0, np.array([1, 5], dtype=np.uint32), b2s, f"perm{nq}x{nsym}s{seed}")


def perm_input(n, seed, nsym=3):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, nsym, n) + ord("a")).astype(np.uint8)


def cases():
    return {
        "c3b": lambda n: (configs.c3_byte_dfa(), configs.c3_byte_input(n)),
        "c1": lambda n: (configs.c1_dfa(2), configs.c1_input(n)),
        "cols6": lambda n: (column_dfa(91, 92, 150, 6), streams.uniform_bytes(93, n)),
        "c3p": lambda n: (configs.c3_protein_dfa(), configs.c3_protein_input(n)),
        "perm": lambda n: (permutation_dfa(7), perm_input(n, 8)),
        "anchored": lambda n: (from_pattern(patterns.pattern_dfa(32, contains=False)),
                               configs.c2_input(n, seed=62)),
    }


@pytest.fixture(autouse=True)
def packed_matcher(monkeypatch):
    """The packed matcher even for inputs under 4 MiB."""
    monkeypatch.setenv("DFA_KERNEL", "2")


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def run_bounds(dfa_mod, d, dev, chunk, look, **kw):
    import torch
    res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=chunk, lookahead=look, boundaries=True,
                                    interleave=True, single_step=True, **kw)
    torch.cuda.synchronize()
    return dfa_mod.result_tuple(res), bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF


@pytest.mark.parametrize("case", list(cases()))
@pytest.mark.parametrize("rounds", [2, 3, 5, 6])
def test_tail_boundaries_match_oracle(dfa_mod, case, rounds):
    n = (3 << 20) + 13
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    dev = to_dev(x)
    seen = 0
    for chunk in (2048, 8192, 65536):
        for look in (1, 3):
            plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds, interleave=True,
                                    single_step=True)
            if plan.kernel != 1:
                continue
            seen += plan.tail_lanes
            if plan.tail_lanes:
                assert plan.tail_start == 32 << (2 * (plan.rounds - 2))
            probes = [min(i * chunk, n) for i in range(plan.num_chunks + 1)]
            ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
            g, b = run_bounds(dfa_mod, d, dev, chunk, look, rounds=rounds)
            say(f"{case} rounds {rounds} chunk {chunk} r {look}: tail {plan.tail_lanes} "
                f"from {plan.tail_start} result {g}")
            assert g[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
            bad = np.nonzero(b != ps)[0]
            assert bad.size == 0, f"chunks {bad[:8]}: {b[bad[:8]]} vs {ps[bad[:8]]}"
    assert seen > 0, "no setting took the one-chunk-per-lane last round"
    d.close()


@pytest.mark.parametrize("case,chunk,look,rounds", [
    ("c3b", 8192, 2, 5),
    ("c3b", 4096, 1, 3),
    ("perm", 2048, 1, 3),        # every chunk overflows its lane's slots
    ("perm", 4096, 0, 4),
    ("anchored", 4096, 3, 4),    # walks end in the absorbing state before the last round
    ("cols6", 2048, 3, 2),
])
def test_tail_maps_match_oracle(dfa_mod, case, chunk, look, rounds):
    n = (2 << 20) + 77
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds, interleave=True, single_step=True)
    assert plan.kernel == 1 and plan.tail_lanes == 1, (plan.kernel, plan.tail_lanes)
    say(f"maps {case} chunk {chunk} r {look} rounds {rounds}, set max {plan.set_max}")
    pairs = check_maps(dfa_mod, w, x, to_dev(x), d, chunk, look, rounds=rounds, interleave=True,
                       single_step=True)
    say(f"  {pairs} pairs")
    d.close()


@pytest.mark.parametrize("n", [4096 + 1, 4096 + 2048, 4096 + 2049, 4096 + 2063, 3 * 4096 - 1])
def test_tail_ragged_last_chunk(dfa_mod, n):
    """The last chunk ends before, at and after the last round's start."""
    w, x = cases()["c3b"](n)
    d = dfa_mod.DFA.from_workload(w)
    for rounds in (4, 5):
        plan = dfa_mod.dfa_plan(d, n, 4096, 2, rounds=rounds, interleave=True)
        probes = [min(i * 4096, n) for i in range(plan.num_chunks + 1)]
        ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
        g, b = run_bounds(dfa_mod, d, to_dev(x), 4096, 2, rounds=rounds)
        assert g[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
        assert np.array_equal(b, ps)
    d.close()


@pytest.mark.parametrize("case", ["c3p", "anchored", "perm"])
@pytest.mark.parametrize("where", ["tail", "last_bytes", "prefix"])
def test_tail_invalid_byte(dfa_mod, case, where):
    """A byte outside Sigma in the part of a chunk only the last round reads
    (including chunks whose walks all ended early), in the input's last
    bytes, and in the translated prefix: always DFA_FLAG_SYMBOL."""
    import torch
    n = (1 << 20) + 5
    w, x = cases()[case](n)
    x = x.copy()
    bad_byte = 0xC1
    assert w.byte_to_symbol[bad_byte] >= w.num_symbols
    chunk, rounds = 8192, 4
    t0 = 32 << (2 * (rounds - 2))
    pos = {"tail": 77 * chunk + t0 + 1000, "last_bytes": n - 2, "prefix": 91 * chunk + 100}[where]
    x[pos] = bad_byte
    d = dfa_mod.DFA.from_workload(w)
    plan = dfa_mod.dfa_plan(d, n, chunk, 1, rounds=rounds, interleave=True, single_step=True)
    assert plan.tail_lanes == 1
    res, _ = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=chunk, lookahead=1, rounds=rounds,
                                  interleave=True, single_step=True)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL
    d.close()


def test_tail_plan_conditions(dfa_mod, monkeypatch):
    """Taken for interleaved one-symbol merged rounds on aligned inputs; not
    for two-symbol steps, linear code streams, unaligned inputs or DFA_TAIL=0,
    whose results are the same."""
    import torch
    n = (2 << 20) + 3
    w, x = cases()["c1"](n)
    d = dfa_mod.DFA.from_workload(w)
    assert dfa_mod.dfa_plan(d, n, 4096, 1, rounds=3, interleave=True).tail_lanes == 1
    assert dfa_mod.dfa_plan(d, n, 4096, 1, rounds=3).tail_lanes == 0
    assert dfa_mod.dfa_plan(d, n, 4096, 1, rounds=1, interleave=True).tail_lanes == 0
    c2 = dfa_mod.DFA.from_workload(configs.c2_dfa())
    p2 = dfa_mod.dfa_plan(c2, n, 4096, 6, rounds=3, interleave=True)
    assert p2.symbols_per_step == 2 and p2.tail_lanes == 0
    c2.close()
    probes = [min(i * 4096, n) for i in range((n + 4095) // 4096 + 1)]
    ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    want = (ofin, oracle.accepts(ofin, w.accepting), 0)
    buf = torch.empty(n + 16, dtype=torch.uint8, device="cuda")
    buf[1:n + 1].copy_(torch.from_numpy(x))
    for dev in (to_dev(x), buf[1:n + 1]):           # aligned, then unaligned
        g, b = run_bounds(dfa_mod, d, dev, 4096, 1, rounds=3)
        assert g[:3] == want and np.array_equal(b, ps)
    monkeypatch.setenv("DFA_TAIL", "0")
    assert dfa_mod.dfa_plan(d, n, 4096, 1, rounds=3, interleave=True).tail_lanes == 0
    g, b = run_bounds(dfa_mod, d, to_dev(x), 4096, 1, rounds=3)
    assert g[:3] == want and np.array_equal(b, ps)
    d.close()


@pytest.mark.parametrize("case", list(cases()))
def test_tail_two_chunks_per_lane_boundaries(dfa_mod, monkeypatch, case):
    """Two chunks per lane: every boundary state and the result equal the
    oracle's, for chunk counts that leave the last wavefront's second chunks
    partly or wholly past the end."""
    monkeypatch.setenv("DFA_TAIL_K", "2")
    n = (3 << 20) + 13
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    dev = to_dev(x)
    seen = 0
    for chunk, look, rounds in ((2048, 1, 2), (8192, 3, 4), (4096, 3, 3), (65536, 1, 5), (8192, 2, 4)):
        plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds, interleave=True, single_step=True)
        if plan.kernel != 1 or plan.tail_lanes == 0:
            continue
        assert plan.tail_lanes == 2, plan.tail_lanes
        seen += 1
        probes = [min(i * chunk, n) for i in range(plan.num_chunks + 1)]
        ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
        g, b = run_bounds(dfa_mod, d, dev, chunk, look, rounds=rounds)
        say(f"{case} two per lane, chunk {chunk} r {look} rounds {rounds}: {plan.num_chunks} chunks, "
            f"result {g}")
        assert g[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
        bad = np.nonzero(b != ps)[0]
        assert bad.size == 0, f"chunks {bad[:8]}: {b[bad[:8]]} vs {ps[bad[:8]]}"
    assert seen > 0, "no setting took the one-chunk-per-lane last round"
    d.close()


@pytest.mark.parametrize("case,chunk,look,rounds", [
    ("c3b", 8192, 2, 5),
    ("perm", 2048, 1, 3),
    ("anchored", 4096, 3, 4),
    ("c3p", 4096, 4, 2),
])
def test_tail_two_chunks_per_lane_maps(dfa_mod, monkeypatch, case, chunk, look, rounds):
    monkeypatch.setenv("DFA_TAIL_K", "2")
    n = (2 << 20) + 77
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds, interleave=True, single_step=True)
    assert plan.kernel == 1 and plan.tail_lanes == 2, (plan.kernel, plan.tail_lanes)
    pairs = check_maps(dfa_mod, w, x, to_dev(x), d, chunk, look, rounds=rounds, interleave=True,
                       single_step=True)
    say(f"two per lane maps {case}: {pairs} pairs")
    d.close()


@pytest.mark.parametrize("n", [4096 + 1, 4096 + 2063, 3 * 4096 - 1, 129 * 4096 + 700, 130 * 4096])
def test_tail_two_chunks_per_lane_ragged(dfa_mod, monkeypatch, n):
    """The last chunk short, and the chunk count below, at and past one
    wavefront's 128 chunks."""
    monkeypatch.setenv("DFA_TAIL_K", "2")
    w, x = cases()["c3b"](n)
    d = dfa_mod.DFA.from_workload(w)
    for rounds in (4, 5):
        plan = dfa_mod.dfa_plan(d, n, 4096, 2, rounds=rounds, interleave=True)
        assert plan.tail_lanes == 2
        probes = [min(i * 4096, n) for i in range(plan.num_chunks + 1)]
        ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
        g, b = run_bounds(dfa_mod, d, to_dev(x), 4096, 2, rounds=rounds)
        assert g[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
        assert np.array_equal(b, ps)
    d.close()


@pytest.mark.parametrize("where", ["tail", "last_bytes", "prefix"])
def test_tail_two_chunks_per_lane_invalid_byte(dfa_mod, monkeypatch, where):
    import torch
    monkeypatch.setenv("DFA_TAIL_K", "2")
    n = (1 << 20) + 5
    w, x = cases()["c3p"](n)
    x = x.copy()
    chunk, rounds = 8192, 4
    t0 = 32 << (2 * (rounds - 2))
    # chunk 77 is the second chunk of its lane (77 = 64 + 13)
    pos = {"tail": 77 * chunk + t0 + 1000, "last_bytes": n - 2, "prefix": 91 * chunk + 100}[where]
    x[pos] = 0xC1
    d = dfa_mod.DFA.from_workload(w)
    assert dfa_mod.dfa_plan(d, n, chunk, 1, rounds=rounds, interleave=True,
                            single_step=True).tail_lanes == 2
    res, _ = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=chunk, lookahead=1, rounds=rounds,
                                  interleave=True, single_step=True)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL
    d.close()


@pytest.mark.parametrize("case", ["c3b", "c3p", "c1", "anchored", "perm", "cols6"])
def test_tail_window_lookahead(dfa_mod, case):
    """Lookahead beyond the precomputed sets (the window pass: each chunk's
    Eq. 13 set as the image of a precomputed set over the bytes nearer the
    chunk) with interleaved codes and the one-chunk-per-lane last round: the
    window pass reads those bytes from the input itself.  Every boundary
    state and the result equal the oracle's."""
    n = (3 << 20) + 13
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    dev = to_dev(x)
    r0 = int(d.info().lookahead_tables)
    seen = 0
    for chunk, look, rounds in ((2048, r0 + 1, 2), (8192, r0 + 2, 4), (4096, 16, 3), (64, 40, 2)):
        if look <= r0:
            continue
        plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds, interleave=True, single_step=True)
        if plan.kernel != 1 or plan.tail_lanes == 0:
            continue
        seen += 1
        probes = [min(i * chunk, n) for i in range(plan.num_chunks + 1)]
        ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
        g, b = run_bounds(dfa_mod, d, dev, chunk, look, rounds=rounds)
        say(f"{case} window r {look} (r0 {r0}) chunk {chunk} rounds {rounds}: result {g}")
        assert g[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
        bad = np.nonzero(b != ps)[0]
        assert bad.size == 0, f"chunks {bad[:8]}: {b[bad[:8]]} vs {ps[bad[:8]]}"
    assert seen > 0, "no window-pass setting took the one-chunk-per-lane last round"
    d.close()


@pytest.mark.parametrize("case,chunk,look,rounds", [("c3b", 8192, 4, 4), ("c3p", 4096, 6, 2),
                                                    ("perm", 2048, 10, 3)])
def test_tail_window_lookahead_maps(dfa_mod, case, chunk, look, rounds):
    n = (2 << 20) + 77
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    assert look > int(d.info().lookahead_tables)
    plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds, interleave=True, single_step=True)
    assert plan.kernel == 1 and plan.tail_lanes == 1, (plan.kernel, plan.tail_lanes)
    pairs = check_maps(dfa_mod, w, x, to_dev(x), d, chunk, look, rounds=rounds, interleave=True,
                       single_step=True)
    say(f"window maps {case}: {pairs} pairs")
    d.close()


@pytest.mark.parametrize("case,look,rounds", [("c3b", 2, 4), ("c3p", 4, 2), ("perm", 10, 3),
                                              ("anchored", 3, 3), ("cols6", 3, 2)])
@pytest.mark.parametrize("mode", ["0", "1"])
def test_first_round_chunk_major(dfa_mod, monkeypatch, case, look, rounds, mode):
    """The first merged round chunk-major (DFA_ROUND1=1: one wavefront per
    chunk, grouping by end state) and tile-major (=0), both with the
    one-chunk-per-lane last round: the state maps themselves equal the
    oracle's (chunks with one start state, sets of hundreds, absorbing
    states, walks that never meet)."""
    monkeypatch.setenv("DFA_ROUND1", mode)
    n = (2 << 20) + 77
    w, x = cases()[case](n)
    d = dfa_mod.DFA.from_workload(w)
    plan = dfa_mod.dfa_plan(d, n, 4096, look, rounds=rounds, interleave=True, single_step=True)
    assert plan.kernel == 1 and plan.tail_lanes >= 1, (plan.kernel, plan.tail_lanes)
    pairs = check_maps(dfa_mod, w, x, to_dev(x), d, 4096, look, rounds=rounds, interleave=True,
                       single_step=True)
    say(f"first round mode {mode} {case}: {pairs} pairs")
    d.close()
