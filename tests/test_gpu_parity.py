"""GPU parity: the HIP path (through the C ABI) against the oracle, bit-exact.

Every final state, accept bit and chunk-boundary state must equal the oracle's
sequential walk (Algorithm 1) on the same seeded input: tolerance 0 (integer
work; the final state is unique).  Sizes span many chunks and ragged tails;
the bench configuration (C2 at 256 MiB, planner chunking) is checked in
full."""
import sys

import numpy as np
import pytest

import oracle
from conftest import load_golden
from workloads import configs, from_pattern, patterns, random_dfa, column_dfa, streams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfa_mod():
    import torch
    import paper_1210_5093_amd as dfa
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dfa.lib()
    return dfa


@pytest.fixture(autouse=True)
def packed_matcher_by_default(monkeypatch):
    """Run every case through the packed-pair matcher wherever the DFA's layout
    allows it (the planner alone would pick the one-chunk-per-wave kernel for
    inputs under 4 MiB); tests that want the other kernel override this."""
    monkeypatch.setenv("DFA_KERNEL", "2")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def to_dev(x):
    import torch
    return torch.from_numpy(np.array(x, dtype=np.uint8, copy=True)).to("cuda")


def gpu_run(dfa, d, x, chunk=0, lookahead=1, start=None, boundaries=True):
    import torch
    t = to_dev(x)
    res, bnd = dfa.dfa_match_ex(d, t, start=start, chunk_len=chunk, lookahead=lookahead,
                                boundaries=boundaries)
    torch.cuda.synchronize()
    fin, acc, flags, nch = dfa.result_tuple(res)
    b = None if bnd is None else (bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF)
    return fin, acc, flags, nch, b


def check(dfa, w, x, chunk=0, lookahead=1, start=None, boundaries=True):
    """Run on the GPU and compare everything with the oracle."""
    d = dfa.DFA.from_workload(w)
    s0 = w.q0 if start is None else start
    fin, acc, flags, nch, b = gpu_run(dfa, d, x, chunk, lookahead, start, boundaries)
    ofin, _ = oracle.walk(w.delta, w.byte_to_symbol, s0, x)
    oacc = oracle.accepts(ofin, w.accepting)
    assert flags == 0, f"flags {flags}"
    assert (fin, acc) == (ofin, oacc), f"gpu {(fin, acc)} oracle {(ofin, oacc)}"
    if boundaries:
        used_chunk, n_ch = dfa.dfa_plan_chunks(d, len(x), chunk, lookahead)
        assert nch == n_ch
        probes = [min(i * used_chunk, len(x)) for i in range(nch + 1)]
        _, ps = oracle.walk(w.delta, w.byte_to_symbol, s0, x, probes=probes)
        bad = np.nonzero(b != ps)[0]
        assert bad.size == 0, f"boundary mismatch at chunks {bad[:10]}: {b[bad[:10]]} vs {ps[bad[:10]]}"
    d.close()
    return fin, acc, nch


# ---------------------------------------------------------------------------
# The paper's worked examples
# ---------------------------------------------------------------------------
def golden_workload(name):
    from workloads.dfas import DFA as W
    g = load_golden(name)
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    for i, ch in enumerate(g["symbols"]):
        b2s[ord(ch)] = i
    return g, W(np.asarray(g["delta"], dtype=np.uint32), g["q0"],
                np.asarray(g["accepting"], dtype=np.uint32), b2s, name)


def test_motivating_example_printed_values(dfa_mod):
    g, w = golden_workload("motivating_dfa.json")
    x = np.frombuffer(g["input"].encode(), dtype=np.uint8)
    d = dfa_mod.DFA.from_workload(w)
    fin, acc, flags, nch, b = gpu_run(dfa_mod, d, x, chunk=4)
    assert flags == 0 and nch == 3
    assert fin == g["printed"]["final_state"] and acc == g["printed"]["accepted"]
    assert b.tolist() == g["printed"]["boundary_states"]
    info = d.info()
    assert info.imax == g["printed"]["imax"] and info.num_absorbing == 1


@pytest.mark.parametrize("chunk", [1, 2, 3, 5, 7, 12, 18, 64])
def test_example_dfa_all_chunkings(dfa_mod, chunk):
    g, w = golden_workload("example_dfa.json")
    for key in ("input36", "input20"):
        x = np.frombuffer(g[key].encode(), dtype=np.uint8)
        fin, acc, _ = check(dfa_mod, w, x, chunk=chunk)
        assert fin == g["derived"]["final_state_" + key]


# ---------------------------------------------------------------------------
# C1: 16-state random DFA over bytes, 1 MiB
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_c1_full_size(dfa_mod, seed):
    w = configs.c1_dfa(seed)
    x = configs.c1_input()
    say("C1 seed", seed)
    check(dfa_mod, w, x)                    # planner chunking
    check(dfa_mod, w, x, chunk=4099)        # ragged tail


@pytest.mark.parametrize("chunk", [1, 63, 64, 65, 1000, 65536, 1 << 20, 1 << 21])
def test_c1_chunk_lengths(dfa_mod, chunk):
    w = configs.c1_dfa(1)
    x = configs.c1_input(300_001)
    check(dfa_mod, w, x, chunk=chunk)


def test_c1_lookahead_ablation_matches(dfa_mod):
    """Algorithm 2 (every chunk from all states) and Algorithm 3 (initial-state
    sets) give the same result as the sequential walk."""
    w = configs.c1_dfa(2)
    x = configs.c1_input(200_000)
    a = check(dfa_mod, w, x, chunk=777, lookahead=0)
    b = check(dfa_mod, w, x, chunk=777, lookahead=1)
    assert a == b


# ---------------------------------------------------------------------------
# C2: ~300-state protein DFA, residues
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("chunk", [0, 100, 4096, 5000, 65536])
def test_c2_prefix_many_chunks(dfa_mod, chunk):
    w = configs.c2_dfa()
    x = configs.c2_input(3 * (1 << 20) + 17)
    check(dfa_mod, w, x, chunk=chunk)


def test_c2_full_size_bench_configuration(dfa_mod):
    """256 MiB, planner chunking as timed by bench.py: final state, accept and
    every boundary state."""
    w = configs.c2_dfa()
    x = configs.c2_input()
    say("C2 full", x.size)
    check(dfa_mod, w, x)


@pytest.mark.parametrize("look,chunk,kw", [
    (6, 1024, {"interleave": True}),     # the autotuner's setting on the box
    (6, 1024, {}),
    (5, 2048, {}),
    (5, 2048, {"interleave": True, "rounds": 2}),
    (5, 1536, {}),                        # chunks of a multiple of 48
    (6, 1024, {"chunk_lanes": True}),
])
def test_c2_full_size_tuned_settings(dfa_mod, look, chunk, kw):
    """256 MiB in the settings the autotuner chooses between on the bench
    workload: final state, accept and the state at every chunk boundary."""
    import torch
    w = configs.c2_dfa()
    x = configs.c2_input()
    n = x.size
    probes = list(range(0, n, chunk)) + [n]
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    d = dfa_mod.DFA.from_workload(w)
    dev = torch.from_numpy(x).to("cuda")
    say("C2 full", look, chunk, kw)
    res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=chunk, lookahead=look, boundaries=True, **kw)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res) == (fin, oracle.accepts(fin, w.accepting), 0, len(probes) - 1)
    b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(b, ps.astype(np.int64))
    d.close()


def test_c2_ablation_all_states(dfa_mod):
    w = configs.c2_dfa()
    x = configs.c2_input(1 << 20)
    check(dfa_mod, w, x, chunk=8192, lookahead=0)


# ---------------------------------------------------------------------------
# C3 shapes at moderate size (the 10 GiB runs are in test_gpu_large.py)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("chunk", [4096, 65536, 1 << 20])
def test_c3_protein_1297_states(dfa_mod, chunk):
    w = configs.c3_protein_dfa()
    x = configs.c3_protein_input(16 * (1 << 20) + 3)
    say("C3 protein chunk", chunk)
    check(dfa_mod, w, x, chunk=chunk)


@pytest.mark.parametrize("chunk", [4096, 65536, 1 << 20])
def test_c3_byte_512_states(dfa_mod, chunk):
    w = configs.c3_byte_dfa()
    x = configs.c3_byte_input(16 * (1 << 20) + 5)
    say("C3 byte chunk", chunk)
    check(dfa_mod, w, x, chunk=chunk)


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_empty_and_tiny_inputs(dfa_mod):
    w = configs.c1_dfa(3)
    for n in (0, 1, 2, 63, 64, 65):
        x = configs.c1_input(n) if n else np.zeros(0, dtype=np.uint8)
        check(dfa_mod, w, x, chunk=16)
        check(dfa_mod, w, x)


def test_explicit_start_state_resumes_a_stream(dfa_mod):
    """Matching w = u v in two calls (the second starting in the first's final
    state) equals matching w at once (associativity of Eq. 9)."""
    import torch
    w = configs.c2_dfa()
    x = configs.c2_input(500_000)
    d = dfa_mod.DFA.from_workload(w)
    r1 = dfa_mod.result_tuple(dfa_mod.dfa_match_async(d, to_dev(x[:123_457])))
    r2 = dfa_mod.result_tuple(dfa_mod.dfa_match_async(d, to_dev(x[123_457:]), start=r1[0]))
    whole = dfa_mod.result_tuple(dfa_mod.dfa_match_async(d, to_dev(x)))
    torch.cuda.synchronize()
    assert r2[:3] == whole[:3]
    ofin, _ = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x)
    assert whole[0] == ofin
    for s in (0, 7, w.num_states - 1):
        check(dfa_mod, w, x[:50_000], chunk=999, start=s)


@pytest.mark.parametrize("pos", [0, 1, 999, 1000, 1001, 4095, 4096, 49_999])
def test_invalid_byte_is_reported(dfa_mod, pos):
    w = configs.c2_dfa()
    x = configs.c2_input(50_000).copy()
    x[pos] = ord("B")   # not an amino-acid letter
    with pytest.raises(oracle.InvalidSymbol):
        oracle.walk(w.delta, w.byte_to_symbol, w.q0, x)
    d = dfa_mod.DFA.from_workload(w)
    fin, acc, flags, nch, _ = gpu_run(dfa_mod, d, x, chunk=1000, boundaries=False)
    assert flags & dfa_mod.FLAG_SYMBOL
    with pytest.raises(dfa_mod.DFAError) as ei:
        dfa_mod.dfa_match(d, x)
    assert ei.value.status == dfa_mod.DFA_E_SYMBOL


def test_anchored_pattern_reaches_error_state(dfa_mod):
    """Anchored pattern DFA: the non-accepting sink (q_e) is reached early and
    carried through every later chunk unchanged."""
    pd = patterns.pattern_dfa(32, contains=False)
    w = from_pattern(pd)
    x = configs.c2_input(200_000)
    fin, acc, _ = check(dfa_mod, w, x, chunk=333)
    assert oracle.absorbing(w.delta)[fin]


def test_empty_initial_state_set(dfa_mod):
    """A class whose every transition enters an absorbing state has an empty
    I_sigma: chunks after it have no lanes and are still scanned."""
    from workloads.dfas import DFA as W
    rng = np.random.default_rng(5)
    delta = rng.integers(0, 6, (7, 4)).astype(np.uint32)
    delta[6, :] = 6          # state 6 absorbing
    delta[:, 3] = 6          # symbol 3 always leads into it
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    b2s[:4] = np.arange(4)
    w = W(delta, 0, np.array([1, 6], dtype=np.uint32), b2s, "empty-iset")
    x = rng.integers(0, 3, 20_000).astype(np.uint8)
    x[::997] = 3
    check(dfa_mod, w, x, chunk=50)
    check(dfa_mod, w, x, chunk=997)


def test_single_state_and_two_symbol_dfas(dfa_mod):
    from workloads.dfas import DFA as W
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    b2s[:2] = [0, 1]
    one = W(np.zeros((1, 2), dtype=np.uint32), 0, np.array([0], dtype=np.uint32), b2s, "one")
    x = np.random.default_rng(1).integers(0, 2, 10_000).astype(np.uint8)
    check(dfa_mod, one, x, chunk=128)
    parity = W(np.array([[0, 1], [1, 0]], dtype=np.uint32), 0, np.array([1], dtype=np.uint32),
               b2s, "parity")
    check(dfa_mod, parity, x, chunk=100)


def test_random_dfas_many_shapes(dfa_mod):
    rng = np.random.default_rng(2024)
    for k in range(12):
        q = int(rng.integers(2, 700))
        if k % 2:
            w = random_dfa(k, q, int(rng.integers(2, 40)), 3)
            x = rng.integers(0, w.num_symbols, 100_000).astype(np.uint8)
        else:
            qq = min(q, 500)
            w = column_dfa(k, k + 1, qq, int(rng.integers(2, 64)))
            x = streams.uniform_bytes(k, 100_000)
        say("random shape", k, w.num_states, w.num_symbols)
        check(dfa_mod, w, x, chunk=int(rng.integers(50, 5000)))


def test_host_entry_point_matches(dfa_mod):
    w = configs.c2_dfa()
    x = configs.c2_input(1 << 20)
    d = dfa_mod.DFA.from_workload(w)
    assert dfa_mod.dfa_match(d, x) == oracle.membership(w.delta, w.byte_to_symbol, w.q0,
                                                        w.accepting, x)
    assert dfa_mod.dfa_match(d, b"") == (w.q0, oracle.accepts(w.q0, w.accepting))


def test_batch_equals_individual(dfa_mod):
    import torch
    ws = [configs.c1_dfa(1), configs.c2_dfa(), configs.c3_byte_dfa()]
    ds = [dfa_mod.DFA.from_workload(w) for w in ws]
    rng = np.random.default_rng(3)
    pairs, xs = [], []
    for i in range(20):
        k = i % 3
        n = int(rng.integers(0, 300_000))
        x = configs.c2_input(n, first=i * 1000) if k == 1 else streams.uniform_bytes(i, n)
        pairs.append(k)
        xs.append(x)
    ins = [to_dev(x) for x in xs]
    res = dfa_mod.dfa_match_batch([ds[k] for k in pairs], ins).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    torch.cuda.synchronize()
    for i, (k, x) in enumerate(zip(pairs, xs)):
        ofin, oacc = oracle.membership(ws[k].delta, ws[k].byte_to_symbol, ws[k].q0,
                                       ws[k].accepting, x)
        assert (res[i, 0], bool(res[i, 1]), res[i, 2]) == (ofin, oacc, 0), i


# ---------------------------------------------------------------------------
# Both matcher kernels: packed pairs (default where the layout fits) and one
# chunk per wavefront (forced with DFA_KERNEL=1; the only one for tables that
# need more than 64 KiB of LDS)
# ---------------------------------------------------------------------------
@pytest.fixture
def one_chunk_per_wave(monkeypatch):
    monkeypatch.setenv("DFA_KERNEL", "1")


@pytest.mark.parametrize("chunk", [0, 1000, 4096])
def test_first_generation_kernel_c2_and_c1(dfa_mod, one_chunk_per_wave, chunk):
    check(dfa_mod, configs.c2_dfa(), configs.c2_input(2 * (1 << 20) + 9), chunk=chunk)
    check(dfa_mod, configs.c1_dfa(4), configs.c1_input(300_007), chunk=chunk)


def test_first_generation_kernel_large_sets(dfa_mod, one_chunk_per_wave):
    check(dfa_mod, configs.c3_protein_dfa(), configs.c3_protein_input(4 * (1 << 20) + 1),
          chunk=65536)


def test_planner_default_small_and_large(dfa_mod, monkeypatch):
    """Without an override: small inputs take the one-chunk-per-wave kernel,
    large ones the packed kernel; both agree with the oracle."""
    monkeypatch.delenv("DFA_KERNEL", raising=False)
    check(dfa_mod, configs.c2_dfa(), configs.c2_input(1 << 20))
    check(dfa_mod, configs.c2_dfa(), configs.c2_input(6 * (1 << 20) + 3))


def test_layouts_reported(dfa_mod):
    # residue alphabets (bytes below 128) get byte-indexed rows (3); the
    # 1297-state table needs rows of 50 bytes to stay inside 64 KiB
    assert dfa_mod.DFA.from_workload(configs.c2_dfa()).info().packed_layout == 3
    assert dfa_mod.DFA.from_workload(configs.c3_protein_dfa()).info().packed_layout == 3
    assert dfa_mod.DFA.from_workload(configs.c3_byte_dfa()).info().packed_layout == 2
    assert dfa_mod.DFA.from_workload(configs.c1_dfa(1)).info().packed_layout == 2
    # two-symbol tables: C2's 8 classes give 42 distinct pair columns; the
    # 1297-state table would not fit 16-bit entries, 64 or 256 classes too many
    assert dfa_mod.DFA.from_workload(configs.c2_dfa()).info().pair_columns == 42
    assert dfa_mod.DFA.from_workload(configs.c3_protein_dfa()).info().pair_columns == 0
    assert dfa_mod.DFA.from_workload(configs.c3_byte_dfa()).info().pair_columns == 0
    assert dfa_mod.DFA.from_workload(configs.c1_dfa(1)).info().pair_columns == 0


def test_table_beyond_64k_uses_first_generation_kernel(dfa_mod):
    """700 states x 80 classes = 112 KB class-major table: no packed layout
    fits 16-bit codes, so every chunk goes through the one-chunk-per-wave path."""
    w = column_dfa(21, 22, 700, 80)
    d = dfa_mod.DFA.from_workload(w)
    assert d.info().packed_layout == 0 and d.info().table_bytes > 65536
    x = streams.uniform_bytes(21, 1_000_003)
    check(dfa_mod, w, x)
    check(dfa_mod, w, x, chunk=3333)


@pytest.mark.parametrize("offset", [1, 3, 8, 15])
def test_unaligned_device_input(dfa_mod, offset):
    """Input tensors that start at any byte offset (torch slices)."""
    import torch
    w = configs.c2_dfa()
    x = configs.c2_input(400_000 + offset)
    t = to_dev(x)[offset:]
    d = dfa_mod.DFA.from_workload(w)
    r = dfa_mod.result_tuple(dfa_mod.dfa_match_async(d, t))
    torch.cuda.synchronize()
    assert r[:3] == (*oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x[offset:]), 0)


# ---------------------------------------------------------------------------
# Multi-symbol reverse lookahead (Eq. 13), exact per-chunk image sets
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("r", [2, 3, 4, 8, 16])
def test_multi_symbol_lookahead_c2(dfa_mod, r):
    w = configs.c2_dfa()
    x = configs.c2_input(3 * (1 << 20) + 11)
    check(dfa_mod, w, x, chunk=0, lookahead=r)
    check(dfa_mod, w, x, chunk=4099, lookahead=r)


@pytest.mark.parametrize("r", [2, 4, 64])
def test_multi_symbol_lookahead_other_dfas(dfa_mod, r):
    check(dfa_mod, configs.c3_protein_dfa(), configs.c3_protein_input(2 * (1 << 20) + 1),
          chunk=8192, lookahead=r)
    check(dfa_mod, configs.c1_dfa(2), configs.c1_input(400_000), chunk=1000, lookahead=r)
    check(dfa_mod, configs.c3_byte_dfa(), configs.c3_byte_input(1 << 20), chunk=4096, lookahead=r)
    pd = from_pattern(patterns.pattern_dfa(32, contains=False))
    check(dfa_mod, pd, configs.c2_input(300_000), chunk=777, lookahead=r)


@pytest.mark.parametrize("chunk", [1, 2, 3, 5, 7])
def test_lookahead_longer_than_chunks(dfa_mod, chunk):
    """r larger than the chunk length: the lookahead string spans earlier
    chunks, and chunks with p < r use r' = p (the whole prefix)."""
    g, w = golden_workload("example_dfa.json")
    x = np.frombuffer(g["input36"].encode(), dtype=np.uint8)
    for r in (2, 4, 9):
        fin, acc, _ = check(dfa_mod, w, x, chunk=chunk, lookahead=r)
        assert fin == g["derived"]["final_state_input36"]
    check(dfa_mod, configs.c2_dfa(), configs.c2_input(20_000), chunk=chunk * 13, lookahead=6)


@pytest.mark.parametrize("chunk", [1, 2, 3, 5])
def test_chunks_shorter_than_lookahead_large_sets(dfa_mod, chunk):
    """Chunks shorter than r: chunk 1's lookahead has only `chunk` symbols,
    and sets of fewer symbols can be larger than the r-symbol sets (Lemma,
    Section 4.3), so maps and tiles are sized for the shortest lookahead."""
    d = dfa_mod.DFA.from_workload(configs.c3_byte_dfa())
    plan = dfa_mod.dfa_plan(d, 20_000, chunk, 2)
    assert plan.set_max >= d.info().imax if chunk == 1 else True
    d.close()
    check(dfa_mod, configs.c3_byte_dfa(), configs.c3_byte_input(20_000), chunk=chunk, lookahead=2)
    check(dfa_mod, configs.c3_protein_dfa(), configs.c3_protein_input(20_001), chunk=chunk,
          lookahead=4)
    check(dfa_mod, configs.c2_dfa(), configs.c2_input(20_002), chunk=chunk, lookahead=6)


def test_lookahead_shrinks_sets_and_keeps_result(dfa_mod):
    """Lemma (Section 4.3): more lookahead never enlarges a start set, so the
    result is unchanged and the work (lookups) does not grow."""
    import bench
    w = configs.c2_dfa()
    x = configs.c2_input(1 << 20)
    work = [bench.algorithmic_lookups(w, x, 4096, r) for r in (1, 2, 4, 8)]
    assert all(a >= b for a, b in zip(work, work[1:]))
    res = {check(dfa_mod, w, x, chunk=4096, lookahead=r) for r in (0, 1, 2, 4, 8)}
    assert len(res) == 1


@pytest.mark.parametrize("pos", [4095, 4090, 8191])
def test_invalid_byte_inside_lookahead_window(dfa_mod, pos):
    w = configs.c2_dfa()
    x = configs.c2_input(50_000).copy()
    x[pos] = ord("Z")
    d = dfa_mod.DFA.from_workload(w)
    import torch
    res, _ = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=4096, lookahead=8)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL


# ---------------------------------------------------------------------------
# Precomputed multi-symbol sets (Eq. 13) against the oracle's definition
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["c2", "c1", "c3b", "motiv", "example"])
def test_precomputed_lookahead_sets_match_eq13(dfa_mod, which):
    if which == "c2":
        w = configs.c2_dfa()
    elif which == "c1":
        w = configs.c1_dfa(3)
    elif which == "c3b":
        w = configs.c3_byte_dfa()
    else:
        _, w = golden_workload("motivating_dfa.json" if which == "motiv" else "example_dfa.json")
    d = dfa_mod.DFA.from_workload(w)
    r0 = d.info().lookahead_tables
    assert r0 >= 1
    ab = oracle.absorbing(w.delta)
    valid = np.nonzero(w.byte_to_symbol < w.num_symbols)[0].astype(np.uint8)
    rng = np.random.default_rng(7)
    for k in range(1, r0 + 1):
        for _ in range(40):
            u = rng.choice(valid, k)
            expect = np.nonzero(oracle.iset_word(w.delta, w.byte_to_symbol[u], ab))[0].tolist()
            assert dfa_mod.dfa_lookahead_set(d, u.tobytes()) == expect, (k, u)
    if which == "motiv":
        assert dfa_mod.dfa_lookahead_set(d, b"a") == [0]
        assert dfa_mod.dfa_lookahead_set(d, b"b") == [1]
    if which == "example":
        assert dfa_mod.dfa_lookahead_set(d, b"a") == [1, 3]
        assert dfa_mod.dfa_lookahead_set(d, b"b") == [2, 3]


@pytest.mark.parametrize("r", [2, 3, 5, 7, 9, 12])
def test_precomputed_and_window_lookahead_c2_bench_size(dfa_mod, r):
    """Lookahead within the precomputed tables (r <= r0) and beyond them (window
    pass from the r0-symbol sets), at the bench size with planner chunking."""
    w = configs.c2_dfa()
    x = configs.c2_input(32 * (1 << 20) + 5)
    check(dfa_mod, w, x, lookahead=r)


# ---------------------------------------------------------------------------
# Early exit at absorbing states (the walks of a wavefront stop once all of
# them sit in an absorbing state): results and boundary states unchanged.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,contains", [(32, False), (7, False), (32, True), (5825, True)])
@pytest.mark.parametrize("look", [1, 4])
def test_early_exit_matches_oracle(dfa_mod, seed, contains, look):
    import torch
    w = from_pattern(patterns.pattern_dfa(seed, contains=contains))
    n = 6 << 20
    x = configs.c2_input(n, seed=900 + seed)
    probes = list(range(0, n + 1, 4096))
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    acc = oracle.accepts(fin, w.accepting)
    d = dfa_mod.DFA.from_workload(w)
    dev = torch.from_numpy(x).to("cuda")
    for ex in (False, True):
        res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=4096, lookahead=look, boundaries=True,
                                        early_exit=ex)
        torch.cuda.synchronize()
        assert dfa_mod.result_tuple(res)[:3] == (fin, acc, 0), ex
        b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        assert np.array_equal(b, ps.astype(np.int64)), ex
    d.close()


def test_early_exit_ragged_and_invalid(dfa_mod):
    import torch
    w = from_pattern(patterns.pattern_dfa(32, contains=False))
    d = dfa_mod.DFA.from_workload(w)
    for n in (4 << 20, (4 << 20) + 77):
        x = configs.c2_input(n, seed=n % 1000).copy()
        fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
        res, _ = dfa_mod.dfa_match_ex(d, torch.from_numpy(x).to("cuda"), chunk_len=1024,
                                      early_exit=True)
        torch.cuda.synchronize()
        assert dfa_mod.result_tuple(res)[:3] == (fin, acc, 0)
        x[n - 5] = ord("#")
        res, _ = dfa_mod.dfa_match_ex(d, torch.from_numpy(x).to("cuda"), chunk_len=1024,
                                      early_exit=True)
        torch.cuda.synchronize()
        assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL
    d.close()


# ---------------------------------------------------------------------------
# Tree composition: chunk counts around the group size (up to 1024 maps per
# group) and its powers, for one- and five-symbol lookahead.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nch", [1, 2, 3, 1023, 1024, 1025, 2047, 2049, 1024 * 1024 + 3])
@pytest.mark.parametrize("look", [1, 5])
def test_compose_tree_group_edges(dfa_mod, nch, look):
    import torch
    w = configs.c2_dfa()
    C = 256
    n = nch * C - (C // 2 if nch % 2 else 0)     # odd counts end with a ragged chunk
    x = configs.c2_input(n, seed=nch % 977)
    step = max(C, (n // 64) // C * C)
    probes = list(range(0, n + 1, step))
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    acc = oracle.accepts(fin, w.accepting)
    d = dfa_mod.DFA.from_workload(w)
    res, bnd = dfa_mod.dfa_match_ex(d, torch.from_numpy(x).to("cuda"), chunk_len=C,
                                    lookahead=look, boundaries=True)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res) == (fin, acc, 0, (n + C - 1) // C)
    b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(b[np.array(probes) // C], ps.astype(np.int64))
    d.close()


@pytest.mark.parametrize("look,single", [(1, False), (5, False), (5, True), (3, True)])
def test_translation_pass(dfa_mod, look, single):
    """The translation (or, for direct tables, validation) pass: results,
    boundaries, a byte outside Sigma in the middle and at the very end, and a
    clean call after a flagged one on the same workspace."""
    import torch
    w = configs.c2_dfa()
    C = 2048
    n = 6 * (1 << 20) + 4096 * 3
    x = configs.c2_input(n, seed=40 + look).copy()
    probes = list(range(0, n + 1, 32 * C))
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    d = dfa_mod.DFA.from_workload(w)
    plan = dfa_mod.dfa_plan(d, n, C, look, single_step=single)
    assert plan.kernel == 1 and int(plan.symbols_per_step) == (1 if single else 2)
    dev = torch.from_numpy(x).to("cuda")
    res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=C, lookahead=look, single_step=single,
                                    boundaries=True)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[:3] == (fin, oracle.accepts(fin, w.accepting), 0)
    b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(b[np.array(probes) // C], ps.astype(np.int64))
    for pos in (n // 2 + 7, n - 1):
        y = x.copy()
        y[pos] = ord("#")
        res, _ = dfa_mod.dfa_match_ex(d, torch.from_numpy(y).to("cuda"), chunk_len=C,
                                      lookahead=look, single_step=single)
        torch.cuda.synchronize()
        assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL, pos
    res, _ = dfa_mod.dfa_match_ex(d, dev, chunk_len=C, lookahead=look, single_step=single)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[:3] == (fin, oracle.accepts(fin, w.accepting), 0)
    d.close()


# ---------------------------------------------------------------------------
# Direct tables (rows indexed by the byte itself; the matcher reads the raw
# input and a validation pass replaces the translation): every kind of byte
# outside Sigma, at chunk and block edges, on the whole-block walk (chunk
# 2048) with one- and five-symbol lookahead.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("byte", [ord("B"), ord("0"), ord("z"), 0x00, 0x7F, 0x80, 0xC1, 0xFF])
@pytest.mark.parametrize("pos", [0, 2047, 2048, 100_000, 200_002])
def test_direct_table_invalid_bytes(dfa_mod, byte, pos):
    w = configs.c2_dfa()
    x = configs.c2_input(200_003).copy()
    x[pos] = byte
    with pytest.raises(oracle.InvalidSymbol):
        oracle.walk(w.delta, w.byte_to_symbol, w.q0, x)
    d = dfa_mod.DFA.from_workload(w)
    assert d.info().packed_layout == 3
    for look in (1, 5):
        _, _, flags, _, _ = gpu_run(dfa_mod, d, x, chunk=2048, lookahead=look, boundaries=False)
        assert flags & dfa_mod.FLAG_SYMBOL, look
    d.close()


@pytest.mark.parametrize("n", [1, 15, 16, 17, 2047, 2049, 3 * 4096 + 5, 1_000_001])
@pytest.mark.parametrize("look", [1, 3, 5])
def test_direct_table_ragged_lengths(dfa_mod, n, look):
    """Raw input is read byte by byte past its last whole 16-byte block."""
    check(dfa_mod, configs.c2_dfa(), configs.c2_input(n, seed=40 + n % 97), chunk=2048,
          lookahead=look)


def test_direct_table_full_ascii_window(dfa_mod):
    """128 symbols (bytes 0..127) with 128 distinct columns: too many classes
    for one-byte class codes, so only the direct table gives a state-major
    layout (rows of 65 dwords)."""
    from workloads.dfas import DFA as W
    rng = np.random.default_rng(11)
    nq = 200
    delta = rng.integers(0, nq, (nq, 128)).astype(np.uint32)
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    b2s[:128] = np.arange(128)
    w = W(delta, 0, np.array([1, 2, 3], dtype=np.uint32), b2s, "ascii-200")
    d = dfa_mod.DFA.from_workload(w)
    assert d.info().packed_layout == 3
    d.close()
    x = rng.integers(0, 128, 300_001).astype(np.uint8)
    for look in (1, 2):
        check(dfa_mod, w, x, chunk=4096, lookahead=look)
    x[123_456] = 0x80
    d = dfa_mod.DFA.from_workload(w)
    assert gpu_run(dfa_mod, d, x, chunk=4096, boundaries=False)[2] & dfa_mod.FLAG_SYMBOL
    d.close()


@pytest.mark.parametrize("offset", [0, 4, 8])
def test_direct_table_early_exit_c3_protein(dfa_mod, offset):
    """Rows of 50 bytes (the absorbing bitmap is then indexed in 2-byte units),
    early exit on and off; a misaligned view takes the translating path.  Both
    1297/1298-state DFAs: the early-sink one (walks absorbed within a few KiB)
    and the configured one (never absorbed)."""
    import torch
    for seed in (configs.C3_EARLY_SINK_SEED, configs.C3_PATTERN_SEED):
        direct_table_early_exit_case(dfa_mod, configs.c3_protein_dfa(seed), offset)


def direct_table_early_exit_case(dfa_mod, w, offset):
    import torch
    n = 3 << 20
    x = configs.c3_protein_input(n + offset)[offset:]
    probes = list(range(0, n + 1, 4096))
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    acc = oracle.accepts(fin, w.accepting)
    d = dfa_mod.DFA.from_workload(w)
    dev = to_dev(configs.c3_protein_input(n + offset))[offset:]
    for ex in (False, True):
        for look in (1, 4):
            res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=4096, lookahead=look,
                                            boundaries=True, early_exit=ex)
            torch.cuda.synchronize()
            assert dfa_mod.result_tuple(res)[:3] == (fin, acc, 0), (ex, look)
            b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(b, ps.astype(np.int64)), (ex, look)
    d.close()


# ---------------------------------------------------------------------------
# Two-symbol steps (a table of delta(delta(s, a), b) over pair columns; one
# code per two input bytes): odd lengths end on a one-symbol column, chunk
# boundaries stay exact, invalid bytes at even and odd positions are flagged.
# DFA_PAIRS=0 gives the one-symbol path on the same inputs.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pairs", ["1", "0"])
@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 4095, 4097, 1_000_001, 3 << 20])
@pytest.mark.parametrize("look", [1, 5])
def test_two_symbol_steps_lengths(dfa_mod, monkeypatch, pairs, n, look):
    if pairs == "0":
        monkeypatch.setenv("DFA_PAIRS", "0")
    w = configs.c2_dfa()
    x = configs.c2_input(n, seed=70 + n % 89)
    for chunk in (0, 64, 2048):
        check(dfa_mod, w, x, chunk=chunk, lookahead=look)


@pytest.mark.parametrize("byte", [ord("J"), ord("0"), 0x80, 0xC1, 0xE1])
@pytest.mark.parametrize("pos", [0, 1, 30, 31, 2047, 2048, 99_998, 99_999, 100_000])
def test_two_symbol_steps_invalid_bytes(dfa_mod, byte, pos):
    """Bytes outside Sigma below and above 128 (0xC1 & 0x7F is 'A'), on
    either side of a pair and as a lone last byte."""
    w = configs.c2_dfa()
    x = configs.c2_input(100_001).copy()
    x[pos] = byte
    d = dfa_mod.DFA.from_workload(w)
    for look in (1, 4):
        assert gpu_run(dfa_mod, d, x, chunk=2048, lookahead=look, boundaries=False)[2] & \
            dfa_mod.FLAG_SYMBOL
    d.close()


@pytest.mark.parametrize("seed,contains", [(32, False), (7, False), (7, True)])
def test_two_symbol_steps_early_exit_and_other_dfas(dfa_mod, seed, contains):
    import torch
    w = from_pattern(patterns.pattern_dfa(seed, contains=contains))
    d = dfa_mod.DFA.from_workload(w)
    assert d.info().pair_columns > 0
    n = (5 << 20) + 7
    x = configs.c2_input(n, seed=300 + seed)
    probes = list(range(0, n, 1024)) + [n]
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    acc = oracle.accepts(fin, w.accepting)
    dev = torch.from_numpy(x).to("cuda")
    for ex in (False, True):
        for look in (1, 3):
            res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=1024, lookahead=look,
                                            boundaries=True, early_exit=ex)
            torch.cuda.synchronize()
            assert dfa_mod.result_tuple(res)[:3] == (fin, acc, 0), (ex, look)
            b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(b, ps.astype(np.int64)), (ex, look)
    d.close()


def test_two_symbol_steps_random_small_alphabets(dfa_mod):
    """Random byte-alphabet DFAs with 2..60 distinct columns: up to 10
    columns give at most 110 pair columns (a pair table when the states fit
    16-bit entries), more columns too many."""
    rng = np.random.default_rng(77)
    for t, k in enumerate([2, 3, 4, 5, 6, 8, 10, 10, 11, 20, 60, 7]):
        nq = int(rng.integers(2, 300))
        w = column_dfa(500 + t, 600 + t, nq, k)
        d = dfa_mod.DFA.from_workload(w)
        pc = d.info().pair_columns
        d.close()
        x = streams.uniform_bytes(700 + t, int(rng.integers(50_000, 400_000)))
        say(f"random dfa {t}: Q={nq} K={k} pair columns {pc}")
        check(dfa_mod, w, x, chunk=512, lookahead=1)
        check(dfa_mod, w, x, chunk=4096, lookahead=2)


# ---------------------------------------------------------------------------
# Two-symbol steps at chunk lengths of a multiple of 48 and 32: every
# remainder of the length mod 2, 3 and 48, ragged last chunks, boundary
# states, bytes outside Sigma at either place of a pair code, early exit,
# misaligned input and small random alphabets.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 47, 48, 49, 1535, 1536, 1537, 100_003, (3 << 20) + 2])
@pytest.mark.parametrize("look", [1, 5])
def test_pair_steps_lengths(dfa_mod, n, look):
    w = configs.c2_dfa()
    x = configs.c2_input(n, seed=90 + n % 97)
    d = dfa_mod.DFA.from_workload(w)
    assert d.info().pair_columns > 0
    for chunk in (0, 1536, 3072):
        plan = dfa_mod.dfa_plan(d, n, chunk, look)
        if plan.kernel == 1:
            assert plan.symbols_per_step == 2, chunk
        check(dfa_mod, w, x, chunk=chunk, lookahead=look)
    d.close()


@pytest.mark.parametrize("byte", [ord("J"), 0x80, 0xC1])
@pytest.mark.parametrize("pos", [0, 1, 2, 3, 46, 47, 48, 1535, 1536, 99_999, 100_000, 100_001,
                                 100_002])
def test_pair_steps_invalid_bytes(dfa_mod, byte, pos):
    """Bytes outside Sigma below and above 128 as the first and second byte of
    a code, at chunk and 48-byte edges and in the short last code."""
    w = configs.c2_dfa()
    x = configs.c2_input(100_003).copy()
    x[pos] = byte
    d = dfa_mod.DFA.from_workload(w)
    for look in (3, 5):
        assert dfa_mod.dfa_plan(d, x.size, 1536, look).symbols_per_step == 2
        assert gpu_run(dfa_mod, d, x, chunk=1536, lookahead=look, boundaries=False)[2] & \
            dfa_mod.FLAG_SYMBOL
    x[pos] = ord("A")
    fin, acc, flags, _, _ = gpu_run(dfa_mod, d, x, chunk=1536, lookahead=5, boundaries=False)
    ofin, _ = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x)
    assert (fin, flags) == (ofin, 0)
    d.close()


@pytest.mark.parametrize("seed,contains", [(32, True), (32, False), (7, False), (7, True)])
def test_pair_steps_1536_early_exit_and_other_dfas(dfa_mod, seed, contains):
    import torch
    w = from_pattern(patterns.pattern_dfa(seed, contains=contains))
    d = dfa_mod.DFA.from_workload(w)
    n = (5 << 20) + 7
    x = configs.c2_input(n, seed=310 + seed)
    probes = list(range(0, n, 1536)) + [n]
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    acc = oracle.accepts(fin, w.accepting)
    dev = torch.from_numpy(x).to("cuda")
    say(f"pattern {seed} contains={contains}: Q={w.num_states} "
        f"pair columns {d.info().pair_columns}")
    for ex in (False, True):
        for look in (1, 3, 5):
            res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=1536, lookahead=look,
                                            boundaries=True, early_exit=ex)
            torch.cuda.synchronize()
            assert dfa_mod.result_tuple(res)[:3] == (fin, acc, 0), (ex, look)
            b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(b, ps.astype(np.int64)), (ex, look)
    d.close()


@pytest.mark.parametrize("shift", [1, 5, 16])
def test_pair_steps_misaligned_input(dfa_mod, shift):
    import torch
    w = configs.c2_dfa()
    n = (2 << 20) + 5
    x = configs.c2_input(n, seed=95)
    probes = list(range(0, n, 3072)) + [n]
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    buf = torch.from_numpy(np.concatenate([np.full(shift, 65, np.uint8), x])).to("cuda")
    dev = buf[shift:]
    d = dfa_mod.DFA.from_workload(w)
    res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=3072, lookahead=5, boundaries=True)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[:3] == (fin, oracle.accepts(fin, w.accepting), 0)
    b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(b, ps.astype(np.int64))
    d.close()


def test_random_small_alphabets(dfa_mod):
    """Random byte-alphabet DFAs with 2..16 distinct columns (a pair table for
    up to 10 of them)."""
    rng = np.random.default_rng(78)
    for t, k in enumerate([2, 3, 4, 5, 6, 8, 12, 16]):
        nq = int(rng.integers(2, 200))
        w = column_dfa(800 + t, 900 + t, nq, k)
        d = dfa_mod.DFA.from_workload(w)
        pc = d.info().pair_columns
        d.close()
        x = streams.uniform_bytes(1000 + t, int(rng.integers(50_000, 400_000)))
        say(f"random dfa {t}: Q={nq} K={k} pair columns {pc}")
        check(dfa_mod, w, x, chunk=1536, lookahead=2)
        check(dfa_mod, w, x, chunk=4800, lookahead=1)


# ---------------------------------------------------------------------------
# Merged walks (DFA_MATCH_ROUNDS): after each round but the last, walks of a
# chunk in the same state continue as one.  Every boundary state must equal
# the oracle's for any round count, chunk length (32 bytes up, ragged last
# chunk), lookahead mode (0: all states, 1, precomputed 3, window 12) and
# table kind (class codes, direct rows, two-symbol steps, class-major).
# ---------------------------------------------------------------------------
def merged_cases():
    return [
        ("c2", lambda: (configs.c2_dfa(), configs.c2_input((3 << 20) + 5, seed=61))),
        ("c3p", lambda: (configs.c3_protein_dfa(), configs.c3_protein_input((2 << 20) + 17))),
        ("c3b", lambda: (configs.c3_byte_dfa(), configs.c3_byte_input((2 << 20) + 9))),
        ("c1", lambda: (configs.c1_dfa(2), configs.c1_input((1 << 20) + 3))),
        ("anchored", lambda: (from_pattern(patterns.pattern_dfa(32, contains=False)),
                              configs.c2_input((2 << 20) + 1, seed=62))),
        ("cols6", lambda: (column_dfa(91, 92, 150, 6), streams.uniform_bytes(93, (1 << 20) + 31))),
    ]


@pytest.mark.parametrize("case", [c[0] for c in merged_cases()])
@pytest.mark.parametrize("rounds", [1, 2, 3, 4])
def test_merged_rounds_match_oracle(dfa_mod, case, rounds):
    w, x = dict(merged_cases())[case]()
    n = x.size
    d = dfa_mod.DFA.from_workload(w)
    for chunk in (32, 96, 2048, 65536):
        for look in (1, 3):
            plan = dfa_mod.dfa_plan(d, n, chunk, look, rounds=rounds)
            say(f"{case}: rounds {rounds} (plan {plan.rounds}) chunk {chunk} r {look} "
                f"kernel {plan.kernel} sym/step {plan.symbols_per_step}")
            if plan.kernel == 1:
                # the last round must start inside a chunk
                want = rounds
                while want > 1 and 32 << (2 * (want - 2)) >= chunk:
                    want -= 1
                assert plan.rounds == want
            fin, acc, flags, nch, b = gpu_run(dfa_mod, d, x, chunk, look)
            # gpu_run uses the default (planner) rounds; run the requested ones
            # on the interleaved and the linear code stream
            import torch
            probes = [min(i * plan.chunk_len, n) for i in range(plan.num_chunks + 1)]
            ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
            assert (fin, acc) == (ofin, oracle.accepts(ofin, w.accepting))
            for ilv in (False, True):
                res, bnd = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=chunk, lookahead=look,
                                                boundaries=True, rounds=rounds, interleave=ilv)
                torch.cuda.synchronize()
                assert dfa_mod.result_tuple(res)[:3] == \
                    (ofin, oracle.accepts(ofin, w.accepting), 0), ilv
                bb = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
                bad = np.nonzero(bb != ps)[0]
                assert bad.size == 0, f"interleave {ilv} chunks {bad[:8]}: {bb[bad[:8]]} vs {ps[bad[:8]]}"
    d.close()


@pytest.mark.parametrize("rounds", [2, 4])
def test_merged_rounds_all_states_and_window(dfa_mod, rounds):
    """Lookahead 0 (every non-absorbing state starts each chunk) and 12 (the
    window pass beyond the precomputed sets)."""
    w = configs.c2_dfa()
    x = configs.c2_input((1 << 20) + 7, seed=63)
    for look in (0, 12):
        for chunk in (64, 4096):
            import torch
            d = dfa_mod.DFA.from_workload(w)
            res, bnd = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=chunk, lookahead=look,
                                            boundaries=True, rounds=rounds)
            torch.cuda.synchronize()
            n = x.size
            used, nch = dfa_mod.dfa_plan_chunks(d, n, chunk, look)
            probes = [min(i * used, n) for i in range(nch + 1)]
            ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
            assert dfa_mod.result_tuple(res)[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
            assert np.array_equal(bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF,
                                  ps.astype(np.int64))
            d.close()


@pytest.mark.parametrize("pos", [0, 31, 32, 33, 127, 128, 129, 4095, 77_777])
def test_merged_rounds_invalid_bytes(dfa_mod, pos):
    w = configs.c2_dfa()
    x = configs.c2_input(100_003, seed=64).copy()
    x[pos] = 0xC1
    d = dfa_mod.DFA.from_workload(w)
    import torch
    for rounds in (2, 3):
        res, _ = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=4096, lookahead=3, rounds=rounds)
        torch.cuda.synchronize()
        assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL
    d.close()


@pytest.mark.parametrize("case", ["c2", "c3b", "c1", "cols6"])
@pytest.mark.parametrize("single", [False, True])
def test_interleaved_codes_ragged(dfa_mod, case, single):
    """Chunk-interleaved code streams: chunk counts around multiples of 64
    (partial last group), ragged last chunk, one- and two-symbol codes."""
    import torch
    w, _ = dict(merged_cases())[case]()
    d = dfa_mod.DFA.from_workload(w)
    rng = np.random.default_rng(5)
    for nch, chunk in ((1, 64), (63, 64), (64, 96), (65, 128), (129, 2048), (200, 4096)):
        n = int((nch - 1) * chunk + rng.integers(1, chunk + 1))
        x = (configs.c2_input(n, seed=n % 97) if case == "c2" else
             streams.uniform_bytes(70 + nch, n) if case != "cols6" else
             streams.uniform_bytes(93, n))
        plan = dfa_mod.dfa_plan(d, n, chunk, 1, single_step=single, interleave=True)
        assert plan.kernel == 1 and plan.interleaved == 1 and plan.num_chunks == nch
        probes = [min(i * chunk, n) for i in range(nch + 1)]
        ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
        for rounds in (1, 2):
            res, bnd = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=chunk, lookahead=1,
                                            boundaries=True, rounds=rounds, single_step=single,
                                            interleave=True)
            torch.cuda.synchronize()
            assert dfa_mod.result_tuple(res)[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
            assert np.array_equal(bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF,
                                  ps.astype(np.int64)), (nch, chunk, rounds)
    d.close()


@pytest.mark.parametrize("case", [c[0] for c in merged_cases()])
def test_chunk_lanes_match_oracle(dfa_mod, case):
    """One chunk per lane with merged walks (DFA_MATCH_CHUNK_LANES): every
    boundary state equals the oracle's; sets too large for it fall back."""
    import torch
    w, x = dict(merged_cases())[case]()
    n = x.size
    d = dfa_mod.DFA.from_workload(w)
    used = 0
    for chunk in (32, 96, 512, 2048, 65536):
        for look in (1, 3, 5, 6):
            for single in (False, True):
                plan = dfa_mod.dfa_plan(d, n, chunk, look, chunk_lanes=True, single_step=single)
                used += plan.chunk_lanes
                res, bnd = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=chunk, lookahead=look,
                                                boundaries=True, chunk_lanes=True,
                                                single_step=single)
                torch.cuda.synchronize()
                probes = [min(i * plan.chunk_len, n) for i in range(plan.num_chunks + 1)]
                ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
                assert dfa_mod.result_tuple(res)[:3] == \
                    (ofin, oracle.accepts(ofin, w.accepting), 0), (chunk, look, single)
                bb = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
                bad = np.nonzero(bb != ps)[0]
                assert bad.size == 0, (chunk, look, single, bad[:8])
    say(f"{case}: chunk lanes used in {used} settings")
    if case in ("c2", "anchored", "c1"):
        assert used > 0
    d.close()


@pytest.mark.parametrize("pos", [0, 31, 32, 33, 1023, 100_000])
def test_chunk_lanes_invalid_bytes(dfa_mod, pos):
    import torch
    w = configs.c2_dfa()
    x = configs.c2_input(200_001, seed=66).copy()
    x[pos] = 0xC1
    d = dfa_mod.DFA.from_workload(w)
    for single in (False, True):
        res, _ = dfa_mod.dfa_match_ex(d, to_dev(x), chunk_len=1024, lookahead=5, chunk_lanes=True,
                                      single_step=single)
        torch.cuda.synchronize()
        assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL
    d.close()


@pytest.mark.parametrize("which", ["c3p", "c2"])
@pytest.mark.parametrize("offset", [0, 3])
def test_chunk_lanes_over_raw_input(dfa_mod, which, offset):
    """One chunk per lane over a direct table: each lane reads its own chunk of
    the raw input (16-byte aligned; offset 3 takes a linear translated stream
    instead).  Chunks of 32 bytes up with a ragged last chunk; every boundary
    state and the state maps equal the oracle's."""
    import torch
    from test_gpu_maps import check_maps
    if which == "c3p":
        w = configs.c3_protein_dfa()
        full = configs.c3_protein_input((3 << 20) + 21 + offset)
    else:
        w = configs.c2_dfa()
        full = configs.c2_input((3 << 20) + 21 + offset, seed=66)
    x = full[offset:]
    buf = to_dev(full)
    dev = buf[offset:]
    d = dfa_mod.DFA.from_workload(w)
    n = x.size
    # (start sets of at most 128 states: r = 4 for the large protein DFA)
    settings = ((32, 4), (1024, 4), (4096, 4), (65536, 4)) if which == "c3p" else \
        ((32, 4), (1024, 4), (4096, 3), (65536, 2))
    for chunk, look in settings:
        plan = dfa_mod.dfa_plan(d, n, chunk, look, chunk_lanes=True, single_step=True)
        assert plan.chunk_lanes == 1 and plan.interleaved == 0, (chunk, look)
        res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=chunk, lookahead=look, boundaries=True,
                                        chunk_lanes=True, single_step=True)
        torch.cuda.synchronize()
        probes = [min(i * chunk, n) for i in range(plan.num_chunks + 1)]
        ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
        assert dfa_mod.result_tuple(res)[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0)
        b = bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        bad = np.nonzero(b != ps)[0]
        assert bad.size == 0, (chunk, look, bad[:8])
        check_maps(dfa_mod, w, x, dev, d, chunk, look, expect=(ofin, oracle.accepts(ofin, w.accepting)),
                   chunk_lanes=True, single_step=True)
    x2 = x.copy()
    x2[n - 5] = ord("#")
    res, _ = dfa_mod.dfa_match_ex(d, to_dev(x2), chunk_len=1024, lookahead=4, chunk_lanes=True,
                                  single_step=True)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SYMBOL
    d.close()
