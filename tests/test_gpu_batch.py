"""Batched membership tests: many (DFA, string) pairs in one persistent launch.

Every record of a batch must equal the oracle's result for that pair alone
(final state, accept bit; tolerance 0), and equal what the single-string path
returns; a HIP-graph replay must give the same records.  The last test runs
the full batched configuration (1024 pairs, 5.7 GiB)."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from workloads import configs, from_pattern, patterns, streams

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def dfa_mod():
    import torch
    import paper_1210_5093_amd as dfa
    assert torch.cuda.is_available()
    dfa.lib()
    return dfa


def oracle_records(pairs, xs, threads=16):
    def one(k):
        w = pairs[k]
        try:
            fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, xs[k])
            return fin, int(acc), 0
        except oracle.InvalidSymbol:
            return None, None, 1
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(xs))))


def make(dfa_mod, wl):
    import torch
    cache, ds, xs, ins = {}, [], [], []
    for w, n, kind, seed in wl:
        if id(w) not in cache:
            cache[id(w)] = dfa_mod.DFA.from_workload(w)
        ds.append(cache[id(w)])
        x = configs.request_input(kind, seed, n)
        xs.append(x)
        ins.append(torch.from_numpy(x).to("cuda"))
    return ds, xs, ins


def check_records(res, expect):
    r = res.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    for k, (fin, acc, bad) in enumerate(expect):
        if bad:
            assert r[k, 2] & 1, k
        else:
            assert (r[k, 0], r[k, 1], r[k, 2]) == (fin, acc, 0), (k, r[k], fin, acc)


def test_small_batch_matches_oracle_and_graph_replay(dfa_mod):
    import torch
    wl = configs.batch_workload(count=96, seed=17, max_len=2 << 20)
    ds, xs, ins = make(dfa_mod, wl)
    pairs = [w for w, _, _, _ in wl]
    expect = oracle_records(pairs, xs)
    b = dfa_mod.Batch(ds, ins)
    res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
    b.run(res)
    torch.cuda.synchronize()
    check_records(res, expect)
    s = torch.cuda.Stream()
    for _ in range(3):
        res2 = torch.full((len(ds), 4), -1, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(s):
            b.graph_launch(res2, s)
        torch.cuda.synchronize()
        assert torch.equal(res, res2)
    # a graph replay sees new input contents behind the same pointers
    ins[0].copy_(torch.from_numpy(configs.request_input(wl[0][2], 999, ins[0].numel())))
    with torch.cuda.stream(s):
        b.graph_launch(res2, s)
    torch.cuda.synchronize()
    w0 = pairs[0]
    x0 = ins[0].cpu().numpy()
    fin0, acc0 = oracle.membership(w0.delta, w0.byte_to_symbol, w0.q0, w0.accepting, x0)
    assert (int(res2[0, 0]), int(res2[0, 1])) == (fin0, int(acc0))
    b.close()


def test_batch_equals_single_string_path(dfa_mod):
    import torch
    wl = configs.batch_workload(count=40, seed=23, max_len=1 << 20)
    ds, xs, ins = make(dfa_mod, wl)
    res = dfa_mod.dfa_match_batch(ds, ins)
    singles = torch.stack([dfa_mod.dfa_match_async(d, t) for d, t in zip(ds, ins)])
    torch.cuda.synchronize()
    assert torch.equal(res[:, :3], singles[:, :3])


def test_batch_edge_cases(dfa_mod):
    """Empty strings, a byte outside Sigma, one DFA repeated, explicit chunking."""
    import torch
    w = configs.c2_dfa()
    wb = configs.c3_byte_dfa()
    d, db = dfa_mod.DFA.from_workload(w), dfa_mod.DFA.from_workload(wb)
    xs = [np.zeros(0, np.uint8), configs.c2_input(1000), configs.c2_input(70_000).copy(),
          streams.uniform_bytes(5, 123_457), configs.c2_input(1)]
    xs[2][12_345] = ord("J")
    ds = [d, d, d, db, d]
    ins = [torch.from_numpy(np.array(x)).to("cuda") for x in xs]
    for chunk in (0, 1000, 4096):
        b = dfa_mod.Batch(ds, ins, chunk_len=chunk)
        res = torch.empty((5, 4), dtype=torch.int32, device="cuda")
        b.run(res)
        torch.cuda.synchronize()
        r = res.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        assert (r[0, 0], r[0, 2]) == (w.q0, 0)
        for k in (1, 3, 4):
            ww = ds[k] is db and wb or w
            fin, acc = oracle.membership(ww.delta, ww.byte_to_symbol, ww.q0, ww.accepting, xs[k])
            assert (r[k, 0], r[k, 1], r[k, 2]) == (fin, int(acc), 0), (chunk, k)
        assert r[2, 2] & dfa_mod.FLAG_SYMBOL
        b.close()


@pytest.fixture
def first_generation_batch(monkeypatch):
    """Batches created inside the test use one chunk per wavefront."""
    monkeypatch.setenv("DFA_BATCH_KERNEL", "1")


def test_first_generation_batch_matches_oracle(dfa_mod, first_generation_batch):
    import torch
    wl = configs.batch_workload(count=64, seed=31, max_len=2 << 20)
    ds, xs, ins = make(dfa_mod, wl)
    expect = oracle_records([w for w, _, _, _ in wl], xs)
    b = dfa_mod.Batch(ds, ins)
    chunk, nch = b.info()
    res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
    b.run(res)
    torch.cuda.synchronize()
    check_records(res, expect)
    b.close()
    with pytest.raises(dfa_mod.DFAError):
        dfa_mod.Batch(ds, ins, lookahead=2)


@pytest.mark.parametrize("look", [2, 3, 4, 8])
def test_packed_batch_multi_symbol_lookahead(dfa_mod, look):
    import torch
    wl = configs.batch_workload(count=80, seed=40 + look, max_len=4 << 20)
    ds, xs, ins = make(dfa_mod, wl)
    expect = oracle_records([w for w, _, _, _ in wl], xs)
    for chunk in (0, 4096, 65536):
        b = dfa_mod.Batch(ds, ins, chunk_len=chunk, lookahead=look)
        res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
        b.run(res)
        torch.cuda.synchronize()
        check_records(res, expect)
        b.close()


def test_packed_batch_ragged_and_invalid(dfa_mod):
    """Strings of 0, 1, C-1, C, C+1 and 3C+5 bytes; bytes outside Sigma at a
    chunk's first byte, at a lookahead byte and at the last byte."""
    import torch
    C = 1024
    w, wb = configs.c2_dfa(), configs.c3_byte_dfa()
    d, db = dfa_mod.DFA.from_workload(w), dfa_mod.DFA.from_workload(wb)
    lens = [0, 1, C - 1, C, C + 1, 3 * C + 5, 5 * C]
    xs, ds, ws = [], [], []
    for k, n in enumerate(lens):
        xs.append(configs.c2_input(n, seed=300 + k).copy())
        ds.append(d)
        ws.append(w)
        xs.append(streams.uniform_bytes(400 + k, n))
        ds.append(db)
        ws.append(wb)
    bad = []
    for pos in (C, C - 1, 5 * C - 1):
        x = configs.c2_input(5 * C, seed=500 + pos).copy()
        x[pos] = ord("#")
        xs.append(x)
        ds.append(d)
        ws.append(w)
        bad.append(len(xs) - 1)
    ins = [torch.from_numpy(np.array(x)).to("cuda") for x in xs]
    for look in (1, 3):
        b = dfa_mod.Batch(ds, ins, chunk_len=C, lookahead=look)
        res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
        b.run(res)
        torch.cuda.synchronize()
        r = res.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        for k, x in enumerate(xs):
            if k in bad:
                assert r[k, 2] & dfa_mod.FLAG_SYMBOL, k
                continue
            fin, acc = oracle.membership(ws[k].delta, ws[k].byte_to_symbol, ws[k].q0,
                                         ws[k].accepting, x)
            assert (r[k, 0], r[k, 1], r[k, 2], r[k, 3]) == \
                (fin, int(acc), 0, (x.size + C - 1) // C), (look, k)
        b.close()


def test_packed_batch_graph_replays(dfa_mod):
    import torch
    wl = configs.batch_workload(count=48, seed=77, max_len=1 << 20)
    ds, xs, ins = make(dfa_mod, wl)
    expect = oracle_records([w for w, _, _, _ in wl], xs)
    b = dfa_mod.Batch(ds, ins, lookahead=4)
    s = torch.cuda.Stream()
    for _ in range(3):
        res = torch.full((len(ds), 4), -1, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(s):
            b.graph_launch(res, s)
        torch.cuda.synchronize()
        check_records(res, expect)
        res.fill_(0)          # eager work between replays
        torch.cuda.synchronize()
    b.close()


def test_full_batched_configuration(dfa_mod):
    """1024 pairs, DFAs 8-512 states, strings 1 KiB - 64 MiB (5.7 GiB): at the
    planner's defaults, and through HIP-graph replays (eager work between
    replays) at the setting the benchmark times (8 KiB chunks, r = 6) and at
    the one dfa_batch_tune picks; every record against the oracle."""
    import torch
    wl = configs.batch_workload()
    say("building", len(wl), "requests")
    ds, xs, ins = make(dfa_mod, wl)
    pairs = [w for w, _, _, _ in wl]
    say("oracle")
    expect = oracle_records(pairs, xs)
    say("gpu")
    b = dfa_mod.Batch(ds, ins)
    res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
    b.run(res)
    torch.cuda.synchronize()
    check_records(res, expect)
    b.close()
    s = torch.cuda.Stream()
    chunk, look, ms, ex = dfa_mod.dfa_batch_tune(ds, ins, s)
    torch.cuda.synchronize()
    say(f"tuned: chunk {chunk}, lookahead {look}, early exit {ex}, {ms:.2f} ms")
    for chunk, look, ex in ((8192, 6, False), (chunk, look, ex)):
        b = dfa_mod.Batch(ds, ins, chunk_len=chunk, lookahead=look, early_exit=ex)
        for rep in range(3):
            res = torch.full((len(ds), 4), -1, dtype=torch.int32, device="cuda")
            with torch.cuda.stream(s):
                b.graph_launch(res, s)
            torch.cuda.synchronize()
            check_records(res, expect)
            res.fill_(0)
            torch.cuda.synchronize()
        b.close()


def test_packed_batch_early_exit(dfa_mod):
    """Anchored and "contains" pattern DFAs with early exit: same records."""
    import torch
    ws = [from_pattern(patterns.pattern_dfa(s, contains=bool(s % 2))) for s in range(20, 32)]
    xs = [configs.c2_input((1 << 16) * (k + 1) + 13 * k, seed=600 + k) for k in range(len(ws))]
    ds = [dfa_mod.DFA.from_workload(w) for w in ws]
    ins = [torch.from_numpy(x).to("cuda") for x in xs]
    expect = oracle_records(ws, xs)
    for look in (1, 3):
        b = dfa_mod.Batch(ds, ins, chunk_len=2048, lookahead=look, early_exit=True)
        res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
        b.run(res)
        torch.cuda.synchronize()
        check_records(res, expect)
        b.close()
