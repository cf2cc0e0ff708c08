"""Autotuner: the tuned setting must not change any result.

dfa_autotune times (lookahead, chunk length) candidates and caches the
fastest; a later call with the automatic lookahead must give the oracle's
final state and accept bit (tolerance 0), and so must a batch run with the
chunk length dfa_batch_tune picks."""
import sys

import numpy as np
import pytest

import oracle
from workloads import configs

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


@pytest.mark.parametrize("which,n", [("c2", 24 << 20), ("c1", 1 << 20), ("c3b", 16 << 20)])
def test_autotuned_setting_matches_oracle(dfa_mod, which, n):
    import torch
    if which == "c2":
        w, x = configs.c2_dfa(), configs.c2_input(n)
    elif which == "c1":
        w, x = configs.c1_dfa(1), configs.c1_input(n)
    else:
        w, x = configs.c3_byte_dfa(), configs.c3_byte_input(n)
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    d = dfa_mod.DFA.from_workload(w)
    dev = torch.from_numpy(x).to("cuda")
    r, chunk, ms, ex, rounds, single, ilv, lanes = dfa_mod.dfa_autotune(d, dev)
    say(f"{which}: tuned r={r} chunk={chunk} early_exit={ex} rounds={rounds} "
        f"single_step={single} interleave={ilv} chunk_lanes={lanes} {ms:.3f} ms")
    assert 1 <= r <= 10 and ms > 0
    res, _ = dfa_mod.dfa_match_ex(d, dev, lookahead=dfa_mod.DFA_LOOKAHEAD_AUTO)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[:3] == (fin, int(acc), 0)
    auto = dfa_mod.dfa_plan(d, n, 0, dfa_mod.DFA_LOOKAHEAD_AUTO)
    explicit = dfa_mod.dfa_plan(d, n, chunk, r, rounds=rounds, early_exit=ex, single_step=single,
                                interleave=ilv, chunk_lanes=lanes)
    assert (auto.chunk_len, auto.lookahead, auto.kernel, auto.rounds, auto.symbols_per_step,
            auto.interleaved, auto.chunk_lanes) == \
        (explicit.chunk_len, explicit.lookahead, explicit.kernel, explicit.rounds,
         explicit.symbols_per_step, explicit.interleaved, explicit.chunk_lanes)
    # a length of another order was not tuned: one-symbol lookahead
    plan_small = dfa_mod.dfa_plan(d, 1000, 0, dfa_mod.DFA_LOOKAHEAD_AUTO)
    assert plan_small.lookahead == 1
    d.close()


def test_batch_tune_matches_oracle(dfa_mod):
    import torch
    wl = configs.batch_workload(count=48, seed=23, max_len=1 << 20)
    cache, ds, xs, ins = {}, [], [], []
    for w, n, kind, seed in wl:
        if id(w) not in cache:
            cache[id(w)] = dfa_mod.DFA.from_workload(w)
        ds.append(cache[id(w)])
        x = configs.request_input(kind, seed, n)
        xs.append(x)
        ins.append(torch.from_numpy(x).to("cuda"))
    chunk, look, ms, ex = dfa_mod.dfa_batch_tune(ds, ins)
    say(f"batch tuned chunk={chunk} lookahead={look} early_exit={ex} {ms:.3f} ms")
    assert chunk >= 256 and chunk % 64 == 0 and 1 <= look <= 8
    b = dfa_mod.Batch(ds, ins, chunk_len=chunk, lookahead=look, early_exit=ex)
    res = torch.empty((len(ds), 4), dtype=torch.int32, device="cuda")
    b.run(res)
    torch.cuda.synchronize()
    r = res.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    for k, (w, _, _, _) in enumerate(wl):
        try:
            fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, xs[k])
            assert (r[k, 0], r[k, 1], r[k, 2]) == (fin, int(acc), 0), k
        except oracle.InvalidSymbol:
            assert r[k, 2] & 1, k
    b.close()
