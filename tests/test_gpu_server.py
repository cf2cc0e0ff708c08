"""Serving loop: resident DFAs, continuous batching, admission by memory.

Each served record must equal the oracle's result for the request alone
(tolerance 0) and be the same in the mix as alone; requests that arrive while
batches are running must be admitted and completed; a tight memory budget
must still complete every request (in more, smaller batches)."""
import sys
import time
from concurrent.futures import ThreadPoolExecutor

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


def served_setup(dfa_mod, count, max_len, seed):
    import torch
    wl = configs.served_workload(count=count, seed=seed, max_len=max_len)
    dfas, reqs = wl
    ds = [dfa_mod.DFA.from_workload(w) for w in dfas]
    inputs = []
    for k, (i, n, kind, s) in enumerate(reqs):
        x = configs.request_input(kind, s, n)
        inputs.append((x, torch.from_numpy(x).to("cuda")))
    return dfas, ds, reqs, inputs


def oracle_all(dfas, reqs, inputs):
    def one(k):
        w = dfas[reqs[k][0]]
        fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, inputs[k][0])
        return fin, acc
    with ThreadPoolExecutor(16) as ex:
        return list(ex.map(one, range(len(reqs))))


@pytest.mark.parametrize("streams,budget", [(4, 0), (2, 64 << 20), (1, 0)])
def test_served_results_match_oracle(dfa_mod, streams, budget):
    dfas, ds, reqs, inputs = served_setup(dfa_mod, 300, 2 << 20, seed=31)
    expect = oracle_all(dfas, reqs, inputs)
    srv = dfa_mod.Server(streams=streams, budget_bytes=budget, max_batch=32)
    ids = [srv.register(d) for d in ds]
    tickets = []
    # staggered arrivals: some requests arrive while earlier batches run
    for k, (i, n, kind, s) in enumerate(reqs):
        tickets.append(srv.submit(ids[i], inputs[k][1]))
        if k % 50 == 49:
            time.sleep(0.002)
    got = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st.completed == len(reqs) and st.batches >= 2
    for k, (g, e) in enumerate(zip(got, expect)):
        assert (g[0], g[1], g[2]) == (e[0], e[1], 0), k


def test_alone_equals_mix(dfa_mod):
    dfas, ds, reqs, inputs = served_setup(dfa_mod, 64, 1 << 20, seed=41)
    srv = dfa_mod.Server(streams=3, max_batch=16)
    ids = [srv.register(d) for d in ds]
    mix = [srv.submit(ids[i], inputs[k][1]) for k, (i, _, _, _) in enumerate(reqs)]
    mixed = [srv.wait(t) for t in mix]
    alone = []
    for k, (i, _, _, _) in enumerate(reqs):
        alone.append(srv.wait(srv.submit(ids[i], inputs[k][1])))
    srv.close()
    assert mixed == alone


def test_poll_before_and_after(dfa_mod):
    import torch
    w = configs.c2_dfa()
    d = dfa_mod.DFA.from_workload(w)
    x = configs.c2_input(8 << 20)
    t = torch.from_numpy(x).to("cuda")
    srv = dfa_mod.Server(streams=1)
    i = srv.register(d)
    tk = srv.submit(i, t)
    r = None
    for _ in range(200000):
        r = srv.poll(tk)
        if r is not None:
            break
    assert r is not None
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    assert r[:3] == (fin, acc, 0)
    srv.close()
