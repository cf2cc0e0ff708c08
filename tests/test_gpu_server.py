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
    # the result (final state, accept bit, flags) is the same; the chunk count
    # is a property of the path a batch took (a batch of one takes the
    # single-string path)
    assert [m[:3] for m in mixed] == [a[:3] for a in alone]


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


def test_served_multi_symbol_lookahead_and_first_generation_dfas(dfa_mod):
    """Batches with lookahead 4 (packed pairs), and batches that hold a DFA
    without a packed layout (one chunk per wavefront, lookahead 1)."""
    import torch
    from workloads import column_dfa
    dfas, ds, reqs, inputs = served_setup(dfa_mod, 120, 1 << 20, seed=51)
    expect = oracle_all(dfas, reqs, inputs)
    srv = dfa_mod.Server(streams=2, max_batch=24, lookahead=4)
    ids = [srv.register(d) for d in ds]
    tickets = [srv.submit(ids[i], inputs[k][1]) for k, (i, _, _, _) in enumerate(reqs)]
    got = [srv.wait(t) for t in tickets]
    srv.close()
    for k, (g, e) in enumerate(zip(got, expect)):
        assert (g[0], g[1], g[2]) == (e[0], e[1], 0), k
    # a 600-state, 64-class byte DFA has no packed layout (its LDS addresses
    # exceed 16 bits); mixed into every batch it selects the first-generation path
    wide = column_dfa(71, 72, 600, 64)
    dw = dfa_mod.DFA.from_workload(wide)
    assert dw.info().packed_layout == 0
    xs = [configs.request_input("bytes", 7000 + k, 50_000 + 999 * k) for k in range(12)]
    ins = [torch.from_numpy(x).to("cuda") for x in xs]
    srv = dfa_mod.Server(streams=2, max_batch=8, lookahead=4)
    iw = srv.register(dw)
    i0 = reqs[0][0]
    ib = srv.register(ds[i0])
    tickets = []
    for k, t in enumerate(ins):
        tickets.append((srv.submit(iw, t), k, None))
    same = [k for k, r in enumerate(reqs) if r[0] == i0][:6]
    for k in same:
        tickets.append((srv.submit(ib, inputs[k][1]), k, "pool"))
    for t, k, which in tickets:
        g = srv.wait(t)
        if which is None:
            fin, acc = oracle.membership(wide.delta, wide.byte_to_symbol, wide.q0,
                                         wide.accepting, xs[k])
        else:
            fin, acc = expect[k]
        assert (g[0], g[1], g[2]) == (fin, acc, 0), (k, which)
    srv.close()
    dw.close()
