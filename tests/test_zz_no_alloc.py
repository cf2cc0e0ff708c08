"""dfa_match_noalloc (the entry point for callers that cannot allocate device
memory) against dfa_match_ex, the entry point it is a variant of: the same
result record and chunk-boundary states, bit-exact, on two calls in a row
(the second with a smaller input, so the fixed region holds the first
call's contents), on the translated, raw-input, merged-walk and
one-chunk-per-wave paths; a plan beyond the region is refused with
DFA_E_TOOBIG; and the calls allocate no device memory."""
import json
import os
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dfa.lib()
    return dfa


def both(dfa_mod, d, dev, **kw):
    """(record, boundaries) of dfa_match_ex and of dfa_match_noalloc."""
    import torch
    out = []
    for fn in (dfa_mod.dfa_match_ex, dfa_mod.dfa_match_noalloc):
        res, bnd = fn(d, dev, boundaries=True, **kw)
        torch.cuda.synchronize()
        out.append((dfa_mod.result_tuple(res), bnd.cpu().numpy().astype(np.int64) & 0xFFFFFFFF))
    return out


@pytest.mark.parametrize("which,kw", [
    ("c2", {"chunk_len": 1024, "lookahead": 6}),                      # pair codes (translated)
    ("c2", {"chunk_len": 2048, "lookahead": 5, "single_step": True}),  # raw input
    ("c2", {"chunk_len": 1024, "lookahead": 6, "interleave": True}),
    ("c3b", {"chunk_len": 32768, "lookahead": 4, "rounds": 4}),        # merged walks
    ("c1", {"chunk_len": 0, "lookahead": 1}),                          # planner's choice
    # merged walks with the one-chunk-per-lane last round over the raw input:
    # one and two chunks per lane, and after a window pass (r above r0)
    ("c3b", {"chunk_len": 8192, "lookahead": 2, "rounds": 4, "interleave": True}),
    ("c3b", {"chunk_len": 8192, "lookahead": 2, "rounds": 4, "interleave": True, "_tail_k": "2"}),
    ("c3b", {"chunk_len": 8192, "lookahead": 4, "rounds": 4, "interleave": True}),
])
def test_noalloc_equals_match_ex_twice(dfa_mod, monkeypatch, which, kw):
    import torch
    kw = dict(kw)
    if "_tail_k" in kw:
        monkeypatch.setenv("DFA_TAIL_K", kw.pop("_tail_k"))
    w, gen = {"c2": (configs.c2_dfa(), lambda n: configs.c2_input(n, seed=5)),
              "c3b": (configs.c3_byte_dfa(), configs.c3_byte_input),
              "c1": (configs.c1_dfa(2), configs.c1_input)}[which]
    d = dfa_mod.DFA.from_workload(w)
    for n in ((24 << 20) + 7, (3 << 20) + 1):            # second call smaller
        x = gen(n)
        dev = torch.from_numpy(x).to("cuda")
        (r1, b1), (r2, b2) = both(dfa_mod, d, dev, **kw)
        say(f"{which} n={n} {kw}: {r1} / {r2}")
        fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
        assert r1 == r2 and r2[:3] == (fin, acc, 0)
        assert np.array_equal(b1, b2)
    d.close()


def test_noalloc_refuses_plans_beyond_the_region(dfa_mod):
    """256 MiB translated into pair codes needs 128 MiB of code stream."""
    import torch
    w = configs.c2_dfa()
    d = dfa_mod.DFA.from_workload(w)
    dev = torch.from_numpy(configs.c2_input(256 << 20)).to("cuda")
    with pytest.raises(dfa_mod.DFAError) as e:
        dfa_mod.dfa_match_noalloc(d, dev, chunk_len=1024, lookahead=6)
    assert e.value.status == dfa_mod.DFA_E_TOOBIG
    # the raw-input path needs only maps: the same input fits
    res, _ = dfa_mod.dfa_match_noalloc(d, dev, chunk_len=2048, lookahead=5, single_step=True)
    torch.cuda.synchronize()
    from conftest import GOLDEN
    with open(os.path.join(GOLDEN, "large_finals.json")) as f:
        golden = json.load(f)["c2"]
    g = dfa_mod.result_tuple(res)
    assert g[:3] == (golden["final_state"], golden["accepted"], 0)
    d.close()


def test_noalloc_allocates_no_device_memory(dfa_mod):
    """Free device memory is unchanged by calls on a stream the library has
    never seen (dfa_match_ex would make that stream a workspace)."""
    import torch
    w = configs.c2_dfa()
    d = dfa_mod.DFA.from_workload(w)
    x = configs.c2_input(16 << 20, seed=9)
    dev = torch.from_numpy(x).to("cuda")
    res = torch.empty(4, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    dfa_mod.dfa_match_noalloc(d, dev, chunk_len=1024, lookahead=6, stream=s, result=res)
    # a second stream that torch has used (its queue exists) but the library not
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        res.fill_(0)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        dfa_mod.dfa_match_noalloc(d, dev, chunk_len=1024, lookahead=6, stream=s2, result=res)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free0 - free1) < (2 << 20), (free0, free1)
    fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, x)
    assert dfa_mod.result_tuple(res)[:3] == (fin, acc, 0)
    d.close()
