"""Error paths on the GPU: device limits (DFA_E_TOOBIG), the speculation
check (DFA_E_SPECULATION, forced by leaving one state out of every
initial-state set), and the server's admission and ordering contracts.

The speculative method is exact only because every chunk's true start state
lies in its initial-state set (Section 4.2, Eq. 11; Section 4.3 for Eq. 13).
With a state s left out (DFA_DROP_STATE at dfa_create), a chunk whose true
start state is s has no walk from it; the library must then report the
violation instead of any state, and must still return exact results on
inputs where s never starts a chunk."""
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


def test_table_beyond_lds_is_too_big(dfa_mod):
    """32767 states over 3 distinct columns: a 192 KiB class-major table."""
    rng = np.random.default_rng(5)
    nq = 32767
    delta = rng.integers(0, nq, (nq, 3)).astype(np.uint32)
    b2s = np.full(256, 0xFF, dtype=np.uint8)
    b2s[:3] = np.arange(3)
    with pytest.raises(dfa_mod.DFAError) as e:
        dfa_mod.DFA(delta, 0, [1], b2s)
    assert e.value.status == dfa_mod.DFA_E_TOOBIG


# ---------------------------------------------------------------------------
# Forced speculation failure
# ---------------------------------------------------------------------------
CHUNK = 1024


def boundary_states(w, x, chunk):
    probes = list(range(0, x.size, chunk)) + [x.size]
    _, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    return ps


@pytest.fixture(scope="module")
def dropped_case():
    """C1's DFA, an input whose true state at one chunk boundary is s, and an
    input of the same length where s starts no chunk."""
    w = configs.c1_dfa(1)
    x = configs.c1_input(1 << 16)
    ps = boundary_states(w, x, CHUNK)
    s = int(ps[5])
    clean = None
    for seed in range(100, 400):
        y = configs.c1_input(1 << 16, seed=seed)
        if s not in set(boundary_states(w, y, CHUNK)[1:-1].tolist()):
            clean = y
            break
    assert clean is not None
    return w, x, s, clean


@pytest.mark.parametrize("kernel,look", [("1", 1), ("2", 1), ("2", 2), ("2", 0)])
def test_dropped_state_reports_speculation(dfa_mod, monkeypatch, dropped_case, kernel, look):
    import torch
    w, x, s, clean = dropped_case
    monkeypatch.setenv("DFA_KERNEL", kernel)
    monkeypatch.setenv("DFA_DROP_STATE", str(s))
    d = dfa_mod.DFA.from_workload(w)
    monkeypatch.delenv("DFA_DROP_STATE")
    say(f"dropped state {s}, kernel {kernel}, r={look}")
    res, _ = dfa_mod.dfa_match_ex(d, torch.from_numpy(x).to("cuda"), chunk_len=CHUNK,
                                  lookahead=look)
    torch.cuda.synchronize()
    fin, acc, flags, _ = dfa_mod.result_tuple(res)
    # (with r = 0, Algorithm 2's all-state sets lack s as well)
    assert flags & dfa_mod.FLAG_SPECULATION, (fin, flags)
    assert fin == 0xFFFFFFFF and not acc
    # the same DFA on an input where s starts no chunk: exact
    res, _ = dfa_mod.dfa_match_ex(d, torch.from_numpy(clean).to("cuda"), chunk_len=CHUNK,
                                  lookahead=look)
    torch.cuda.synchronize()
    ofin, oacc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, clean)
    assert dfa_mod.result_tuple(res)[:3] == (ofin, oacc, 0)
    d.close()


def test_dropped_state_sync_call_raises(dfa_mod, monkeypatch, dropped_case):
    w, x, s, _ = dropped_case
    monkeypatch.setenv("DFA_KERNEL", "2")
    monkeypatch.setenv("DFA_DROP_STATE", str(s))
    d = dfa_mod.DFA.from_workload(w)
    monkeypatch.delenv("DFA_DROP_STATE")
    monkeypatch.setenv("DFA_CHUNK", str(CHUNK))
    with pytest.raises(dfa_mod.DFAError) as e:
        dfa_mod.dfa_match(d, x.tobytes())
    assert e.value.status == dfa_mod.DFA_E_SPECULATION
    d.close()


def test_dropped_state_in_a_batch(dfa_mod, monkeypatch, dropped_case):
    """Only the string whose boundary hits s is flagged; the others are exact."""
    import torch
    w, x, s, clean = dropped_case
    monkeypatch.setenv("DFA_DROP_STATE", str(s))
    d = dfa_mod.DFA.from_workload(w)
    monkeypatch.delenv("DFA_DROP_STATE")
    ins = [torch.from_numpy(v).to("cuda") for v in (clean, x, clean[:5000])]
    for look in (1, 2):
        b = dfa_mod.Batch([d, d, d], ins, chunk_len=CHUNK, lookahead=look)
        res = torch.empty((3, 4), dtype=torch.int32, device="cuda")
        b.run(res)
        torch.cuda.synchronize()
        r = res.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        assert r[1, 2] & dfa_mod.FLAG_SPECULATION
        for k, v in ((0, clean), (2, clean[:5000])):
            fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, v)
            assert (r[k, 0], r[k, 1], r[k, 2]) == (fin, int(acc), 0), (look, k)
        b.close()
    d.close()


def test_dropped_state_maps_name_no_state(dfa_mod, monkeypatch, dropped_case):
    """The map entry of the walk that reached s reads 0xFFFF in the readout."""
    import torch
    w, x, s, _ = dropped_case
    monkeypatch.setenv("DFA_KERNEL", "2")
    monkeypatch.setenv("DFA_DROP_STATE", str(s))
    d = dfa_mod.DFA.from_workload(w)
    monkeypatch.delenv("DFA_DROP_STATE")
    res, first, ps, pe = dfa_mod.dfa_match_maps(d, torch.from_numpy(x).to("cuda"),
                                                chunk_len=CHUNK, lookahead=1)
    torch.cuda.synchronize()
    assert dfa_mod.result_tuple(res)[2] & dfa_mod.FLAG_SPECULATION
    f = first.cpu().numpy().astype(np.int64)
    st = ps.cpu().numpy().astype(np.int64) & 0xFFFF
    en = pe.cpu().numpy().astype(np.int64) & 0xFFFF
    # the first chunk whose walk from its true start state ends in s
    truth = boundary_states(w, x, CHUNK)
    c = int(np.nonzero(truth[1:] == s)[0][0])      # truth[c + 1] == s, truth[c] != s
    lo, hi = f[c], f[c + 1]
    k = int(np.nonzero(st[lo:hi] == truth[c])[0][0])
    assert en[lo + k] == 0xFFFF
    assert s not in st[f[1]:f[-1]]
    d.close()


# ---------------------------------------------------------------------------
# Server admission and ordering
# ---------------------------------------------------------------------------
def test_server_refuses_request_over_budget(dfa_mod):
    import torch
    w = configs.c1_dfa(1)
    d = dfa_mod.DFA.from_workload(w)
    srv = dfa_mod.Server(budget_bytes=1 << 20, streams=1)
    i = srv.register(d)
    x = torch.from_numpy(configs.c1_input(1 << 20)).to("cuda")
    with pytest.raises(dfa_mod.DFAError) as e:
        srv.submit(i, x)
    assert e.value.status == dfa_mod.DFA_E_TOOBIG
    srv.close()
    d.close()


def test_server_refuses_request_over_slot_arena_and_keeps_serving(dfa_mod):
    """A request that alone does not fit a slot's arena is refused at submit;
    requests that fit are still served exactly."""
    import torch
    w = configs.c2_dfa()
    d = dfa_mod.DFA.from_workload(w)
    srv = dfa_mod.Server(slot_bytes=4 << 20, streams=2)
    i = srv.register(d)
    big = torch.from_numpy(configs.c2_input(64 << 20, seed=71)).to("cuda")
    with pytest.raises(dfa_mod.DFAError) as e:
        srv.submit(i, big)
    assert e.value.status == dfa_mod.DFA_E_TOOBIG
    xs = [configs.c2_input(50_000 + 999 * k, seed=72 + k) for k in range(6)]
    ts = [srv.submit(i, torch.from_numpy(v).to("cuda")) for v in xs]
    got = [srv.wait(t) for t in ts]
    for v, g in zip(xs, got):
        fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, v)
        assert g[:3] == (fin, acc, 0)
    srv.close()
    d.close()


def test_server_waits_for_the_producer_stream(dfa_mod):
    """Inputs written on a side stream right before submit: the batch reads
    them only after the producer's work (a spin, then the copy) finished."""
    import torch
    w = configs.c2_dfa()
    d = dfa_mod.DFA.from_workload(w)
    srv = dfa_mod.Server(streams=2)
    i = srv.register(d)
    xs = [configs.c2_input(300_000 + 77 * k, seed=80 + k) for k in range(4)]
    srcs = [torch.from_numpy(v).to("cuda") for v in xs]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    dsts, ts = [], []
    for src in srcs:
        dst = torch.full_like(src, ord("A"))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            torch.cuda._sleep(20_000_000)       # about 10 ms of spinning
            dst.copy_(src, non_blocking=True)
            ts.append(srv.submit(i, dst))
        dsts.append(dst)
    got = [srv.wait(t) for t in ts]
    side.synchronize()
    for v, g in zip(xs, got):
        fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting, v)
        assert g[:3] == (fin, acc, 0)
    srv.close()
    d.close()
