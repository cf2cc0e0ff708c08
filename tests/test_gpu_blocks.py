"""Block maps of shards and their ordered composition (dfa_match_block,
dfa_compose_blocks): the one-GPU part of matching a string cut into pieces
whose lengths follow processor capacities (Eqs. 1-7, the first piece
lengthened by Eq. 10 since it starts from one state), each piece matched from
its reverse-lookahead set (Eq. 11 / Eq. 13) and the pieces' maps combined in
order (Eq. 9).  Shard boundaries come from the host library's
dfa_host_partition, with capacities from dfa_host_profile or given unequal.

Checked against the oracle: each block map itself (its start states are I
of the r bytes before the shard, absorbing states left out; each end state
is the oracle's direct walk of the shard), the composed final state and
accept bit, and the state before every shard.  Tolerance 0."""
import sys

import numpy as np
import pytest

import oracle
from workloads import column_dfa, configs, streams

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def mods():
    import torch
    import paper_1210_5093_amd as dfa
    from paper_1210_5093_amd import host
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dfa.lib()
    host.lib()
    return dfa, host


def cases():
    return {
        "c1": lambda n: (configs.c1_dfa(2), configs.c1_input(n)),
        "c2": lambda n: (configs.c2_dfa(), configs.c2_input(n, seed=71)),
        "c3b": lambda n: (configs.c3_byte_dfa(), configs.c3_byte_input(n)),
        "c3p": lambda n: (configs.c3_protein_dfa(), configs.c3_protein_input(n)),
        "cols6": lambda n: (column_dfa(91, 92, 150, 6), streams.uniform_bytes(93, n)),
    }


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def oracle_block(w, x, off, end, look, start, absorbing):
    """(start states, end states) of the block [off, end) by the oracle (look:
    the lookahead the library used, after lowering to its precomputed levels)."""
    if off == 0:
        st = np.array([start], dtype=np.int64)
    elif look == 0:
        st = np.nonzero(~absorbing)[0]
    else:
        k = min(look, off)
        syms = tuple(int(s) for s in w.byte_to_symbol[x[off - k:off]])
        st = np.nonzero(oracle.iset_word(w.delta, syms, absorbing))[0]
    ends = oracle.chunk_map(w.delta, w.byte_to_symbol, x, off, end, st.astype(np.uint32))
    return st.astype(np.int64), np.asarray(ends, dtype=np.int64)


def run_blocks(dfa, d, dev, bounds, look, chunk, start=None, check=None, **kw):
    """Block maps of every shard, then their composition."""
    import torch
    G = len(bounds) - 1
    n = bounds[-1]
    # room for any start set (a shard with fewer lookahead bytes before it
    # than r starts from a set of fewer symbols, larger than dfa_plan's)
    mx = (int(d.info().num_states) + 7) // 8 * 8
    infos = torch.empty((G, 4), dtype=torch.int32, device="cuda")
    starts = torch.empty((G, mx), dtype=torch.int16, device="cuda")
    ends = torch.empty((G, mx), dtype=torch.int16, device="cuda")
    for g in range(G):
        dfa.dfa_match_block(d, dev, bounds[g], bounds[g + 1] - bounds[g], start=start,
                            chunk_len=chunk, lookahead=look,
                            out=(infos[g], starts[g], ends[g]), **kw)
    res, bs = dfa.dfa_compose_blocks(d, infos, starts, ends, start=start)
    torch.cuda.synchronize()
    return (dfa.result_tuple(res), bs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF,
            infos.cpu().numpy(), starts.cpu().numpy().astype(np.int64) & 0xFFFF,
            ends.cpu().numpy().astype(np.int64) & 0xFFFF)


def check_all(dfa, w, x, d, bounds, look, chunk, start=None, sample=None, **kw):
    n = x.size
    r0 = int(d.info().lookahead_tables)
    used = look if look < 2 or look <= r0 else (r0 if r0 >= 2 else 1)
    s0 = int(w.q0 if start is None else start)
    g, bs, infos, starts, ends = run_blocks(dfa, d, to_dev(x), bounds, look, chunk, start=start, **kw)
    ofin, ps = oracle.walk(w.delta, w.byte_to_symbol, s0, x, probes=bounds)
    assert g[:3] == (ofin, oracle.accepts(ofin, w.accepting), 0), (g, ofin)
    assert np.array_equal(bs, ps.astype(np.int64)), (bs, ps)
    absorbing = oracle.absorbing(w.delta)
    G = len(bounds) - 1
    pick = range(G) if sample is None else sample
    for k in pick:
        st, en = oracle_block(w, x, bounds[k], bounds[k + 1], used, s0, absorbing)
        m = int(infos[k, 0])
        assert int(infos[k, 1]) == 0
        assert m == st.size, (k, m, st.size)
        assert np.array_equal(starts[k, :m], st), k
        assert np.array_equal(ends[k, :m], en), k
    return g


@pytest.mark.parametrize("case", list(cases()))
@pytest.mark.parametrize("look", [1, 3])
def test_blocks_from_profiled_partition(mods, case, look):
    """Shards from dfa_host_partition with dfa_host_profile capacities (m =
    I_max for one-symbol lookahead, Eq. 10)."""
    dfa, host = mods
    n = (4 << 20) + 11
    w, x = cases()[case](n)
    d = dfa.DFA.from_workload(w)
    hd = host.HostDFA.from_workload(w)
    caps = hd.profile(x[: 1 << 20], 4)
    for G in (1, 3, 8):
        bounds = host.partition(n, float(max(1, hd.imax)), G, caps[:G] if G <= 4 else
                                (caps * 2)[:G])
        say(f"{case} r={look} G={G}: {bounds}")
        check_all(dfa, w, x, d, bounds, look, 4096)
    hd.close()
    d.close()


@pytest.mark.parametrize("kw", [{}, {"rounds": 3, "interleave": True, "single_step": True},
                                {"chunk_lanes": True}, {"rounds": 2}])
def test_blocks_matcher_variants(mods, kw):
    """The block map is the same whichever packed matcher runs each shard."""
    dfa, host = mods
    n = (3 << 20) + 5
    w, x = cases()["c3b"](n)
    d = dfa.DFA.from_workload(w)
    bounds = host.partition(n, 8.0, 5, [1.0, 2.0, 1.5, 0.7, 1.2])
    check_all(dfa, w, x, d, bounds, 2, 8192, **kw)
    d.close()


def test_blocks_lookahead_all_states_and_short_offsets(mods):
    """r = 0 (every non-absorbing state), and shards starting fewer than r
    bytes into the string (the lookahead shrinks to what exists)."""
    dfa, host = mods
    n = 1 << 20
    w, x = cases()["cols6"](n)
    d = dfa.DFA.from_workload(w)
    check_all(dfa, w, x, d, [0, 5000, 300_000, n], 0, 2048)
    check_all(dfa, w, x, d, [0, 1, 2, 3, 70_001, n], 3, 4096)
    d.close()


def test_blocks_explicit_start_state(mods):
    dfa, host = mods
    n = (1 << 20) + 3
    w, x = cases()["c1"](n)
    d = dfa.DFA.from_workload(w)
    check_all(dfa, w, x, d, [0, 123_457, 600_000, n], 1, 4096, start=7)
    d.close()


def test_blocks_symbol_outside_sigma(mods):
    """A byte outside Sigma inside shard 2: that block's flags, and the
    composition's."""
    import torch
    dfa, host = mods
    n = (1 << 20) + 9
    w, x = cases()["c3p"](n)
    x = x.copy()
    x[700_000] = 0xC1
    d = dfa.DFA.from_workload(w)
    bounds = [0, 300_000, 650_000, 800_000, n]
    g, bs, infos, _, _ = run_blocks(dfa, d, to_dev(x), bounds, 4, 4096)
    assert infos[2, 1] & dfa.FLAG_SYMBOL and not infos[0, 1] and not infos[1, 1]
    assert g[2] & dfa.FLAG_SYMBOL
    d.close()


def test_blocks_argument_errors(mods):
    import torch
    dfa, host = mods
    w, x = cases()["c1"](1 << 16)
    d = dfa.DFA.from_workload(w)
    dev = to_dev(x)
    small = (torch.empty(4, dtype=torch.int32, device="cuda"),
             torch.empty(1, dtype=torch.int16, device="cuda"),
             torch.empty(1, dtype=torch.int16, device="cuda"))
    with pytest.raises(dfa.DFAError) as e:
        dfa.dfa_match_block(d, dev, 1000, 4000, lookahead=1, out=small)
    assert e.value.status == dfa.DFA_E_TOOBIG
    with pytest.raises(dfa.DFAError) as e:
        dfa.dfa_match_block(d, dev, 1000, 0, lookahead=1)
    assert e.value.status == dfa.DFA_E_INVAL
    d.close()
