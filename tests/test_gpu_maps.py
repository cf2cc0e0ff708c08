"""GPU parity of the state maps themselves (Section 4.1: L_i[j] = delta*(q_j, c_i)).

dfa_match_maps returns, for every (chunk, start state) pair of the packed
matcher, the start state and the end state of its walk.  Each chunk's list of
start states must equal the oracle's initial-state set (Eq. 11 for r = 1,
Eq. 13's image of Q under the r bytes before the chunk otherwise, all states
for r = 0; absorbing states left out), and each end state must equal the
oracle's direct walk of the chunk from that start state.  The protein-style
DFAs here never reach their accepting sink on their configured inputs, so
the walks cover the whole input and every map entry is discriminating.

The full 256 MiB protein-style input is checked chunk by chunk in the settings
the benchmark times; the 10 GiB inputs of the large configuration are
sampled (test_gpu_large.py).  Tolerance 0."""
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


class OracleSets:
    """Initial-state sets by the oracle, cached per lookahead symbol string."""

    def __init__(self, w, r):
        self.w, self.r = w, r
        self.absorbing = oracle.absorbing(w.delta)
        self.sym = w.byte_to_symbol
        self.cache = {}

    def of_chunk(self, x, i, chunk, start):
        if i == 0:
            return np.array([start], dtype=np.uint32)
        if self.r == 0:
            return np.nonzero(~self.absorbing)[0].astype(np.uint32)
        p = i * chunk
        rr = min(self.r, p)
        syms = tuple(int(s) for s in self.sym[x[p - rr:p]])
        got = self.cache.get(syms)
        if got is None:
            got = np.nonzero(oracle.iset_word(self.w.delta, syms, self.absorbing))[0]
            got = got.astype(np.uint32)
            self.cache[syms] = got
        return got


def gpu_maps(dfa_mod, d, dev, chunk, look, start=None, **kw):
    import torch
    res, first, ps, pe = dfa_mod.dfa_match_maps(d, dev, start=start, chunk_len=chunk,
                                                lookahead=look, **kw)
    torch.cuda.synchronize()
    return res, first, ps, pe


def check_maps(dfa_mod, w, x, dev, d, chunk, look, chunks=None, start=None, expect=None,
               threads=16, **kw):
    """Compare the decoded maps of `chunks` (all when None) with the oracle.
    `expect` = (final, accepted) if already known (else the oracle walks x).
    Returns the number of pairs checked."""
    import os
    import torch
    from concurrent.futures import ThreadPoolExecutor
    s0 = int(w.q0 if start is None else start)
    # the readout is of the packed-pair matcher's maps: take it even where the
    # planner would pick one chunk per wavefront
    saved = os.environ.get("DFA_KERNEL")
    os.environ["DFA_KERNEL"] = "2"
    try:
        res, first_t, ps_t, pe_t = gpu_maps(dfa_mod, d, dev, chunk, look, start=start, **kw)
    finally:
        if saved is None:
            del os.environ["DFA_KERNEL"]
        else:
            os.environ["DFA_KERNEL"] = saved
    fin, acc, flags, nch = dfa_mod.result_tuple(res)
    assert flags == 0, flags
    if expect is None:
        ofin, _ = oracle.walk(w.delta, w.byte_to_symbol, s0, x)
        expect = (ofin, oracle.accepts(ofin, w.accepting))
    assert (fin, acc) == tuple(expect)
    first = first_t.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert first.size == nch + 1 and first[0] == 0
    assert first[-1] <= ps_t.numel(), "readout capacity"
    if chunks is None:
        chunks = np.arange(nch)
        ps = ps_t[:first[-1]].cpu().numpy().astype(np.int64) & 0xFFFF
        pe = pe_t[:first[-1]].cpu().numpy().astype(np.int64) & 0xFFFF
        off = first
    else:
        chunks = np.unique(np.asarray(chunks, dtype=np.int64))
        idx = np.concatenate([np.arange(first[c], first[c + 1]) for c in chunks])
        it = torch.from_numpy(idx).to("cuda")
        ps = ps_t[it].cpu().numpy().astype(np.int64) & 0xFFFF
        pe = pe_t[it].cpu().numpy().astype(np.int64) & 0xFFFF
        sizes = first[chunks + 1] - first[chunks]
        off = np.concatenate([[0], np.cumsum(sizes)])
        off = {int(c): (int(off[k]), int(off[k + 1])) for k, c in enumerate(chunks)}
    sets = OracleSets(w, look)
    wants = [sets.of_chunk(x, int(c), chunk, s0) for c in chunks]   # serial: shared cache
    n = x.size

    def one(k):
        c = int(chunks[k])
        lo, hi = (int(first[c]), int(first[c + 1])) if isinstance(off, np.ndarray) else off[c]
        want = wants[k]
        got_s = ps[lo:hi]
        if not np.array_equal(got_s, want.astype(np.int64)):
            return (f"chunk {c}: start set {got_s[:8]} vs oracle {want[:8]} "
                    f"({got_s.size} vs {want.size})")
        ends = oracle.chunk_map(w.delta, w.byte_to_symbol, x, c * chunk,
                                min(n, (c + 1) * chunk), want)
        bad = np.nonzero(pe[lo:hi] != ends.astype(np.int64))[0]
        if bad.size:
            return (f"chunk {c}: ends {pe[lo:hi][bad[:6]]} vs oracle {ends[bad[:6]]} "
                    f"(starts {want[bad[:6]]})")
        return None

    with ThreadPoolExecutor(threads) as ex:
        errors = [e for e in ex.map(one, range(len(chunks))) if e]
    assert not errors, errors[:5]
    return int(sum(w.size for w in wants))


def sample_chunks(nch, mean_set, chunk, seed, budget=20e9, most=10000):
    """First and last two chunks plus random ones, as many as keep the oracle's
    work (chunks x start states x chunk bytes) near `budget` lookups."""
    k = int(min(most, max(16, budget / max(1.0, mean_set * chunk))))
    rng = np.random.default_rng(seed)
    pick = rng.choice(nch, size=min(k, nch), replace=False)
    return np.unique(np.concatenate([[0, 1, nch - 2, nch - 1], pick]).clip(0, nch - 1))


# ---------------------------------------------------------------------------
# The protein-style configuration at full size: every chunk's map
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2_full(dfa_mod):
    import torch
    w = configs.c2_dfa()
    x = configs.c2_input()
    ab = oracle.absorbing(w.delta)
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=[x.size])
    assert not ab[fin], "the configured walk must stay out of the accepting sink"
    dev = torch.from_numpy(x).to("cuda")
    d = dfa_mod.DFA.from_workload(w)
    yield w, x, dev, d
    d.close()


@pytest.mark.parametrize("look,chunk,kw", [
    (6, 1024, {"interleave": True}),           # the benchmark's tuned setting
    (6, 1024, {}),                             # direct pair codes, linear stream
    (5, 2048, {"rounds": 2}),                  # merged walks
    (6, 1024, {"chunk_lanes": True}),          # one chunk per lane
    (5, 2048, {"single_step": True}),          # one symbol per lookup, raw input
    (1, 8192, {}),                             # one-symbol sets (Eq. 11)
])
def test_c2_full_size_every_map(dfa_mod, c2_full, look, chunk, kw):
    w, x, dev, d = c2_full
    say(f"C2 maps r={look} chunk={chunk} {kw}")
    pairs = check_maps(dfa_mod, w, x, dev, d, chunk, look, **kw)
    say(f"  {pairs} pairs checked")


def test_c2_full_size_maps_from_other_start(dfa_mod, c2_full):
    """An explicit start state other than q0: chunk 0's single pair starts there."""
    w, x, dev, d = c2_full
    check_maps(dfa_mod, w, x[: 32 << 20], dev[: 32 << 20], d, 2048, 5,
               start=int(w.num_states // 2))


# ---------------------------------------------------------------------------
# Smaller cases: every lookahead mode and table kind, ragged last chunks
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which,n,chunk,look,kw", [
    ("c1", (1 << 20) + 3, 4096, 1, {}),
    ("c1", (1 << 20) + 3, 4096, 0, {}),
    ("c1", (1 << 20) + 3, 4096, 3, {}),
    ("c3b", (4 << 20) + 9, 8192, 1, {}),
    ("c3b", (4 << 20) + 9, 8192, 4, {"rounds": 4}),
    ("c3b", (4 << 20) + 9, 32768, 12, {}),            # window pass beyond the tables
    ("c3p", (4 << 20) + 17, 4096, 1, {}),
    ("c3p", (4 << 20) + 17, 8192, 6, {"rounds": 3}),
    ("c3p", (4 << 20) + 17, 8192, 4, {"early_exit": True}),
    ("c2", (3 << 20) + 5, 2048, 9, {}),               # window pass
    ("c2", (3 << 20) + 5, 1536, 3, {"early_exit": True}),
])
def test_maps_small(dfa_mod, which, n, chunk, look, kw):
    import torch
    w, x = {
        "c1": lambda: (configs.c1_dfa(3), configs.c1_input(n)),
        "c3b": lambda: (configs.c3_byte_dfa(), configs.c3_byte_input(n)),
        "c3p": lambda: (configs.c3_protein_dfa(), configs.c3_protein_input(n)),
        "c2": lambda: (configs.c2_dfa(), configs.c2_input(n)),
    }[which]()
    d = dfa_mod.DFA.from_workload(w)
    dev = torch.from_numpy(x).to("cuda")
    say(f"maps {which} n={n} chunk={chunk} r={look} {kw}")
    check_maps(dfa_mod, w, x, dev, d, chunk, look, **kw)
    d.close()


def test_maps_readout_needs_packed_path(dfa_mod, monkeypatch):
    """The one-chunk-per-wave matcher keeps strided maps: no readout."""
    import torch
    monkeypatch.setenv("DFA_KERNEL", "1")
    w = configs.c1_dfa(1)
    x = configs.c1_input(1 << 16)
    d = dfa_mod.DFA.from_workload(w)
    with pytest.raises(dfa_mod.DFAError) as e:
        dfa_mod.dfa_match_maps(d, torch.from_numpy(x).to("cuda"), chunk_len=1024)
    assert e.value.status == dfa_mod.DFA_E_INVAL
    d.close()
