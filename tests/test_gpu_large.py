"""Full-size large-DFA configuration: 10 GiB inputs, chunk sweep 4 KiB - 1 MiB.

The oracle walks each 10 GiB input once (Algorithm 1, one host core) and
records the prefix states at every 1 MiB boundary; every GPU run of the sweep
must reproduce the final state, the accept bit and every sampled boundary
state (each 1 MiB boundary is a chunk boundary for all chunk lengths of the
sweep).  The state maps themselves (Section 4.1) are then read back in the
settings the benchmark times and compared with the oracle's direct walks on
a sample of chunks (the first and last two and up to 10,000 random ones).
The protein DFA never reaches its accepting sink on this input, and the byte
DFA has no absorbing state, so every sampled map entry is discriminating.
Tolerance 0."""
import sys
import time

import numpy as np
import pytest

import oracle
from test_gpu_maps import check_maps, sample_chunks
from workloads import configs

pytestmark = pytest.mark.gpu

GiB = 1 << 30
MiB = 1 << 20

# (lookahead, chunk, options) of the readout checks: the benchmark's settings
# first, then others (32 KiB chunks with merged rounds: more chunks than one
# pass of one-chunk-per-lane holds, so the last round takes two per lane)
PROTEIN_MAPS = [(4, 65536, {"rounds": 2, "interleave": True, "single_step": True}),
                (4, 32768, {"rounds": 2, "interleave": True, "single_step": True}),
                (4, 8192, {"chunk_lanes": True, "single_step": True}), (6, 65536, {"rounds": 4}),
                (1, 4096, {}), (8, 1 << 20, {})]
BYTE_MAPS = [(2, 65536, {"rounds": 4, "interleave": True}), (2, 32768, {"rounds": 4, "interleave": True}),
             (2, 131072, {"rounds": 6, "interleave": True}),
             (4, 32768, {"rounds": 4}), (1, 4096, {}), (3, 1 << 20, {})]


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def dfa_mod():
    import torch
    import paper_1210_5093_amd as dfa
    assert torch.cuda.is_available()
    dfa.lib()
    return dfa


def run_sweep(dfa_mod, w, gen, lookaheads, map_checks, n=configs.C3_BYTES):
    import torch
    t0 = time.time()
    x = np.empty(n, dtype=np.uint8)
    gen(n, out=x)
    say(f"generated {n} bytes in {time.time() - t0:.1f}s")
    t0 = time.time()
    probes = list(range(0, n + 1, MiB))
    fin, ps = oracle.walk(w.delta, w.byte_to_symbol, w.q0, x, probes=probes)
    acc = oracle.accepts(fin, w.accepting)
    ab = oracle.absorbing(w.delta)
    assert not ab[ps].any(), "the walk must stay out of absorbing states"
    say(f"oracle walk {time.time() - t0:.1f}s final {fin}")
    dev = torch.from_numpy(x).to("cuda")
    d = dfa_mod.DFA.from_workload(w)
    for r in lookaheads:
        for chunk in configs.C3_CHUNKS:
            _, nch = dfa_mod.dfa_plan_chunks(d, n, chunk, r)
            bnd = torch.empty(nch + 1, dtype=torch.int32, device="cuda")
            res, bnd = dfa_mod.dfa_match_ex(d, dev, chunk_len=chunk, lookahead=r,
                                            boundaries=True, bound_out=bnd)
            torch.cuda.synchronize()
            g = dfa_mod.result_tuple(res)
            say(f"r={r} chunk={chunk} chunks={nch} gpu={g[:3]}")
            assert g[:3] == (fin, acc, 0)
            step = MiB // chunk
            b = bnd[::step].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(b[:len(ps)], ps.astype(np.int64)), f"chunk {chunk}"
            del bnd
    for r, chunk, kw in map_checks:
        plan = dfa_mod.dfa_plan(d, n, chunk, r, **kw)
        if chunk == 32768 and kw.get("interleave"):
            assert plan.tail_lanes == 2, plan.tail_lanes
        nch = int(plan.num_chunks)
        # the mean start-set size bounds the oracle's work per sampled chunk
        mean_set = max(1.0, float(plan.set_max) / 2)
        pick = sample_chunks(nch, mean_set, chunk, seed=r * 1000 + chunk % 997)
        t0 = time.time()
        pairs = check_maps(dfa_mod, w, x, dev, d, chunk, r, chunks=pick, expect=(fin, acc), **kw)
        say(f"maps r={r} chunk={chunk} {kw}: {pick.size} chunks, {pairs} pairs "
            f"in {time.time() - t0:.1f}s")
        torch.cuda.empty_cache()
    d.close()


def test_c3_protein_10gib_chunk_sweep(dfa_mod):
    run_sweep(dfa_mod, configs.c3_protein_dfa(), configs.c3_protein_input, (1, 8), PROTEIN_MAPS)


def test_c3_byte_10gib_chunk_sweep(dfa_mod):
    run_sweep(dfa_mod, configs.c3_byte_dfa(), configs.c3_byte_input, (1,), BYTE_MAPS)
