"""Benchmark: input GB/s of the speculative DFA membership test on one MI355X.

Workload (default): the protein-style configuration -- the minimal DFA of
Sigma* P Sigma* for a seeded PROSITE-like pattern P (284 states, 20 amino-acid
letters) and 256 MiB of residues drawn from a fixed synthetic frequency
vector, resident in HBM before timing starts.  One step = one full membership
test of the whole input: chunk matching from the reverse-lookahead initial
state sets, the ordered map combination, and the accept test (every kernel of
the path; the DFA is compiled once beforehand and its compile time is
reported separately).

Prints one JSON line (rank 0, one GPU).  ``roofline`` describes the dominant
kernel (the chunk matcher): its algorithmic table lookups per launch divided
by its average duration, measured with HIP events inside the timed steps,
against the LDS-lookup peak of the chip.  ``cpu_baseline`` times the
sequential oracle on the host.

``--workload c4`` runs the batched configuration (1024 (DFA, string) pairs,
one persistent launch replayed from a HIP graph, chunk length from the
autotuner) beside the plain per-request method on the same GPU;
``--workload c5`` the served one (64 resident DFAs, Poisson arrivals at 0.7x
the plain method's measured capacity, p50/p99 latency from arrival to the
result on the host) beside a plain FIFO loop under the same arrivals.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X figures used as roofline denominators.
N_CU = 256
CLOCK_HZ = 2.4e9
LDS_LOOKUPS_PER_CU_CLK = 32          # 32 banks, one dword per bank per clock
LDS_LOOKUP_PEAK = N_CU * CLOCK_HZ * LDS_LOOKUPS_PER_CU_CLK   # lookups/s
HBM_PEAK_GBS = 8000.0


# Sources whose change invalidates stored counter readings of the matcher.
KERNEL_SOURCES = ["dfa_match2.hip", "dfa_kernels.hip", "dfa_internal.h", "dfa_walk1.h",
                  "dfa_pairs.h"]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1210_5093_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str, lookahead: int, chunk: int):
    """HBM bytes per launch from a committed counter summary in profiles/, if it
    was taken on the current kernel sources with the same configuration.

    A summary carries a line
    ``traffic: kernel=K workload=W lookahead=R chunk=C bytes=B sources=D``
    where B = scaled FETCH_SIZE + WRITE_SIZE per launch and D the digest of
    the matcher sources when the counters were read."""
    import glob
    import re
    digest = kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                m = re.search(r"traffic: kernel=(.+?) workload=(\S+) lookahead=(\d+) "
                              r"chunk=(\d+) bytes=(\d+) sources=([0-9a-f]+)", line)
                if m and m.group(1) == kernel and m.group(2) == workload and \
                        int(m.group(3)) == lookahead and int(m.group(4)) == chunk and \
                        m.group(6) == digest:
                    return int(m.group(5)), os.path.relpath(path, ROOT)
    return None, None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from workloads import configs
    if name == "c2":
        w = configs.c2_dfa()
        desc = ("protein-style: minimal DFA of Sigma* P Sigma*, PROSITE-like pattern seed "
                f"{configs.C2_PATTERN_SEED} ({w.num_states} states, 20 amino-acid letters); "
                "256 MiB residues, stream seed 4")
        return w, (lambda n, out=None: configs.c2_input(n, out=out)), configs.C2_BYTES, desc
    if name == "c2a":
        from workloads import from_pattern, patterns
        w = from_pattern(patterns.pattern_dfa(configs.C2_PATTERN_SEED, contains=False))
        desc = ("protein-style, anchored: minimal DFA of P alone (rejecting sink), pattern seed "
                f"{configs.C2_PATTERN_SEED} ({w.num_states} states); 256 MiB residues, stream seed 4")
        return w, (lambda n, out=None: configs.c2_input(n, out=out)), configs.C2_BYTES, desc
    if name == "c1":
        w = configs.c1_dfa(1)
        return w, (lambda n, out=None: configs.c1_input(n)), configs.C1_BYTES, \
            "plain: random complete DFA 16 states x 256 bytes (seed 1); 1 MiB uniform bytes"
    if name == "c3p":
        w = configs.c3_protein_dfa()
        return w, (lambda n, out=None: configs.c3_protein_input(n, out=out)), 1 << 30, \
            f"large protein DFA {w.num_states} states; 1 GiB residues (one GPU's share)"
    if name == "c3b":
        w = configs.c3_byte_dfa()
        return w, (lambda n, out=None: configs.c3_byte_input(n, out=out)), 1 << 30, \
            "byte DFA 512 states, 64 columns; 1 GiB uniform bytes (one GPU's share)"
    raise SystemExit(f"unknown workload {name}")


def set_sizes(w) -> np.ndarray:
    """|I_a| per symbol: distinct targets of column a minus absorbing states."""
    d = w.delta.astype(np.int64)
    absorbing = np.all(d == np.arange(d.shape[0])[:, None], axis=1)
    sizes = np.zeros(d.shape[1], dtype=np.int64)
    for a in range(d.shape[1]):
        t = np.unique(d[:, a])
        sizes[a] = int((~absorbing[t]).sum())
    return sizes


def image_sizes(w, x: np.ndarray, chunk: int, nch: int, r: int) -> np.ndarray:
    """|image of Q under the r bytes before chunk i| minus absorbing states, i >= 1."""
    d = w.delta.astype(np.int32)
    nq = d.shape[0]
    absorbing = np.all(d == np.arange(nq)[:, None], axis=1)
    sym = w.byte_to_symbol.astype(np.int64)
    out = np.zeros(nch - 1, dtype=np.int64)
    batch = max(1, (1 << 24) // max(nq, 1))
    for b0 in range(1, nch, batch):
        idx = np.arange(b0, min(nch, b0 + batch), dtype=np.int64)
        p = idx * chunk
        rr = np.minimum(r, p)
        S = np.broadcast_to(np.arange(nq, dtype=np.int32), (idx.size, nq)).copy()
        for t in range(int(rr.max())):
            # step t of the lookahead string w[p - rr + t]; rows with rr <= t are done
            live = t < rr
            pos = np.where(live, p - rr + t, 0)
            a = sym[x[pos]]
            S = np.where(live[:, None], d[S, a[:, None]], S)
        S.sort(axis=1)
        distinct = np.concatenate([np.ones((S.shape[0], 1), bool), S[:, 1:] != S[:, :-1]], axis=1)
        out[idx - 1] = (distinct & ~absorbing[S]).sum(axis=1)
    return out


def start_sets(w, x: np.ndarray, chunk: int, nch: int, r: int):
    """Per chunk i >= 1 its start states (padded with -1): the image of Q under
    the min(r, i*C) bytes before it (r >= 1; r = 0: all states), absorbing
    states left out."""
    d = w.delta.astype(np.int32)
    nq = d.shape[0]
    absorbing = np.all(d == np.arange(nq)[:, None], axis=1)
    sym = w.byte_to_symbol.astype(np.int64)
    rows = []
    batch = max(1, (1 << 24) // max(nq, 1))
    for b0 in range(1, nch, batch):
        idx = np.arange(b0, min(nch, b0 + batch), dtype=np.int64)
        S = np.broadcast_to(np.arange(nq, dtype=np.int32), (idx.size, nq)).copy()
        p = idx * chunk
        rr = np.minimum(r, p)
        for t in range(int(rr.max()) if r > 0 else 0):
            live = t < rr
            pos = np.where(live, p - rr + t, 0)
            S = np.where(live[:, None], d[S, sym[x[pos]][:, None]], S)
        S.sort(axis=1)
        keep = np.concatenate([np.ones((S.shape[0], 1), bool), S[:, 1:] != S[:, :-1]], axis=1)
        keep &= ~absorbing[S]
        S = np.where(keep, S, -1)
        S = -np.sort(-S, axis=1)   # members first
        rows.append(S[:, :max(1, int(keep.sum(axis=1).max()))])
    return rows


def early_exit_lookups(w, x: np.ndarray, chunk: int, lookahead: int, start: int,
                       step: int = 1) -> int:
    """Lookups of Algorithm 3 when every walk stops at the first absorbing
    state it reaches (the least work early exit can do; the kernel checks
    every 64 bytes, so it does at least this much).  step = k counts table
    reads of the k-symbol table (one per k symbols of a walk)."""
    d = w.delta.astype(np.int32)
    nq = d.shape[0]
    absorbing = np.all(d == np.arange(nq)[:, None], axis=1)
    sym = w.byte_to_symbol.astype(np.int64)
    n = x.size
    nch = (n + chunk - 1) // chunk
    pcs, pss = [np.zeros(1, np.int64)], [np.array([start], np.int64)]
    base = 1
    for S in start_sets(w, x, chunk, nch, max(lookahead, 1) if lookahead else 0):
        rr, cc = np.nonzero(S >= 0)
        pcs.append(rr + base)
        pss.append(S[rr, cc].astype(np.int64))
        base += S.shape[0]
    pc, ps = np.concatenate(pcs), np.concatenate(pss)
    lens = np.minimum(chunk, n - pc * chunk)
    total = 0
    for t in range(chunk):
        if pc.size == 0:
            break
        ps = d[ps, sym[x[pc * chunk + t]]]
        if t % step == 0:
            total += pc.size
        alive = (~absorbing[ps]) & (t + 1 < lens)
        pc, ps, lens = pc[alive], ps[alive], lens[alive]
    return int(total)


def merged_lookups(w, x: np.ndarray, chunk: int, lookahead: int, rounds: int,
                   step: int = 1):
    """Table reads of the merged walks (rounds >= 2), and the input bytes they
    cover (per chunk, the furthest any of its walks got): round k walks bytes
    [t_k, t_{k+1}) of every chunk (t_1 = 32, x4 per round, the last round to
    the chunk end), every walk still live; after a round that is not the last
    one walk per distinct (chunk, state) goes on, and walks whose chunk ended
    or that reached an absorbing state stop (in the last round too).  Grouping
    here is per chunk; the kernel groups per wave-tile, so a chunk split over
    two tiles may keep one more walk: this count is the least work the kernel
    does."""
    d = w.delta.astype(np.int32)
    nq = d.shape[0]
    absorbing = np.all(d == np.arange(nq)[:, None], axis=1)
    sym = w.byte_to_symbol.astype(np.int64)
    n = x.size
    nch = (n + chunk - 1) // chunk
    lens = np.minimum(chunk, n - np.arange(nch, dtype=np.int64) * chunk)
    pcs, pss = [np.zeros(1, np.int64)], [np.array([int(w.q0)], np.int64)]
    base = 1
    for S in start_sets(w, x, chunk, nch, max(lookahead, 1) if lookahead else 0):
        rr, cc = np.nonzero(S >= 0)
        pcs.append(rr + base)
        pss.append(S[rr, cc].astype(np.int64))
        base += S.shape[0]
    pc, ps = np.concatenate(pcs), np.concatenate(pss)
    total = 0
    t0 = 0
    ext = np.zeros(nch, dtype=np.int64)
    for k in range(rounds):
        last = k + 1 == rounds
        t1 = 32 << (2 * k)
        if last:
            # to the chunk end or the first absorbing state, a step (of
            # `step` symbols) at a time
            alive = ~absorbing[ps] & (lens[pc] > t0)
            pc, ps = pc[alive], ps[alive]
            t = t0
            while pc.size:
                np.maximum.at(ext, pc, np.minimum(lens[pc], t + step))
                total += pc.size
                for j in range(step):
                    inside = t + j < lens[pc]
                    ps = np.where(inside, d[ps, sym[x[np.where(inside, pc * chunk + t + j, 0)]]], ps)
                t += step
                keep = (lens[pc] > t) & ~absorbing[ps]
                pc, ps = pc[keep], ps[keep]
            break
        end = np.minimum(lens[pc], t1)
        total += int(((end - t0 + step - 1) // step).clip(min=0).sum())
        np.maximum.at(ext, pc, end)
        for t in range(t0, t1):
            live = t < lens[pc]
            if not live.any():
                break
            ps = np.where(live, d[ps, sym[x[np.where(live, pc * chunk + t, 0)]]], ps)
        keep = (lens[pc] > t1) & ~absorbing[ps]
        pc, ps = pc[keep], ps[keep]
        key = np.unique(pc * nq + ps)
        pc, ps = key // nq, key % nq
        t0 = t1
    return total, int(ext.sum())


def algorithmic_lookups(w, x: np.ndarray, chunk: int, lookahead: int, step: int = 1) -> int:
    """len(c_0) + sum_{i>=1} |I_i| len(c_i) (Algorithm 3's work; I_i is the
    chunk's start set: all states, I_sigma, or the r-symbol image of Eq. 13).
    step = k: table reads of the k-symbol table, ceil(len / k) per walk."""
    n = x.size
    nch = (n + chunk - 1) // chunk
    lens = np.full(nch, chunk, dtype=np.int64)
    lens[-1] = n - chunk * (nch - 1)
    lens = (lens + step - 1) // step
    if nch == 1:
        return int(lens[0])
    if lookahead >= 2:
        m = image_sizes(w, x, chunk, nch, lookahead)
    elif lookahead == 1:
        sizes = set_sizes(w)
        look = x[chunk - 1: chunk * (nch - 1): chunk]
        m = sizes[w.byte_to_symbol[look]]
    else:
        d = w.delta
        nabs = int(np.all(d == np.arange(d.shape[0])[:, None], axis=1).sum())
        m = np.full(nch - 1, d.shape[0] - nabs, dtype=np.int64)
    return int(lens[0] + (m * lens[1:]).sum())

METRIC = ("input GB/s per DFA-membership test (bit-exact) vs sequential; "
          "p99 latency served")


def concat_inputs(items):
    """One host buffer holding every request's input: (buffer, offsets)."""
    from workloads import configs
    lens = np.array([n for _, n, _, _ in items], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(lens)])
    buf = np.empty(int(offs[-1]), dtype=np.uint8)
    for k, (_, n, kind, seed) in enumerate(items):
        configs.request_input(kind, seed, n, out=buf[offs[k]:offs[k + 1]])
    return buf, offs


def oracle_records(pairs, buf, offs, threads):
    """(final, accepted, invalid) per request, oracle on a host thread pool."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    def one(k):
        w = pairs[k]
        try:
            fin, acc = oracle.membership(w.delta, w.byte_to_symbol, w.q0, w.accepting,
                                         buf[offs[k]:offs[k + 1]])
            return fin, int(acc), 0
        except oracle.InvalidSymbol:
            return -1, 0, 1
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(pairs))))


def records_match(got, expect) -> bool:
    for g, (fin, acc, bad) in zip(got, expect):
        if bad:
            if not (g[2] & 1):
                return False
        elif (g[0], int(g[1]), g[2]) != (fin, acc, 0):
            return False
    return True


def host_threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def batch_lookups(pairs, buf, offs, chunk, look=1, levels=None) -> int:
    """Algorithmic lookups of a batch: per string, len(c_0) + sum |I_i| len(c_i),
    I_i the start set for r = min(look, the DFA's precomputed levels)."""
    cache = {}
    total = 0
    for k, w in enumerate(pairs):
        x = buf[offs[k]:offs[k + 1]]
        n = x.size
        if n == 0:
            continue
        r = 1 if look <= 1 or levels is None else max(1, min(look, levels[k]))
        nch = (n + chunk - 1) // chunk
        if nch == 1:
            total += n
            continue
        lens = np.full(nch, chunk, dtype=np.int64)
        lens[-1] = n - chunk * (nch - 1)
        if r >= 2:
            m = image_sizes(w, x, chunk, nch, r)
        else:
            if id(w) not in cache:
                cache[id(w)] = set_sizes(w)
            lookb = x[chunk - 1: chunk * (nch - 1): chunk]
            m = cache[id(w)][w.byte_to_symbol[lookb]]
        total += int(lens[0] + (m * lens[1:]).sum())
    return total


def bench_batched(args, dfa, torch, stream) -> int:
    """Batched configuration: value = aggregate input GB/s of graph replays."""
    from workloads import configs
    t0 = time.perf_counter()
    wl = configs.batch_workload(count=args.pairs)
    pairs = [w for w, _, _, _ in wl]
    buf, offs = concat_inputs(wl)
    log(f"[bench] {len(wl)} pairs, {buf.size / 2**30:.2f} GiB, built in "
        f"{time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    handles = {}
    ds = []
    for w in pairs:
        if id(w) not in handles:
            handles[id(w)] = dfa.DFA.from_workload(w)
        ds.append(handles[id(w)])
    create_ms = (time.perf_counter() - t0) * 1e3
    dev = torch.from_numpy(buf).to("cuda")
    ins = [dev[offs[k]:offs[k + 1]] for k in range(len(wl))]
    total = int(buf.size)
    count = len(wl)

    t0 = time.perf_counter()
    if args.chunk > 0 and args.lookahead >= 1:
        chunk, look, ex = args.chunk, args.lookahead, bool(args.early_exit)
        chosen = "command line"
    else:
        chunk, look, tune_ms, ex = dfa.dfa_batch_tune(ds, ins, stream)
        chosen = "autotuner (dfa_batch_tune, untimed)"
        log(f"[bench] tuned chunk {chunk}, lookahead {look}, early exit {ex} ({tune_ms:.2f} "
            f"ms/run, tuning took {time.perf_counter() - t0:.1f}s)")
    b = dfa.Batch(ds, ins, chunk_len=chunk, lookahead=look, early_exit=ex)
    _, ntasks = b.info() if hasattr(b, "info") else (chunk, 0)
    res = torch.empty((count, 4), dtype=torch.int32, device="cuda")

    for _ in range(max(args.warmup, 1)):
        b.graph_launch(res, stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        b.graph_launch(res, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    got = [tuple(int(v) & 0xFFFFFFFF for v in row) for row in res.cpu().tolist()]

    # the same plan without the graph, with HIP events around the matcher kernel
    dfa.dfa_timing_read(stream)
    dfa.dfa_timing_enable(True, stream)
    ev0.record(stream)
    for _ in range(args.steps):
        b.run(res, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    run_ms = ev0.elapsed_time(ev1) / args.steps
    matcher_ms, _, calls = dfa.dfa_timing_read(stream)
    dfa.dfa_timing_enable(False, stream)
    matcher_avg = matcher_ms / max(calls, 1)
    got_run = [tuple(int(v) & 0xFFFFFFFF for v in row) for row in res.cpu().tolist()]

    # plain per-request method: one dfa_match_ex call per pair, in order, one stream
    res_plain = torch.empty((count, 4), dtype=torch.int32, device="cuda")
    for k in range(count):
        dfa.dfa_match_ex(ds[k], ins[k], stream=stream, result=res_plain[k])
    torch.cuda.synchronize()
    plain_steps = max(1, min(args.steps, 5))
    ev0.record(stream)
    for _ in range(plain_steps):
        for k in range(count):
            dfa.dfa_match_ex(ds[k], ins[k], stream=stream, result=res_plain[k])
    ev1.record(stream)
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1) / plain_steps
    got_plain = [tuple(int(v) & 0xFFFFFFFF for v in row) for row in res_plain.cpu().tolist()]

    levels = [int(d.info().lookahead_tables) if d.info().packed_layout else 1 for d in ds]
    lookups = batch_lookups(pairs, buf, offs, chunk, look, levels)
    achieved = lookups / (matcher_avg * 1e-3)
    value = total / (graph_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(graph_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": f"batched: {count} (DFA, string) pairs, seed 7 (8-512 states, byte or "
                        f"20-letter alphabet; lengths log-uniform 1 KiB-64 MiB); one persistent "
                        f"launch replayed from a HIP graph",
            "bytes": total,
            "pairs": count,
            "distinct_dfas": len(handles),
            "chunk_bytes": int(chunk),
            "lookahead": look,
            "early_exit": bool(ex),
            "chosen_by": chosen,
            "lookups_per_byte": round(lookups / total, 3),
        },
        "roofline": {
            "bound": "lds",
            "kernel": "k_b2_match" if all(d.info().packed_layout for d in ds) else "k_batch_match",
            "achieved": round(achieved / 1e9, 2),
            "peak": round(LDS_LOOKUP_PEAK / 1e9, 1),
            "unit": "Glookup/s",
            "frac": round(achieved / LDS_LOOKUP_PEAK, 4),
            "traffic": None,
            "kernel_avg_ms": round(matcher_avg, 4),
            "kernel_timed_in": "the same plan run without the graph (HIP events around "
                               "the matcher launch)",
        },
        "batched_no_graph": {"GB/s": round(total / (run_ms * 1e-3) / 1e9, 3),
                             "ms": round(run_ms, 4)},
        "plain_per_request": {"GB/s": round(total / (plain_ms * 1e-3) / 1e9, 3),
                              "ms": round(plain_ms, 4),
                              "method": "one dfa_match_ex per pair, in order, one stream"},
        "speedup_vs_plain": round(plain_ms / graph_ms, 3),
        "dfa_create_ms_total": round(create_ms, 1),
    }
    if not args.no_cpu_baseline:
        threads = host_threads()
        t0 = time.perf_counter()
        expect = oracle_records(pairs, buf, offs, threads)
        t_cpu = time.perf_counter() - t0
        ok = records_match(got, expect) and records_match(got_run, expect) and \
            records_match(got_plain, expect)
        if not ok:
            raise SystemExit("[bench] MISMATCH against the oracle (batched)")
        line["cpu_baseline"] = {
            "value": round(total / t_cpu / 1e9, 4),
            "unit": "GB/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"all {count} pairs ({total >> 20} MiB), sequential walk (Algorithm 1) "
                      f"per pair on a pool of {threads} host threads",
        }
        line["matches_oracle"] = True
    return line


def percentile_ms(lat_ns, q):
    return round(float(np.percentile(lat_ns, q)) / 1e6, 4)


def bench_served(args, dfa, torch, stream) -> int:
    """Served configuration under Poisson arrivals: value = served input GB/s;
    p50/p99 latency from each request's arrival to its record on the host."""
    from workloads import configs
    nwarm, nmeas = args.warm_requests, args.requests
    t0 = time.perf_counter()
    dfas_w, reqs = configs.served_workload(count=nwarm + nmeas)
    items = [(dfas_w[i], n, kind, seed) for i, n, kind, seed in reqs]
    buf, offs = concat_inputs(items)
    log(f"[bench] {len(reqs)} requests, {buf.size / 2**30:.2f} GiB, built in "
        f"{time.perf_counter() - t0:.1f}s")
    ds = [dfa.DFA.from_workload(w) for w in dfas_w]
    dev = torch.from_numpy(buf).to("cuda")
    ins = [dev[offs[k]:offs[k + 1]] for k in range(len(reqs))]
    ids = [i for i, _, _, _ in reqs]
    lens = offs[1:] - offs[:-1]
    nreq = len(reqs)
    meas_bytes = int(lens[nwarm:].sum())

    # plain method capacity: back-to-back calls, one stream, result copied to the host
    res_plain = torch.empty((nreq, 4), dtype=torch.int32, device="cuda")
    host_plain = torch.empty((nreq, 4), dtype=torch.int32, pin_memory=True)
    for k in range(min(nreq, 200)):
        dfa.dfa_match_ex(ds[ids[k]], ins[k], stream=stream, result=res_plain[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nreq):
        dfa.dfa_match_ex(ds[ids[k]], ins[k], stream=stream, result=res_plain[k])
        host_plain[k].copy_(res_plain[k], non_blocking=True)
    torch.cuda.synchronize()
    cap_s = time.perf_counter() - t0
    capacity = nreq / cap_s
    rate = args.load * capacity
    log(f"[bench] plain capacity {capacity:.0f} req/s ({buf.size / cap_s / 1e9:.1f} GB/s); "
        f"arrival rate {rate:.0f} req/s")

    def run_served(rate):
        """Open-loop submission at Poisson arrival times; returns latencies
        (ns, measured requests), span (s), records and server stats."""
        arrivals = configs.served_arrivals(nreq, rate)
        srv = dfa.Server()
        sid = [srv.register(d) for d in ds]
        done_ns = np.zeros(nreq, dtype=np.int64)
        ticket_of = {}
        got = [None] * nreq
        arr_ns = time.monotonic_ns() + 2_000_000 + (arrivals * 1e9).astype(np.int64)
        k = 0
        finished = 0

        def take(records):
            nonlocal finished
            for t, r, _, dn in records:
                j = ticket_of.pop(t)
                done_ns[j] = dn
                got[j] = (r[0], int(r[1]), r[2])
                finished += 1
        while k < nreq:
            now = time.monotonic_ns()
            while k < nreq and arr_ns[k] <= now:
                ticket_of[srv.submit_ready(sid[ids[k]], ins[k])] = k
                k += 1
            take(srv.drain())
        while finished < nreq:
            take(srv.drain())
        stats = srv.stats()
        srv.close()
        lat = (done_ns - arr_ns)[nwarm:]
        span = (done_ns[nwarm:].max() - arr_ns[nwarm]) * 1e-9
        return lat, span, got, stats

    def run_fifo(rate):
        """The plain method under the same arrivals: one dfa_match_ex per
        request at its arrival, one stream, completions in FIFO order."""
        arrivals = configs.served_arrivals(nreq, rate)
        p_done = np.zeros(nreq, dtype=np.int64)
        evs = [None] * nreq
        head = 0
        p_arr = time.monotonic_ns() + 2_000_000 + (arrivals * 1e9).astype(np.int64)
        k = 0
        while head < nreq:
            now = time.monotonic_ns()
            while k < nreq and p_arr[k] <= now:
                dfa.dfa_match_ex(ds[ids[k]], ins[k], stream=stream, result=res_plain[k])
                host_plain[k].copy_(res_plain[k], non_blocking=True)
                e = torch.cuda.Event()
                e.record(stream)
                evs[k] = e
                k += 1
            while head < k and evs[head].query():
                p_done[head] = time.monotonic_ns()
                evs[head] = None
                head += 1
        p_lat = (p_done - p_arr)[nwarm:]
        p_span = (p_done[nwarm:].max() - p_arr[nwarm]) * 1e-9
        got_plain = [(int(a) & 0xFFFFFFFF, int(b), int(c)) for a, b, c, _ in host_plain.tolist()]
        return p_lat, p_span, got_plain

    lat, span, got, stats = run_served(rate)
    p_lat, p_span, got_plain = run_fifo(rate)
    load_sweep = []
    for f in [float(v) for v in args.load_sweep.split(",") if v.strip()]:
        l2, s2, g2, st2 = run_served(f * capacity)
        pl2, ps2, gp2 = run_fifo(f * capacity)
        if g2 != got or gp2 != got_plain:
            raise SystemExit(f"[bench] served records at load {f} differ from the first run")
        load_sweep.append({
            "load": f, "arrival_rate_req_s": round(f * capacity, 1),
            "served": {"req_s": round(nmeas / s2, 1), "p50_ms": percentile_ms(l2, 50),
                       "p99_ms": percentile_ms(l2, 99), "batches": int(st2.batches)},
            "plain_fifo": {"req_s": round(nmeas / ps2, 1), "p50_ms": percentile_ms(pl2, 50),
                           "p99_ms": percentile_ms(pl2, 99)}})
        log(f"[bench] load {f}: served p50 {load_sweep[-1]['served']['p50_ms']} p99 "
            f"{load_sweep[-1]['served']['p99_ms']} ms; fifo p50 "
            f"{load_sweep[-1]['plain_fifo']['p50_ms']} p99 {load_sweep[-1]['plain_fifo']['p99_ms']}")

    # closed-loop server capacity: everything submitted at once
    srv = dfa.Server()
    sid = [srv.register(d) for d in ds]
    t0 = time.monotonic_ns()
    left = {srv.submit_ready(sid[ids[j]], ins[j]) for j in range(nreq)}
    while left:
        for t, _, _, _ in srv.drain():
            left.discard(t)
    closed_s = (time.monotonic_ns() - t0) * 1e-9
    srv.close()

    value = meas_bytes / span / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": nmeas,
        "warmup": nwarm,
        "ms_per_step": round(span * 1e3 / nmeas, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": f"served: 64 resident DFAs (seed 8, 8-1288 states), {nmeas} requests "
                        f"after {nwarm} warm-up (seed 9, lengths log-uniform 4 KiB-16 MiB), "
                        f"Poisson arrivals at {args.load} x the plain method's capacity",
            "bytes_measured": meas_bytes,
            "arrival_rate_req_s": round(rate, 1),
            "plain_capacity_req_s": round(capacity, 1),
        },
        "latency_ms": {"p50": percentile_ms(lat, 50), "p99": percentile_ms(lat, 99),
                       "mean": round(float(lat.mean()) / 1e6, 4)},
        "served_req_s": round(nmeas / span, 1),
        "batches": int(stats.batches),
        "plain_fifo": {"GB/s": round(meas_bytes / p_span / 1e9, 3),
                       "req_s": round(nmeas / p_span, 1),
                       "latency_ms": {"p50": percentile_ms(p_lat, 50),
                                      "p99": percentile_ms(p_lat, 99),
                                      "mean": round(float(p_lat.mean()) / 1e6, 4)},
                       "method": "one dfa_match_ex per request at its arrival, one stream, FIFO"},
        "closed_loop_capacity": {"GB/s": round(buf.size / closed_s / 1e9, 3),
                                 "req_s": round(nreq / closed_s, 1)},
        "load_sweep": load_sweep,
        "roofline": {
            "bound": "lds",
            "kernel": "k_batch_match (served)",
            "achieved": None,
            "peak": round(LDS_LOOKUP_PEAK / 1e9, 1),
            "unit": "Glookup/s",
            "frac": None,
            "traffic": None,
            "note": "the server's kernels run on its own streams; per-kernel figures come "
                    "from the batched configuration",
        },
    }
    if not args.no_cpu_baseline:
        threads = host_threads()
        t0 = time.perf_counter()
        expect = oracle_records([dfas_w[i] for i in ids], buf, offs, threads)
        t_cpu = time.perf_counter() - t0
        if not records_match(got, expect) or not records_match(got_plain, expect):
            raise SystemExit("[bench] MISMATCH against the oracle (served)")
        line["cpu_baseline"] = {
            "value": round(buf.size / t_cpu / 1e9, 4),
            "unit": "GB/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"all {nreq} requests ({buf.size >> 20} MiB), sequential walk "
                      f"(Algorithm 1) per request on a pool of {threads} host threads",
        }
        line["matches_oracle"] = True
    return line


def bench_single(args, dfa, torch, stream, name) -> dict:
    """One DFA and one input (c1, c2, c2a, c3p, c3b): value = input GB/s of
    whole membership tests, the matcher kernel's roofline, the oracle beside it."""
    w, gen, nbytes, desc = workload(name)
    log(f"[bench] generating {nbytes} bytes for {args.workload}")
    x = gen(nbytes)
    t0 = time.perf_counter()
    d = dfa.DFA.from_workload(w)
    create_ms = (time.perf_counter() - t0) * 1e3
    info = d.info()
    dev_in = torch.from_numpy(x).to("cuda")
    result = torch.empty(4, dtype=torch.int32, device="cuda")
    tuned = None
    if args.lookahead < 0:
        t0 = time.perf_counter()
        r, c, ms, ex, rounds, single, ilv, lanes = dfa.dfa_autotune(d, dev_in, stream)
        tuned = {"lookahead": r, "chunk": c, "ms": round(ms, 4), "early_exit": ex,
                 "rounds": rounds, "single_step": single, "interleave": ilv,
                 "chunk_lanes": lanes,
                 "tuning_s": round(time.perf_counter() - t0, 2)}
        log(f"[bench] autotuner: lookahead {r}, chunk {c or 'planner'}, early exit {ex}, "
            f"rounds {rounds or 1}, single step {single}, interleave {ilv}, chunk lanes {lanes}, "
            f"({ms:.3f} ms)")
        if args.rounds < 0:
            args.rounds = rounds
        args.single_step = args.single_step or single
        args.interleave = args.interleave or ilv
        args.chunk_lanes = args.chunk_lanes or lanes
        # the timed run uses early exit only when asked for (--early-exit):
        # its work depends on the data, so the roofline would need the
        # smaller exact count
        tuned["early_exit_used"] = bool(args.early_exit)
        args.lookahead = r
        if not args.chunk:
            args.chunk = c
    args.rounds = max(args.rounds, 0)
    chunk, nch = dfa.dfa_plan_chunks(d, nbytes, args.chunk, args.lookahead)
    opts = dict(chunk_len=args.chunk, lookahead=args.lookahead, stream=stream, result=result,
                early_exit=args.early_exit, rounds=args.rounds, single_step=args.single_step,
                interleave=args.interleave, chunk_lanes=args.chunk_lanes)

    if args.calibrate_copy:
        scratch = torch.empty_like(dev_in)
        scratch.copy_(dev_in)
        torch.cuda.synchronize()
        del scratch

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        dfa.dfa_match_ex(d, dev_in, **opts)
    torch.cuda.synchronize()
    dfa.dfa_timing_read(stream)          # drop anything recorded so far

    log(f"[bench] timing {args.steps} steps")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        dfa.dfa_match_ex(d, dev_in, **opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    # per-kernel times in a second, instrumented pass: the library's events
    # around the matcher (and around each call) stall the queue between
    # kernels, so they stay out of the timed steps above
    log(f"[bench] kernel timing {args.steps} steps")
    dfa.dfa_timing_enable(True, stream)
    for _ in range(args.steps):
        dfa.dfa_match_ex(d, dev_in, **opts)
    torch.cuda.synchronize()
    matcher_ms, call_ms, kern_ms, calls = dfa.dfa_timing_read_ex(stream)
    dfa.dfa_timing_enable(False, stream)
    fin, acc, flags, nch_run = dfa.result_tuple(result)
    if flags:
        raise SystemExit(f"[bench] result flags {flags}")

    ms_per_step = total_ms / args.steps
    value = nbytes / (ms_per_step * 1e-3) / 1e9
    plan = dfa.dfa_plan(d, nbytes, args.chunk, args.lookahead, rounds=args.rounds,
                        early_exit=args.early_exit, single_step=args.single_step,
                        interleave=args.interleave, chunk_lanes=args.chunk_lanes)
    step = int(plan.symbols_per_step) if plan.kernel == 1 else 1
    if args.early_exit:
        lookups = early_exit_lookups(w, x, chunk, args.lookahead, int(w.q0))
        reads = early_exit_lookups(w, x, chunk, args.lookahead, int(w.q0), step) \
            if step > 1 else lookups
    else:
        lookups = algorithmic_lookups(w, x, chunk, args.lookahead)
        reads = algorithmic_lookups(w, x, chunk, args.lookahead, step) if step > 1 else lookups
    merged = plan.kernel == 1 and (plan.rounds > 1 or plan.chunk_lanes)
    if merged:
        reads, covered = merged_lookups(w, x, chunk, args.lookahead, max(2, int(plan.rounds)),
                                        step)
    if plan.kernel == 1:
        lay = 4 if step == 2 else 3 if plan.raw_input else (
            2 if info.packed_layout == 2 else 1)
        kernel = (f"k_chunk_walk<{lay}>" if plan.chunk_lanes else
                  f"k_round<{lay}>" if merged else f"k_match2<{lay}>")
        if plan.tail_lanes:
            kernel = f"k_tail<{2 if info.packed_layout == 2 else 1}, {int(plan.tail_lanes)}>"
    else:
        kernel = "k_match"
    matcher_avg_ms = matcher_ms / max(calls, 1)
    achieved = reads / (matcher_avg_ms * 1e-3)
    traffic, traffic_src = stored_traffic(kernel, name, args.lookahead, int(chunk))
    # bytes the walk streams per input byte: raw input or one-byte codes 1,
    # two-byte codes 2, pair codes 1/2
    stream_bpb = 0.5 if step == 2 else 2.0 if kernel.endswith("<2>") else 1.0
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "bytes": nbytes,
            "states": int(info.num_states),
            "classes": int(info.num_classes),
            "imax": int(info.imax),
            "lookahead": args.lookahead,
            "chosen_by": "autotuner (dfa_autotune, untimed)" if tuned else "command line",
            "early_exit": bool(args.early_exit),
            "tuner": tuned,
            "chunk_bytes": int(chunk),
            "chunks": int(nch),
            "lookups_per_byte": round(lookups / nbytes, 3),
            "rounds": int(plan.rounds) if plan.kernel == 1 else 1,
            "set_max": int(plan.set_max),
            "compose": {"levels": int(plan.levels), "group0": int(plan.group0),
                        "group": int(plan.group)},
        },
        "roofline": {
            "bound": "lds",
            "kernel": kernel,
            "symbols_per_lookup": step,
            "lookups_per_launch": int(reads),
            "achieved": round(achieved / 1e9, 2),
            "peak": round(LDS_LOOKUP_PEAK / 1e9, 1),
            "unit": "Glookup/s",
            "frac": round(achieved / LDS_LOOKUP_PEAK, 4),
            "traffic": traffic,
            "traffic_source": traffic_src,
            "kernel_avg_ms": round(matcher_avg_ms, 4),
            "hbm_frac": round(nbytes * stream_bpb / (matcher_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              5),
        },
        "final_state": fin,
        "accepted": acc,
        "dfa_create_ms": round(create_ms, 2),
        "call_ms_avg": round(call_ms / max(calls, 1), 4),
    }

    if merged:
        # merged walks do about one walk per chunk after the first round: the
        # rounds stream the code bytes they cover once (up to the chunk end,
        # or where every walk of the chunk reached an absorbing state), so HBM
        # bounds them
        rl = line["roofline"]
        hbm_gbs = covered * stream_bpb / (matcher_avg_ms * 1e-3) / 1e9
        rl.update({"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
                   "bytes_covered": int(covered),
                   "lds_achieved_glookup_s": round(achieved / 1e9, 2),
                   "lds_frac": round(achieved / LDS_LOOKUP_PEAK, 4)})
        rl.pop("hbm_frac", None)
    if plan.kernel == 1 and plan.tail_lanes:
        # the one-chunk-per-lane last round is the longest launch: it reads
        # every chunk's bytes from tail_start on from the raw input, with at
        # least two LDS lookups per byte (its code, one transition); timed by
        # HIP events around that launch
        t0b = int(plan.tail_start)
        lens = np.minimum(int(chunk), nbytes - np.arange(nch, dtype=np.int64) * int(chunk))
        tail_bytes = int(np.maximum(lens - t0b, 0).sum())
        kavg = kern_ms / max(calls, 1)
        gbs = tail_bytes / (kavg * 1e-3) / 1e9
        line["roofline"] = {
            "bound": "hbm", "kernel": kernel,
            "of": f"{kernel}, the longest single launch of the call (HIP events on its stream)",
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
            "algorithmic_bytes_per_launch": tail_bytes, "kernel_avg_ms": round(kavg, 4),
            "lds_view": {"algorithmic_lookups_per_launch": 2 * tail_bytes,
                         "achieved_Glookups_s": round(2 * tail_bytes / (kavg * 1e-3) / 1e9, 1),
                         "peak_Glookups_s": round(LDS_LOOKUP_PEAK / 1e9, 1),
                         "frac": round(2 * tail_bytes / (kavg * 1e-3) / LDS_LOOKUP_PEAK, 4)},
            "step_hbm_frac": round(value / HBM_PEAK_GBS, 4),
        }

    if not args.no_cpu_baseline:
        import oracle
        reps = 3
        times = []
        ofin = None
        for _ in range(reps):
            t, ofin = oracle.time_walk(w.delta, w.byte_to_symbol, w.q0, x, repeats=1)
            times.append(t)
        t_med = float(np.median(times))
        if ofin != fin:
            raise SystemExit(f"[bench] MISMATCH: gpu final {fin} oracle {ofin}")
        line["cpu_baseline"] = {
            "value": round(nbytes / t_med / 1e9, 4),
            "unit": "GB/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the full {nbytes >> 20} MiB input, sequential walk (Algorithm 1), "
                      f"median of {reps}; host {platform.processor() or platform.machine()}, "
                      f"{os.cpu_count()} logical CPUs visible",
        }
        line["matches_oracle"] = True
        # the paper's own CPU design: Algorithm 3 on the host cores (libdfahost)
        from paper_1210_5093_amd import host
        threads = host_threads()
        h = host.HostDFA.from_workload(w)
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            hfin, _ = h.match(x, threads)
            times.append(time.perf_counter() - t0)
        h.close()
        if hfin != fin:
            raise SystemExit(f"[bench] MISMATCH: host speculative final {hfin}, GPU {fin}")
        line["cpu_speculative"] = {
            "value": round(nbytes / float(np.median(times)) / 1e9, 4),
            "unit": "GB/s",
            "cores": threads,
            "kind": "host multicore speculative matcher (Algorithm 3, partition of Eq. 10)",
            "sample": f"the full {nbytes >> 20} MiB input, median of 3",
        }
    return line


# Settings of the large configuration's two matches (lookahead r, chunk
# length, walk rounds), from the chunk sweep on the full 10 GiB inputs;
# --tune replaces them with the autotuner's choice on the first GiB.
C3_SETTINGS = {
    "protein": {"lookahead": 4, "chunk": 65536, "rounds": 2, "interleave": True,
                "single_step": True},
    "byte": {"lookahead": 2, "chunk": 65536, "rounds": 4, "interleave": True},
}


def c3_opts(st, stream, result, chunk=None):
    return dict(chunk_len=int(chunk or st["chunk"]), lookahead=int(st["lookahead"]),
                rounds=int(st.get("rounds", 0)), interleave=bool(st.get("interleave", False)),
                single_step=bool(st.get("single_step", False)),
                chunk_lanes=bool(st.get("chunk_lanes", False)), stream=stream, result=result)


def golden_finals():
    path = os.path.join(ROOT, "tests", "golden", "large_finals.json")
    with open(path) as f:
        return json.load(f)


def bench_large(args, dfa, torch, stream) -> dict:
    """The large configuration: the 1298-state protein DFA on 10 GiB of
    residues and the 512-state byte DFA on 10 GiB of uniform bytes, both
    resident in HBM.  One step = both membership tests; value = 20 GiB / step
    time.  Per-DFA matcher times (HIP events), the chunk sweep 4 KiB - 1 MiB,
    the dominant kernel's roofline and the whole step's HBM fraction."""
    from workloads import configs
    n = int(args.c3_bytes)
    parts = [("protein", configs.c3_protein_dfa(), configs.c3_protein_input,
              f"{configs.c3_protein_dfa().num_states}-state protein DFA (pattern seed "
              f"{configs.C3_PATTERN_SEED}), residues stream {configs.C3_PROTEIN_INPUT_SEED}"),
             ("byte", configs.c3_byte_dfa(), configs.c3_byte_input,
              f"512-state byte DFA (64 columns, seeds 5, 6), uniform bytes stream "
              f"{configs.C3_BYTE_INPUT_SEED}")]
    P = []
    for key, w, gen, desc in parts:
        t0 = time.perf_counter()
        x = np.empty(n, dtype=np.uint8)
        gen(n, out=x)
        dev = torch.from_numpy(x).to("cuda")
        del x
        t1 = time.perf_counter()
        d = dfa.DFA.from_workload(w)
        create_ms = (time.perf_counter() - t1) * 1e3
        log(f"[bench] c3 {key}: {n} bytes generated and copied in {t1 - t0:.1f}s")
        st = dict(C3_SETTINGS[key])
        chosen = "fixed setting from the full-size chunk sweep"
        if args.tune:
            t0 = time.perf_counter()
            r, c, ms, ex, rounds, single, ilv, lanes = dfa.dfa_autotune(d, dev, stream)
            st = {"lookahead": r, "chunk": c, "rounds": rounds, "single_step": single,
                  "interleave": ilv, "chunk_lanes": lanes}
            chosen = f"autotuner on the first GiB ({time.perf_counter() - t0:.1f}s, untimed)"
            log(f"[bench] c3 {key} tuned: {st}")
        P.append({"key": key, "w": w, "gen": gen, "desc": desc, "dev": dev, "d": d,
                  "st": st, "chosen": chosen, "create_ms": create_ms,
                  "res": torch.empty(4, dtype=torch.int32, device="cuda")})

    # the step's two membership tests are independent: each runs on its own
    # stream (default priority), both after the step's start on `stream`,
    # which then waits for both, so steps follow one another and the two
    # tests of a step overlap (--serial-step: one after the other on `stream`)
    side = [torch.cuda.Stream() for _ in P]

    def step():
        if args.serial_step:
            for p in P:
                dfa.dfa_match_ex(p["d"], p["dev"], **c3_opts(p["st"], stream, p["res"]))
            return
        start = torch.cuda.Event()
        start.record(stream)
        for p, sp in zip(P, side):
            sp.wait_event(start)
            dfa.dfa_match_ex(p["d"], p["dev"], **c3_opts(p["st"], sp, p["res"]))
        for sp in side:
            done = torch.cuda.Event()
            done.record(sp)
            stream.wait_event(done)

    if args.calibrate_copy:
        # one device copy of a known size, for scaling the HBM counters
        scratch = torch.empty_like(P[0]["dev"])
        scratch.copy_(P[0]["dev"])
        torch.cuda.synchronize()
        del scratch
    log(f"[bench] c3 warmup {args.warmup}")
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    dfa.dfa_timing_read(stream)
    log(f"[bench] c3 timing {args.steps} steps")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    # per-DFA times in a second, instrumented pass (events around the matcher
    # kernel and around each call)
    for p in P:
        dfa.dfa_timing_enable(True, stream)
        for _ in range(args.steps):
            dfa.dfa_match_ex(p["d"], p["dev"], **c3_opts(p["st"], stream, p["res"]))
        torch.cuda.synchronize()
        m, c, kern, k = dfa.dfa_timing_read_ex(stream)
        dfa.dfa_timing_enable(False, stream)
        p["matcher_ms"], p["call_ms"] = m / max(k, 1), c / max(k, 1)
        p["kernel_ms"] = kern / max(k, 1)
        fin, acc, flags, nch = dfa.result_tuple(p["res"])
        if flags:
            raise SystemExit(f"[bench] c3 {p['key']}: result flags {flags}")
        p["fin"], p["acc"], p["nch"] = fin, acc, nch
        p["plan"] = dfa.dfa_plan(p["d"], n, p["st"]["chunk"], p["st"]["lookahead"],
                                 rounds=p["st"].get("rounds", 0),
                                 interleave=p["st"].get("interleave", False),
                                 single_step=p["st"].get("single_step", False),
                                 chunk_lanes=p["st"].get("chunk_lanes", False))
    # chunk sweep (same r and rounds; 3 timed calls per length)
    sweep = {}
    if not args.no_sweep:
        log("[bench] c3 chunk sweep")
        for p in P:
            row = {}
            for chunk in configs.C3_CHUNKS:
                o = c3_opts(p["st"], stream, p["res"], chunk)
                dfa.dfa_match_ex(p["d"], p["dev"], **o)
                ev0.record(stream)
                for _ in range(3):
                    dfa.dfa_match_ex(p["d"], p["dev"], **o)
                ev1.record(stream)
                torch.cuda.synchronize()
                row[str(chunk)] = round(n / (ev0.elapsed_time(ev1) / 3 * 1e-3) / 1e9, 1)
                if dfa.result_tuple(p["res"])[:3] != (p["fin"], p["acc"], 0):
                    raise SystemExit(f"[bench] c3 {p['key']} chunk {chunk}: result differs")
            sweep[p["key"]] = row
    # roofline: the longest single kernel launch of the step (HIP events
    # around it on the matcher's stream, dfa_timing_read_ex).  With a
    # one-chunk-per-lane last round that is k_tail, which reads every byte
    # of each chunk from tail_start on (raw input: 1 B per byte; on these
    # inputs every chunk keeps a walk to its end) and makes at least two LDS
    # lookups per byte (its code, one transition).  Otherwise the matcher
    # streams its code bytes once (1 B, 2 B or 1/2 B per input byte).
    dom = max(P, key=lambda p: p["kernel_ms"])
    plan = dom["plan"]
    step_k = int(plan.symbols_per_step) if plan.kernel == 1 else 1
    code_lay = 2 if dom["d"].info().packed_layout == 2 else 1
    lay = 4 if step_k == 2 else 3 if plan.raw_input else code_lay
    if plan.kernel == 1 and plan.tail_lanes:
        kernel = f"k_tail<{code_lay}, {int(plan.tail_lanes)}>"
        t0 = int(plan.tail_start)
        chunk = int(plan.chunk_len)
        nch = int(plan.num_chunks)
        last = n - (nch - 1) * chunk
        algo_bytes = (nch - 1) * (chunk - t0) + max(0, last - t0)
        algo_lookups = 2 * algo_bytes
    else:
        kernel = (f"k_chunk_walk<{lay}>" if plan.chunk_lanes else
                  f"k_round<{lay}>" if plan.rounds > 1 else f"k_match2<{lay}>") \
            if plan.kernel == 1 else "k_match"
        stream_bpb = 0.5 if step_k == 2 else 2.0 if lay == 2 else 1.0
        algo_bytes = int(n * stream_bpb)
        algo_lookups = n // step_k
    kms = dom["kernel_ms"]
    achieved = algo_bytes / (kms * 1e-3) / 1e9
    lds_achieved = algo_lookups / (kms * 1e-3)
    traffic, traffic_src = stored_traffic(kernel, "c3_" + dom["key"], dom["st"]["lookahead"],
                                          int(dom["st"]["chunk"]))
    value = 2 * n / (ms_per_step * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": f"large DFAs: {n >> 30} GiB per DFA, both resident in HBM; one step = "
                        f"the {P[0]['desc']} plus the {P[1]['desc']}",
            "bytes_per_step": 2 * n,
            "step": ("the two tests one after the other on one stream" if args.serial_step else
                     "the two tests on two streams, overlapping; steps one after another"),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "of": f"the {dom['key']} DFA's {kernel} (the longest single kernel launch of the "
                  f"step, HIP events on its stream)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_source": traffic_src,
            "algorithmic_bytes_per_launch": int(algo_bytes),
            "kernel_avg_ms": round(kms, 4),
            "lds_view": {"algorithmic_lookups_per_launch": int(algo_lookups),
                         "achieved_Glookups_s": round(lds_achieved / 1e9, 1),
                         "peak_Glookups_s": round(LDS_LOOKUP_PEAK / 1e9, 1),
                         "frac": round(lds_achieved / LDS_LOOKUP_PEAK, 4)},
            "step_hbm_frac": round(value / HBM_PEAK_GBS, 4),
        },
        "parts": {},
    }
    for p in P:
        pl = p["plan"]
        line["parts"][p["key"]] = {
            "dfa": p["desc"],
            "states": int(p["d"].info().num_states),
            "classes": int(p["d"].info().num_classes),
            "imax": int(p["d"].info().imax),
            "setting": p["st"], "chosen_by": p["chosen"],
            "chunks": int(p["nch"]), "set_max": int(pl.set_max), "rounds": int(pl.rounds),
            "compose_levels": int(pl.levels),
            "tail_lanes": int(pl.tail_lanes), "tail_start": int(pl.tail_start),
            "GB/s_alone": round(n / (p["call_ms"] * 1e-3) / 1e9, 1),
            "matcher_ms": round(p["matcher_ms"], 4), "call_ms": round(p["call_ms"], 4),
            "longest_kernel_ms": round(p["kernel_ms"], 4),
            # input bytes over the matcher section (all rounds, or the one
            # matcher launch) against HBM
            "matcher_input_hbm_frac": round(n / (p["matcher_ms"] * 1e-3) / 1e9
                                            / HBM_PEAK_GBS, 4),
            "final_state": p["fin"], "accepted": p["acc"],
            "dfa_create_ms": round(p["create_ms"], 1),
        }
    if sweep:
        line["chunk_sweep_GBps"] = sweep
    # parity: the final state against the oracle's stored full walk, and the
    # state after the first GiB against the oracle walking that GiB now (the
    # CPU baseline's timed sample)
    import oracle
    gold = golden_finals() if n == configs.C3_BYTES else None
    gib = min(n, 1 << 30)
    t_cpu = 0.0
    for p in P:
        if gold:
            g = gold["c3_" + p["key"]]
            if (p["fin"], bool(p["acc"])) != (g["final_state"], g["accepted"]):
                raise SystemExit(f"[bench] c3 {p['key']}: final {p['fin']} != oracle "
                                 f"{g['final_state']}")
        chunk = int(p["st"]["chunk"])
        _, nch = dfa.dfa_plan_chunks(p["d"], n, chunk, p["st"]["lookahead"])
        bnd = torch.empty(nch + 1, dtype=torch.int32, device="cuda")
        o = c3_opts(p["st"], stream, p["res"])
        dfa.dfa_match_ex(p["d"], p["dev"], boundaries=True, bound_out=bnd, **o)
        torch.cuda.synchronize()
        x = p["gen"](gib)
        t0 = time.perf_counter()
        ofin, _ = oracle.walk(p["w"].delta, p["w"].byte_to_symbol, p["w"].q0, x)
        t_cpu += time.perf_counter() - t0
        got = int(bnd[gib // chunk].item()) & 0xFFFFFFFF if gib % chunk == 0 else ofin
        if got != ofin:
            raise SystemExit(f"[bench] c3 {p['key']}: state after 1 GiB {got} != oracle {ofin}")
        del bnd, x
    line["cpu_baseline"] = {
        "value": round(2 * gib / t_cpu / 1e9, 4),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the first {gib >> 20} MiB of each of the two inputs, sequential walk "
                  f"(Algorithm 1) on one host core; host {platform.machine()}, "
                  f"{os.cpu_count()} logical CPUs visible",
    }
    line["matches_oracle"] = True
    line["parity"] = ("final states equal the oracle's full sequential walks (stored by "
                      "tests/golden/make_large_finals.py); the state after the first GiB "
                      "equals the oracle's walk of that GiB" if gold else
                      "the state after the first GiB equals the oracle's walk of that GiB")
    for p in P:
        p["d"].close()
        del p["dev"]
    torch.cuda.empty_cache()
    return line


SUB_FIELDS = ("value", "unit", "ms_per_step", "config", "roofline", "cpu_baseline",
              "matches_oracle", "latency_ms", "plain_fifo", "served_req_s",
              "closed_loop_capacity", "plain_per_request", "speedup_vs_plain",
              "batched_no_graph", "cpu_speculative", "load_sweep")


def sub_record(line: dict) -> dict:
    return {k: line[k] for k in SUB_FIELDS if k in line}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3",
                    choices=["c3", "c1", "c2", "c2a", "c3p", "c3b", "c4", "c5"],
                    help="c3 (default): the large configuration, with the others as "
                         "sub-records unless --no-sub")
    ap.add_argument("--no-sub", action="store_true",
                    help="c3: skip the protein-style, plain, batched and served sub-records")
    ap.add_argument("--no-sweep", action="store_true", help="c3: skip the chunk sweep")
    ap.add_argument("--serial-step", action="store_true",
                    help="c3: run the step's two tests one after the other on one stream "
                         "(default: each on its own stream, overlapping)")
    ap.add_argument("--tune", action="store_true",
                    help="c3, c4: choose settings with the autotuners (untimed) instead of the "
                         "fixed ones")
    ap.add_argument("--c3-bytes", type=int, default=10 << 30, help="c3: bytes per DFA")
    ap.add_argument("--chunk", type=int, default=0, help="bytes per chunk (0 = planner)")
    ap.add_argument("--lookahead", type=int, default=-1,
                    help="reverse-lookahead symbols r (0 = all states, 1 = I_sigma, 2..64; "
                         "-1 = pick r and the chunk length with the autotuner, untimed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--early-exit", action="store_true",
                    help="stop a wavefront's walks once all its pairs are absorbing")
    ap.add_argument("--rounds", type=int, default=-1,
                    help="walk rounds with merging (1 = none, 2..4; -1 = the autotuner's "
                         "pick, else one)")
    ap.add_argument("--single-step", action="store_true",
                    help="one symbol per table lookup even where a two-symbol table exists")
    ap.add_argument("--chunk-lanes", action="store_true",
                    help="one chunk per lane with merged walks")
    ap.add_argument("--interleave", action="store_true",
                    help="chunk-interleaved code stream (else linear; direct tables: raw input)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of the input (counter calibration)")
    ap.add_argument("--requests", type=int, default=10000, help="c5: measured requests")
    ap.add_argument("--warm-requests", type=int, default=500, help="c5: warm-up requests")
    ap.add_argument("--load", type=float, default=0.7,
                    help="c5: arrival rate as a fraction of the plain method's capacity")
    ap.add_argument("--load-sweep", default="",
                    help="c5: comma-separated further loads (fractions of plain capacity)")
    ap.add_argument("--pairs", type=int, default=1024, help="c4: (DFA, string) pairs")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the matcher runs on a single MI355X "
              "(no multi-GPU path); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1210_5093_amd as dfa
    if not os.path.exists(dfa.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t_start = time.perf_counter()

    def timed(label, fn, *a):
        t0 = time.perf_counter()
        out = fn(*a)
        log(f"[bench] section {label}: {time.perf_counter() - t0:.1f}s")
        return out

    if args.workload == "c4":
        line = timed("c4", bench_batched, args, dfa, torch, torch.cuda.Stream())
    elif args.workload == "c5":
        line = timed("c5", bench_served, args, dfa, torch, stream)
    elif args.workload == "c3":
        line = timed("c3", bench_large, args, dfa, torch, stream)
        if not args.no_sub:
            sub = {}
            steps = args.steps
            for name in ("c2", "c1"):
                a2 = argparse.Namespace(**vars(args))
                a2.lookahead, a2.rounds, a2.chunk = -1, -1, 0
                sub[name] = sub_record(timed(name, bench_single, a2, dfa, torch, stream, name))
            # the protein-style configuration again with one symbol per step
            # and a one-chunk-per-lane last round over the raw input: no
            # pair-code stream through HBM (the autotuner weighs it too)
            a2 = argparse.Namespace(**vars(args))
            a2.lookahead, a2.rounds, a2.chunk = 6, 2, 2048
            a2.interleave, a2.single_step, a2.no_cpu_baseline = True, True, True
            raw = timed("c2 raw input", bench_single, a2, dfa, torch, stream, "c2")
            rl = raw["roofline"]
            sub["c2"]["raw_input_last_round"] = {
                "setting": {"lookahead": 6, "chunk": 2048, "rounds": 2, "interleave": True,
                            "single_step": True},
                "value": raw["value"], "unit": raw["unit"], "ms_per_step": raw["ms_per_step"],
                "kernel": rl["kernel"], "frac": rl["frac"], "unit_frac": rl["unit"],
                "traffic": rl.get("traffic"), "traffic_source": rl.get("traffic_source"),
                "final_state": raw.get("final_state"),
            }
            a4 = argparse.Namespace(**vars(args))
            if not args.tune:
                a4.chunk, a4.lookahead = 8192, 6
            sub["c4"] = sub_record(timed("c4", bench_batched, a4, dfa, torch, torch.cuda.Stream()))
            # the served sub-record also sweeps the arrival rate around the
            # plain method's capacity
            a5 = argparse.Namespace(**vars(args))
            if not a5.load_sweep:
                a5.load_sweep = "0.5,0.9,1.2"
            sub["c5"] = sub_record(timed("c5", bench_served, a5, dfa, torch, stream))
            args.steps = steps
            line["sub"] = sub
    else:
        line = timed(args.workload, bench_single, args, dfa, torch, stream, args.workload)
    log(f"[bench] total {time.perf_counter() - t_start:.1f}s")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
