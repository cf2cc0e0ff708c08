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


def algorithmic_lookups(w, x: np.ndarray, chunk: int, lookahead: int) -> int:
    """len(c_0) + sum_{i>=1} |I_i| len(c_i) (Algorithm 3's work; I_i is the
    chunk's start set: all states, I_sigma, or the r-symbol image of Eq. 13)."""
    n = x.size
    nch = (n + chunk - 1) // chunk
    lens = np.full(nch, chunk, dtype=np.int64)
    lens[-1] = n - chunk * (nch - 1)
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3p", "c3b"])
    ap.add_argument("--chunk", type=int, default=0, help="bytes per chunk (0 = planner)")
    ap.add_argument("--lookahead", type=int, default=1,
                    help="reverse-lookahead symbols r (0 = all states, 1 = I_sigma, 2..64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of the input (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs the matcher on a single MI355X "
              "(no multi-GPU path); use --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1210_5093_amd as dfa
    if not os.path.exists(dfa.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    w, gen, nbytes, desc = workload(args.workload)
    log(f"[bench] generating {nbytes} bytes for {args.workload}")
    x = gen(nbytes)
    t0 = time.perf_counter()
    d = dfa.DFA.from_workload(w)
    create_ms = (time.perf_counter() - t0) * 1e3
    info = d.info()
    dev_in = torch.from_numpy(x).to("cuda")
    result = torch.empty(4, dtype=torch.int32, device="cuda")
    chunk, nch = dfa.dfa_plan_chunks(d, nbytes, args.chunk, args.lookahead)
    opts = dict(chunk_len=args.chunk, lookahead=args.lookahead, stream=stream, result=result)

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
    dfa.dfa_timing_enable(True, stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        dfa.dfa_match_ex(d, dev_in, **opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    matcher_ms, call_ms, calls = dfa.dfa_timing_read(stream)
    dfa.dfa_timing_enable(False, stream)
    fin, acc, flags, nch_run = dfa.result_tuple(result)
    if flags:
        log(f"[bench] result flags {flags}")
        return 1

    ms_per_step = total_ms / args.steps
    value = nbytes / (ms_per_step * 1e-3) / 1e9
    lookups = algorithmic_lookups(w, x, chunk, args.lookahead)
    plan = dfa.dfa_plan(d, nbytes, args.chunk, args.lookahead)
    kernel = f"k_match2<{info.packed_layout}>" if plan.kernel == 1 else "k_match"
    matcher_avg_ms = matcher_ms / max(calls, 1)
    achieved = lookups / (matcher_avg_ms * 1e-3)
    line = {
        "metric": "input GB/s per DFA-membership test (bit-exact) vs sequential; "
                  "p99 latency served",
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
            "chunk_bytes": int(chunk),
            "chunks": int(nch),
            "lookups_per_byte": round(lookups / nbytes, 3),
        },
        "roofline": {
            "bound": "lds",
            "kernel": kernel,
            "achieved": round(achieved / 1e9, 2),
            "peak": round(LDS_LOOKUP_PEAK / 1e9, 1),
            "unit": "Glookup/s",
            "frac": round(achieved / LDS_LOOKUP_PEAK, 4),
            "traffic": None,
            "kernel_avg_ms": round(matcher_avg_ms, 4),
            "hbm_frac": round(nbytes / (matcher_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
        },
        "final_state": fin,
        "accepted": acc,
        "dfa_create_ms": round(create_ms, 2),
        "call_ms_avg": round(call_ms / max(calls, 1), 4),
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
            log(f"[bench] MISMATCH: gpu final {fin} oracle {ofin}")
            return 1
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
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
