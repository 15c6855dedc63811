"""Hardware probes of one GPU through the C ABI: the paper's microbenchmarks
and the cache inference fed with real fine-grained P-chase latencies.

    python -m paper_1509_02308_amd.hwprobe stream [--bytes B] [--sweep]
    python -m paper_1509_02308_amd.hwprobe lds
    python -m paper_1509_02308_amd.hwprobe ldsbw
    python -m paper_1509_02308_amd.hwprobe valu
    python -m paper_1509_02308_amd.hwprobe l1 [--flavor 0]
    python -m paper_1509_02308_amd.hwprobe curve --s 128 --n-lo 4096 --n-hi 131072

* stream: copy throughput (Section 5.1) for one launch shape, or the grid of
  shapes (blocks per CU x block size x words in flight per thread).
* lds: average cycles per LDS load against the word stride of the 64 lanes
  (Section 6.2, the bank-conflict sweep).
* ldsbw: LDS throughput over blocks per CU x block size x reads in flight,
  4-byte and 16-byte accesses, read-only and LDS-to-LDS copy (Section 6.1).
* valu: 32-bit VALU lane operations per second over blocks per CU (the
  replay's roofline denominator, measured).
* curve: the classic average-latency curve (Section 4.1): for each array
  size N, the mean and median cycles per access of a P-chase.
* l1: the Section 4.2 procedure on the per-CU vector L1: fine-grained
  P-chase runs with N swept across the candidate capacities and strides
  around the line sizes, the latencies classified into hits and misses by
  the widest gap, and every candidate cache replayed against them with
  infer_cache_params.

Each command prints JSON lines.  Everything runs in the library's kernels;
this file only marshals arguments and formats results.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def _torch_capi():
    import torch
    from paper_1509_02308_amd import capi
    if not torch.cuda.is_available():
        sys.exit("hwprobe needs a GPU")
    torch.cuda.set_device(0)
    return torch, capi


def cmd_stream(a):
    torch, capi = _torch_capi()
    n = a.bytes
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    shapes = [(a.grid, a.block, a.ilp, a.dtype)]
    if a.sweep:
        shapes = [(g * cus, blk, ilp, dt) for dt in (0, 1) for g in (1, 2, 4, 8)
                  for blk in (64, 256, 1024) for ilp in (1, 2, 4, 8)]
    best = None
    for grid, block, ilp, dt in shapes:
        gbps = capi.microbench_hbm_stream(src, dst, n, dt, grid, block, ilp, a.reps)
        row = {"probe": "hbm_stream", "bytes": n, "dtype": ["f32", "f32x4"][dt], "grid": grid,
               "block": block, "ilp": ilp, "reps": a.reps, "GBps": gbps}
        print(json.dumps(row), flush=True)
        if best is None or gbps > best["GBps"]:
            best = row
    if a.sweep:
        print(json.dumps({"probe": "hbm_stream_best", **best}), flush=True)


def cmd_lds(a):
    torch, capi = _torch_capi()
    cyc = torch.zeros(64, dtype=torch.int32, device="cuda")
    capi.microbench_lds_bank(1, 64, a.reps, cyc)
    c = cyc.cpu().numpy() / 100.0
    print(json.dumps({"probe": "lds_bank", "stride_words": list(range(1, 65)),
                      "cycles_per_load": [round(float(v), 2) for v in c]}), flush=True)


def cmd_ldsbw(a):
    torch, capi = _torch_capi()
    best = {}
    for copy in (False, True):
        for width in (4, 16):
            for bpc in (1, 2, 4, 8):
                for block in (64, 256, 1024):
                    for ilp in (1, 2, 4, 8):
                        if bpc * block > 2048:
                            continue
                        g = capi.microbench_lds_stream(bpc, block, ilp, width, a.reps, copy=copy)
                        row = {"probe": "lds_stream", "copy": copy, "width_bytes": width, "blocks_per_cu": bpc,
                               "block": block, "ilp": ilp, "GBps": g,
                               "bytes_per_clk_per_cu": g * 1e9 / (256 * 2.4e9)}
                        print(json.dumps(row), flush=True)
                        if copy not in best or g > best[copy]["GBps"]:
                            best[copy] = row
    for row in best.values():
        print(json.dumps({**row, "probe": "lds_stream_best"}), flush=True)


def cmd_valu(a):
    torch, capi = _torch_capi()
    best = 0.0
    for bpc in (1, 2, 4, 8, 16):
        v = capi.microbench_valu(bpc, a.reps)
        best = max(best, v)
        print(json.dumps({"probe": "valu", "blocks_per_cu": bpc, "lane_ops_per_s": v,
                          "frac_of_nominal": v / (256 * 64 * 2.4e9)}), flush=True)
    print(json.dumps({"probe": "valu_best", "lane_ops_per_s": best, "frac_of_nominal": best / (256 * 64 * 2.4e9)}),
          flush=True)


def _chase(torch, capi, N, s, passes, flavor, arr):
    p = capi.PchaseProbe(N, s, 0, 0, 4, passes)
    L = capi.pchase_trace_len(capi.PchaseProbe(N, s, 0, 0, 4, 1))[0]
    k = passes * L
    lat = torch.zeros(k, dtype=torch.int32, device="cuda")
    idx = torch.zeros(k, dtype=torch.int32, device="cuda")
    ovh = capi.microbench_pchase(p, flavor, arr, k, lat, idx)
    return lat, ovh, L


def cmd_curve(a):
    torch, capi = _torch_capi()
    arr = torch.zeros(a.n_hi // 4 + 64, dtype=torch.int32, device="cuda")
    maxk = capi.pchase_microbench_max_k()
    for N in range(a.n_lo, a.n_hi + 1, a.n_step):
        L = N // a.s
        if L > maxk:
            break
        lat, ovh, L = _chase(torch, capi, N, a.s, 1, a.flavor, arr)
        v = lat.cpu().numpy().view(np.uint32).astype(np.int64) - ovh
        print(json.dumps({"probe": "latency_curve", "N": N, "s": a.s, "flavor": a.flavor, "overhead": ovh,
                          "mean": float(v.mean()), "median": float(np.median(v)), "min": int(v.min()),
                          "max": int(v.max())}), flush=True)


def cmd_l1(a):
    torch, capi = _torch_capi()
    from paper_1509_02308_amd import workloads as W
    # candidates for a per-CU vector L1 of 16-64 KB
    cands = W.candidate_grid(Cs=(16384, 24576, 32768, 49152, 65536), bs=(64, 128),
                             As=(1, 2, 4, 8, 16, 32, 64), policies=(W.LRU, W.FIFO, W.PLRU))
    crows = [tuple(int(v) for v in c) for c in cands]
    carr = capi.models(crows)
    # fine-grained runs: N across [C/2, 2C] of the candidates in line steps, s in {64, 128, 256}
    rows = []
    for s in (64, 128, 256):
        for N in range(8192, 131072 + 1, 1024):
            if 2 * N // s <= capi.pchase_microbench_max_k():
                rows.append((N, s, 2))
    parr = capi.probes(rows)
    arr = torch.zeros(131072 // 4 + 64, dtype=torch.int32, device="cuda")
    lats, offs = [], [0]
    ovhs = []
    for N, s, passes in rows:
        lat, ovh, L = _chase(torch, capi, N, s, passes, a.flavor, arr)
        ovhs.append(ovh)
        lats.append(lat)
        offs.append(offs[-1] + lat.numel())
    lat_all = torch.cat(lats)
    res, zero = capi.infer_cache_params(parr, carr, lat=lat_all, lat_off=np.array(offs, np.uint64),
                                        probe_select=capi.PROBES_ALL, want_zero=True)
    v = lat_all.cpu().numpy().view(np.uint32)
    zc = [crows[i] for i in range(len(crows)) if (zero[i // 32] >> (i % 32)) & 1]
    best = crows[res.best] if res.best >= 0 else None
    print(json.dumps({"probe": "l1_inference", "flavor": a.flavor, "probes": len(rows),
                      "accesses": int(offs[-1]), "candidates": len(crows),
                      "threshold_cycles": int(res.threshold_used),
                      "latency_p10_p50_p90": [int(np.percentile(v, q)) for q in (10, 50, 90)],
                      "timer_overhead_median": int(np.median(ovhs)),
                      "best": {"C": best[0], "b": best[1], "a": best[2], "policy": ["LRU", "FIFO", "PLRU"][best[3]]}
                      if best else None,
                      "best_mismatch": int(res.best_m), "best_compared": int(res.best_n),
                      "zero_class": [list(r) for r in zc]}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("stream")
    p.add_argument("--bytes", type=int, default=1 << 30)
    p.add_argument("--dtype", type=int, default=1)
    p.add_argument("--grid", type=int, default=2048)
    p.add_argument("--block", type=int, default=256)
    p.add_argument("--ilp", type=int, default=4)
    p.add_argument("--reps", type=int, default=5)
    p.add_argument("--sweep", action="store_true")
    p = sub.add_parser("lds")
    p.add_argument("--reps", type=int, default=16)
    p = sub.add_parser("ldsbw")
    p.add_argument("--reps", type=int, default=2048)
    p = sub.add_parser("valu")
    p.add_argument("--reps", type=int, default=20000)
    p = sub.add_parser("curve")
    p.add_argument("--s", type=int, default=128)
    p.add_argument("--n-lo", type=int, default=4096)
    p.add_argument("--n-hi", type=int, default=131072)
    p.add_argument("--n-step", type=int, default=4096)
    p.add_argument("--flavor", type=int, default=0)
    p = sub.add_parser("l1")
    p.add_argument("--flavor", type=int, default=0)
    a = ap.parse_args(argv)
    {"stream": cmd_stream, "lds": cmd_lds, "ldsbw": cmd_ldsbw, "valu": cmd_valu, "curve": cmd_curve,
     "l1": cmd_l1}[a.cmd](a)


if __name__ == "__main__":
    main()
