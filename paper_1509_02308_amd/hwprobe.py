"""Hardware probes of one GPU through the C ABI: the paper's microbenchmarks
and the cache inference fed with real fine-grained P-chase latencies.

    python -m paper_1509_02308_amd.hwprobe stream [--bytes B] [--sweep]
    python -m paper_1509_02308_amd.hwprobe lds
    python -m paper_1509_02308_amd.hwprobe ldsbw
    python -m paper_1509_02308_amd.hwprobe valu
    python -m paper_1509_02308_amd.hwprobe l1 [--flavor 0] [--shifts]
    python -m paper_1509_02308_amd.hwprobe l2 [--flavor 1]
    python -m paper_1509_02308_amd.hwprobe curve --s 128 --n-lo 4096 --n-hi 131072
    python -m paper_1509_02308_amd.hwprobe grid [--flavors 0,1,2,3]
    python -m paper_1509_02308_amd.hwprobe tlb [--pages 65536,2097152]

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
  infer_cache_params (--shifts adds candidates whose set index comes from
  higher address bits, Section 4.3).
* l2: the same procedure on the L2 (system-scope loads, which miss the
  vector L1), one steady pass per run in compact records.
* grid: median and mean latency over array sizes 4 KB-512 MB x strides
  4 B-2 MB, powers of two, for every load flavour.
* tlb: the TLB sweep of Section 4.4 at page-scale strides, then the pages
  treated as cache lines and the TLB candidates replayed against it.

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


def _chase(torch, capi, N, s, passes, flavor, arr, compact=False):
    """`passes` timed passes after the preheat; compact: 16-bit records and
    no indices (four times the capacity)."""
    p = capi.PchaseProbe(N, s, 0, 0, 4, passes)
    L = capi.pchase_trace_len(capi.PchaseProbe(N, s, 0, 0, 4, 1))[0]
    k = passes * L
    lat = torch.zeros(k, dtype=torch.int32, device="cuda")
    idx = None if compact else torch.zeros(k, dtype=torch.int32, device="cuda")
    ovh = capi.microbench_pchase(p, flavor, arr, k, lat, idx)
    return lat, ovh, L


def _chase_steady(torch, capi, N, s, flavor, arr):
    """One timed pass after the preheat (compact records), laid out as the
    observation of a two-pass probe: the first pass, which the comparison
    skips, repeats the second."""
    lat, ovh, L = _chase(torch, capi, N, s, 1, flavor, arr, compact=True)
    return torch.cat([lat, lat]), ovh, L


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


def _pol_name(p):
    return ["LRU", "FIFO", "PLRU", "RANDOM"][p]


def _infer_runs(torch, capi, rows, flavor, arr, crows, threshold=None, steady=False):
    """Fine-grained runs of `rows` (N, s, passes) with one load flavour, the
    latencies classified (widest gap, or `threshold` cycles) and every
    candidate of `crows` replayed against them (Section 4.2).  steady: rows
    have 2 passes and only the second is timed (compact records)."""
    carr = capi.models(crows)
    parr = capi.probes(rows)
    lats, offs, ovhs = [], [0], []
    for N, s, passes in rows:
        if steady:
            lat, ovh, L = _chase_steady(torch, capi, N, s, flavor, arr)
        else:
            lat, ovh, L = _chase(torch, capi, N, s, passes, flavor, arr)
        ovhs.append(ovh)
        lats.append(lat)
        offs.append(offs[-1] + lat.numel())
    lat_all = torch.cat(lats)
    kw = {} if threshold is None else {"threshold": int(threshold)}
    res, zero = capi.infer_cache_params(parr, carr, lat=lat_all, lat_off=np.array(offs, np.uint64),
                                        probe_select=capi.PROBES_ALL, want_zero=True, **kw)
    v = lat_all.cpu().numpy().view(np.uint32)
    zc = [crows[i] for i in range(len(crows)) if (zero[i // 32] >> (i % 32)) & 1]
    best = crows[res.best] if res.best >= 0 else None
    return {"flavor": flavor, "probes": len(rows), "accesses": int(offs[-1]), "candidates": len(crows),
            "threshold_cycles": int(res.threshold_used),
            "latency_p10_p50_p90": [int(np.percentile(v, q)) for q in (10, 50, 90)],
            "timer_overhead_median": int(np.median(ovhs)),
            "best": {"C": best[0], "b": best[1], "a": best[2], "policy": _pol_name(best[3]),
                     "set_shift": best[4] if len(best) > 4 else 0} if best else None,
            "best_mismatch": int(res.best_m), "best_compared": int(res.best_n),
            "zero_class": [list(r) for r in zc]}


def _grid_rows(Cs, bs, As, pols, shifts=(0,)):
    rows = []
    for C in Cs:
        for b in bs:
            for a in As:
                if C % (a * b):
                    continue
                for sh in shifts:
                    if sh and (1 << sh) < b:
                        continue
                    for pol in pols:
                        rows.append((C, b, a, pol, sh))
    return rows


def cmd_l1(a):
    torch, capi = _torch_capi()
    # candidates for a per-CU vector L1 of 16-64 KB, modulo and shifted set mappings
    crows = _grid_rows((16384, 24576, 32768, 49152, 65536), (64, 128), (1, 2, 4, 8, 16, 32, 64), (0, 1, 2),
                       shifts=(0,) + tuple(range(8, 13)) if a.shifts else (0,))
    # fine-grained runs: N across [8 KB, 128 KB] in 1 KB steps, s in {64, 128, 256}
    rows = [(N, s, 2) for s in (64, 128, 256) for N in range(8192, 131072 + 1, 1024)
            if 2 * N // s <= capi.pchase_microbench_max_k()]
    arr = torch.zeros(131072 // 4 + 64, dtype=torch.int32, device="cuda")
    print(json.dumps({"probe": "l1_inference", **_infer_runs(torch, capi, rows, a.flavor, arr, crows)}), flush=True)


def cmd_l2(a):
    """The Section 4.2 procedure on the L2: system-scope loads (they miss the
    vector L1), N across the candidate capacities at line and two-line
    strides, one steady pass each in compact records."""
    torch, capi = _torch_capi()
    maxk = 4 * capi.pchase_microbench_max_k()
    MB = 1 << 20
    crows = _grid_rows((2 * MB, 4 * MB, 6 * MB, 8 * MB, 16 * MB), (64, 128), (8, 16, 32, 64), (0, 1, 2))
    rows = []
    for s, lo, hi, step in ((128, 2 * MB, 10 * MB, 128 * 1024), (256, 4 * MB, 20 * MB, 256 * 1024)):
        rows += [(N, s, 2) for N in range(lo, hi + 1, step) if N // s <= maxk]
    arr = torch.zeros(20 * MB // 4 + 64, dtype=torch.int32, device="cuda")
    print(json.dumps({"probe": "l2_inference", **_infer_runs(torch, capi, rows, a.flavor, arr, crows, steady=True)}),
          flush=True)


def cmd_grid(a):
    """Average and median latency over array sizes x strides (Section 4.1's
    curves, every load flavour): N and s powers of two, each point one
    steady pass (after the untimed preheat) of L = N / s accesses; points
    whose pass does not fit the LDS record store are not measurable with
    one lane's fine-grained records and are skipped."""
    torch, capi = _torch_capi()
    maxk = 4 * capi.pchase_microbench_max_k()   # compact records
    arr = torch.zeros(a.n_hi // 4 + 1024, dtype=torch.int32, device="cuda")
    lat = torch.zeros(maxk, dtype=torch.int32, device="cuda")
    idx = None
    for fl in (int(f) for f in a.flavors.split(",")):
        N = a.n_lo
        while N <= a.n_hi:
            s = a.s_lo
            while s <= min(a.s_hi, N // 2):
                L = N // s
                if L <= maxk:
                    ovh = capi.microbench_pchase(capi.PchaseProbe(N, s, 0, 0, 4, 1), fl, arr, L, lat, idx)
                    v = lat[:L].cpu().numpy().view(np.uint32).astype(np.int64) - ovh
                    print(json.dumps({"probe": "latency_grid", "flavor": fl, "N": N, "s": s, "L": L, "overhead": ovh,
                                      "mean": round(float(v.mean()), 1), "median": float(np.median(v)),
                                      "p10": int(np.percentile(v, 10)), "p90": int(np.percentile(v, 90))}),
                          flush=True)
                s *= 2
            N *= 2


def cmd_tlb(a):
    """TLB sweep (Section 4.4): strides of one page plus `pad` bytes, so that
    access k touches page k while the data lines spread over the cache sets;
    n = 1 .. max_pages pages, each run k = passes * n timed loads after the
    preheat.  Then the pages are treated as the lines of a cache (b = page)
    and the candidates replayed against the classified latencies."""
    torch, capi = _torch_capi()
    maxk = 4 * capi.pchase_microbench_max_k()   # compact records
    for pg, max_pages in zip((int(x) for x in a.pages.split(",")), (int(x) for x in a.max_pages.split(","))):
        s = pg + a.pad
        step = max(8, max_pages // 256)
        counts = sorted(set(list(range(1, 65)) + list(range(64, max_pages + 1, step)) + [max_pages]))
        arr = torch.zeros((max_pages * s) // 4 + 1024, dtype=torch.int32, device="cuda")
        rows, curve = [], []
        for n in counts:
            passes = max(2, min(maxk // n, 4096 // n))
            N = n * s
            lat, ovh, L = _chase(torch, capi, N, s, passes, a.flavor, arr, compact=True)
            v = lat.cpu().numpy().view(np.uint32).astype(np.int64)[n:] - ovh   # steady passes
            curve.append({"pages": n, "median": float(np.median(v)), "mean": round(float(v.mean()), 1),
                          "p90": int(np.percentile(v, 90))})
            print(json.dumps({"probe": "tlb_curve", "page": pg, "stride": s, "flavor": a.flavor, **curve[-1]}),
                  flush=True)
            rows.append((N, s, 2))
        entries = (8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
        crows = _grid_rows(tuple(e * pg for e in entries if e <= max_pages), (pg,), (1, 2, 4, 8, 16, 32, 64, 128),
                           (0, 1, 2))
        sel = [r for r in rows if r[0] // r[1] >= 8]
        out = _infer_runs(torch, capi, sel, a.flavor, arr, crows, threshold=a.threshold, steady=True)
        print(json.dumps({"probe": "tlb_inference", "page": pg, "stride": s, **out}), flush=True)


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
    p.add_argument("--shifts", action="store_true", help="add shifted set mappings to the candidates")
    p = sub.add_parser("l2")
    p.add_argument("--flavor", type=int, default=2)
    p = sub.add_parser("grid")
    p.add_argument("--flavors", default="0,1,2,3")
    p.add_argument("--n-lo", type=int, default=4096)
    p.add_argument("--n-hi", type=int, default=512 << 20)
    p.add_argument("--s-lo", type=int, default=4)
    p.add_argument("--s-hi", type=int, default=2 << 20)
    p = sub.add_parser("tlb")
    p.add_argument("--pages", default="65536,2097152")
    p.add_argument("--pad", type=int, default=128)
    p.add_argument("--max-pages", default="10240,3900", help="per page size")
    p.add_argument("--flavor", type=int, default=2)
    p.add_argument("--threshold", type=int, default=None, help="hit/miss threshold in cycles (default: widest gap)")
    a = ap.parse_args(argv)
    {"stream": cmd_stream, "lds": cmd_lds, "ldsbw": cmd_ldsbw, "valu": cmd_valu, "curve": cmd_curve,
     "l1": cmd_l1, "l2": cmd_l2, "grid": cmd_grid, "tlb": cmd_tlb}[a.cmd](a)


if __name__ == "__main__":
    main()
