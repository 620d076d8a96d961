"""Benchmark: compress + decompress of a 513^3 FP32 |k|^-3 random field at a
relative L-inf bound of 1e-3 on one MI355X.

One step = one compress and one decompress of the whole field (every stage of
the path: range pass, per-level decomposition with quantisation, codebook,
encoding, decoding, per-level recomposition).  The input is resident in HBM
before timing starts.  ``value`` is the round-trip throughput
2 * input_bytes / step_time (each direction moves the uncompressed size).

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (per-launch algorithmic bytes over its HIP-event-timed duration) and a
CPU baseline (the FP64 oracle on a bounded sub-cube, one core).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "GB/s compress/decompress at rel L-inf 1e-3, % HBM peak; batched vs plain"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def stage_bytes(N: int, Nc: int, in_size: int, stream_bytes: int):
    """Algorithmic HBM bytes per launch of the finest-level / full-array stages.

    N points on the input grid, Nc on the next-coarser grid, in_size bytes per
    input value; symbols are 2 bytes; coarse grids are FP64.
    """
    new = N - Nc
    return {
        "range": in_size * N,
        "dec_level[finest]": in_size * N + 2 * new + 8 * Nc,
        "thomas[finest]": 2 * 8 * Nc,
        "histogram": 2 * N,
        "chunk_words": 2 * N,
        "encode": 2 * N + stream_bytes,
        "decode": stream_bytes + 2 * N,
        "rec_restrict[finest]": 2 * new + 8 * Nc,
        "rec_interp[finest]": 8 * Nc + 2 * new + in_size * N,
    }


def cpu_baseline(u: np.ndarray, rel: float, edge: int):
    """Time the FP64 oracle (compress + decompress) on a sub-cube, one thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    sub = np.ascontiguousarray(u[:edge, :edge, :edge])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        b = oracle.compress(sub, rel)
        t1 = time.perf_counter()
        oracle.decompress(b)
        t2 = time.perf_counter()
    return {"value": round(2 * sub.nbytes / (t2 - t0) / 1e9, 5), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d^3 FP32 sub-cube of the same field, compress %.1fs + decompress %.1fs"
                      % (edge, t1 - t0, t2 - t1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rel", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--cpu-edge", type=int, default=257)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(arrays are independent; see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_06322_amd as mgc
    import synthetic

    shape = (args.n, args.n, args.n)
    log("generating %s FP32 |k|^-3 field (seed 2)" % (shape,))
    u = synthetic.grf(shape, 2)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(u).to(dev)
    in_bytes = u.nbytes
    ws_c, out_c = mgc.compress_query(shape, torch.float32)
    ws = torch.empty(ws_c, dtype=torch.uint8, device=dev)
    out = torch.empty(out_c, dtype=torch.uint8, device=dev)
    blob = mgc.compress(x, args.rel, workspace=ws, out=out)
    info = mgc.header_info(blob)
    ws_d = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device=dev)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    log("warmup %d steps" % args.warmup)
    for _ in range(args.warmup):
        blob = mgc.compress(x, args.rel, workspace=ws, out=out)
        mgc.decompress(blob, workspace=ws_d, out=y, info=info)
    torch.cuda.synchronize()

    mgc.profile_enable(True)
    mgc.profile_reset()
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        blob = mgc.compress(x, args.rel, workspace=ws, out=out)
        ev[i][1].record(stream)
        mgc.decompress(blob, workspace=ws_d, out=y, info=info)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mgc.profile_read()
    mgc.profile_enable(False)
    c_ms = float(np.median([a.elapsed_time(b) for a, b, _ in ev]))
    d_ms = float(np.median([b.elapsed_time(c) for _, b, c in ev]))
    ms_step = wall * 1e3 / args.steps
    log("timed %d steps: %.3f ms/step (compress %.3f ms, decompress %.3f ms)"
        % (args.steps, ms_step, c_ms, d_ms))

    stream_bytes = int(blob.numel())
    yu = y.cpu().numpy().astype(np.float64)
    tau = args.rel * (float(u.max()) - float(u.min()))
    err = float(np.max(np.abs(yu - u)))
    N = u.size
    Nc = ((args.n + 1) // 2) ** 3
    sb = stage_bytes(N, Nc, 4, stream_bytes)
    stages = []
    for name, (cnt, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        per = ms / max(cnt, 1)
        row = {"stage": name, "launches": cnt, "ms_per_step": round(ms / args.steps, 4),
               "ms_per_launch": round(per, 4)}
        if name in sb:
            row["GBps"] = round(sb[name] / (per * 1e-3) / 1e9, 1)
        stages.append(row)
    for r in stages:
        log("  %-22s %4d launches  %8.4f ms/step  %s" % (r["stage"], r["launches"], r["ms_per_step"],
                                                       ("%.0f GB/s" % r["GBps"]) if "GBps" in r else ""))
    dom = next(r for r in stages if r["stage"] in sb)
    achieved = sb[dom["stage"]] / (dom["ms_per_launch"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom["stage"], "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                "traffic": None, "bytes_per_launch": int(sb[dom["stage"]])}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a %d^3 sub-cube" % args.cpu_edge)
        cpu = cpu_baseline(u, args.rel, args.cpu_edge)

    value = 2 * in_bytes / (ms_step * 1e-3) / 1e9
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grf%d_f32_linf_rel%g" % (args.n, args.rel),
                   "shape": list(shape), "input_dtype": "f32", "norm": "linf", "mode": "rel",
                   "bound": args.rel, "field": "Gaussian random field, power |k|^-3, seed 2",
                   "parallelism": "single GPU"},
        "compress_GBps": round(in_bytes / (c_ms * 1e-3) / 1e9, 2),
        "decompress_GBps": round(in_bytes / (d_ms * 1e-3) / 1e9, 2),
        "compress_ms": round(c_ms, 4), "decompress_ms": round(d_ms, 4),
        "compression_ratio": round(in_bytes / stream_bytes, 3),
        "max_err_over_tau": round(err / tau, 4),
        "roofline": roofline, "cpu_baseline": cpu, "stages": stages,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
