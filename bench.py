"""Benchmark of the ED hot path on one MI355X.

Workload: the 4x4 Hubbard cluster (16 orbitals, t = -1 on the 24 open-boundary
bonds, U = 8, mu = U/2) in the half-filled sector N_up = N_dn = 8, dimension
165,636,900 (1.33 GB per FP64 vector).  One timed step is one product w = H v
through the C ABI (qcm_hv), with v the SplitMix64 start vector of seed 1,
already resident in HBM.  The value is the algorithmic bandwidth of the
product: 2 * s * d bytes (read v once, write w once; s = 8 in FP64) divided by
the time per product.

Printed: one JSON line with the metric, the roofline of the product against
the HBM peak, the CPU oracle timed on a bounded sample of rows, and the FP32-
vector product and a Lanczos step on the same sector.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·v GB/s (%HBM peak) at 16 sites; batched ED solves/s + p99 latency vs FP64"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--U", type=float, default=8.0)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extra", action="store_true", help="skip FP32-vector and Lanczos figures")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only copy one FP64 sector vector (d doubles) 10 times, for scaling "
                        "the FETCH_SIZE / WRITE_SIZE counters; prints its own line")
    p.add_argument("--cpu-rows", type=int, default=0,
                   help="rows of the sector the oracle computes for the CPU baseline "
                        "(0: every row, one full product)")
    return p.parse_args()


def time_calls(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sector product "
              "is not sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2305_18643_amd as q
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    q.load_library()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = synth.cluster_4x4(args.U)
    b = q.sector_basis(16, 8, 8)
    d = b.dim
    # start vector (SplitMix64, seed 1) generated on the device by the library's
    # own kernel: a 1-step fixed Lanczos run would normalise it, so instead fill
    # a uniform vector from torch and keep it resident; v's values do not change
    # the work of the product
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    v = torch.rand(d, dtype=torch.float64, device=dev, generator=g) * 2 - 1
    w = torch.empty_like(v)
    if args.copy_calibration:
        torch.cuda.synchronize()
        for _ in range(10):
            w.copy_(v)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 8 * d,
                                               "bytes_written_per_copy": 8 * d, "copies": 10}}))
        return
    ws = None
    # workspace once, reused by every call
    import ctypes
    from paper_2305_18643_amd import _binding as B
    hm = B.as_model(m)
    need = ctypes.c_size_t(0)
    lib = B.load_library()
    B._check(lib.qcm_hv(ctypes.byref(hm.c), ctypes.byref(b.c), 0, None, None, None, 0,
                        ctypes.byref(need), None))
    ws = torch.empty(need.value, dtype=torch.uint8, device=dev)

    def hv64():
        q.hv(hm, b, v, w, ws=ws)

    ms, wall = time_calls(torch, hv64, args.steps, args.warmup, stream)
    bytes_alg = 2 * 8 * d
    gbs = bytes_alg / (ms * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "4x4 Hubbard cluster, t=-1, U=%g, mu=U/2, sector (8,8), "
                               "d=165636900, one H.v per step" % args.U,
                   "sites": 16, "n_up": 8, "n_dn": 8, "dim": d, "prec": "fp64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "H.v (k_hv_inrow_team + k_hv_down_acc)",
                     "bytes_per_launch": bytes_alg},
    }

    if not args.no_extra:
        v32 = v.float()
        w32 = torch.empty_like(v32)

        def hv32():
            q.hv(hm, b, v32, w32, ws=ws)

        ms32, _ = time_calls(torch, hv32, max(3, args.steps // 2), 2, stream)
        gbs32 = 2 * 4 * d / (ms32 * 1e-3) / 1e9
        out["fp32v_hv"] = {"ms": round(ms32, 4), "GBps": round(gbs32, 2),
                           "frac_of_hbm_peak": round(gbs32 / HBM_PEAK_GBS, 4)}
        del v32, w32
        # a short fixed-step Lanczos run on the same sector (seconds per step)
        for prec in ("fp64", "fp32v"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = q.lanczos_gs(m, b, fixed_steps=10, want_vector=False, prec=prec,
                             reorth=1 if prec == "fp32v" else 0, check_every=10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out[f"lanczos_{prec}"] = {"steps": r["n_iter"], "s_per_step": round(dt / r["n_iter"], 5),
                                      "theta0_after_10": r["e0"]}

    if not args.no_cpu:
        import oracle
        nrows = d if args.cpu_rows <= 0 else min(args.cpu_rows, d)
        vh = oracle.start_vector(1, d)
        rows = np.arange(nrows, dtype=np.int64) * (d // nrows)
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        oracle.hv_rows(m.t, m.U, 8, 8, vh, rows, nthreads=threads)
        dt = time.perf_counter() - t0
        cpu_gbs = 2 * 8 * nrows / dt / 1e9
        out["cpu_baseline"] = {"value": round(cpu_gbs, 4), "unit": "GB/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{nrows} of {d} rows of the same sector (one full "
                                         f"product when equal), FP64, {dt:.1f} s; GB/s counts "
                                         f"16 bytes per row like the GPU figure"}
        del vh
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
