"""Benchmark of the ED hot path on one MI355X.

Workload: the 4x4 Hubbard cluster (16 orbitals, t = -1 on the 24 open-boundary
bonds, U = 8, mu = U/2) in the half-filled sector N_up = N_dn = 8, dimension
165,636,900 (1.33 GB per FP64 vector).  One timed step is one product w = H v
through the C ABI (qcm_hv_plan_apply on tables built once), with v a seeded
uniform vector already resident in HBM.  The value is the algorithmic bandwidth of the
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
    p.add_argument("--lanczos-steps", type=int, default=300, help="fixed Lanczos steps at 16 sites")
    p.add_argument("--no-cdmft", action="store_true", help="skip the CDMFT loop figures")
    p.add_argument("--no-vca", action="store_true", help="skip the VCA functional figures")
    p.add_argument("--no-sym", action="store_true",
                   help="skip the symmetry-adapted (C2v, A1) 4x4 sector figures")
    p.add_argument("--no-context", action="store_true",
                   help="skip the 14-site chain (the paper's timed workload)")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-solve figures")
    p.add_argument("--no-serve", action="store_true", help="skip the serving figures")
    p.add_argument("--batch-count", type=int, default=256, help="batched solves (seed 18643)")
    p.add_argument("--serve-count", type=int, default=110, help="serving requests per rate")
    p.add_argument("--serve-warmup", type=int, default=10,
                   help="first requests of each rate left out of the latency statistics")
    p.add_argument("--serve-rates", default="1,2,4",
                   help="arrival rates as multiples of the one-at-a-time FP64 rate")
    p.add_argument("--serve-budget-gib", type=float, default=64.0, help="engine pool (GiB)")
    return p.parse_args()


def measured_traffic(U: float, name="hv_4x4_fp64_hbm_traffic.txt",
                     sources=("hv.hip", "hv_split.hip"), key="traffic_bytes_per_hv"):
    """HBM bytes per product from a committed counter summary, or None when
    the product kernels changed since the counters were taken (source hash)
    or the workload differs from the one counted (U = 8)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if U != 8.0 or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2305_18643_amd", "csrc", f), "rb").read())
    if vals.get("source_sha256") != h.hexdigest() or key not in vals:
        return None
    return int(vals[key])


def cpu_info() -> dict:
    """CPU model, physical cores and logical CPUs of this host (lscpu)."""
    import subprocess
    info = {"logical_cpus": os.cpu_count()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return info
    kv = {}
    for line in txt.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    info["model"] = kv.get("Model name")
    try:
        info["physical_cores"] = int(kv["Core(s) per socket"]) * int(kv["Socket(s)"])
    except (KeyError, ValueError):
        pass
    return info


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
              "is not sharded across GPUs", file=sys.stderr)
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
    # a seeded uniform(-1, 1) vector, resident in HBM; its values do not
    # change the work of the product
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
    # the tables are built once (an H.v plan); each timed step is one product
    plan64 = q.HvPlan(m, b, "fp64")

    def hv64():
        plan64(v, w)

    ms, wall = time_calls(torch, hv64, args.steps, args.warmup, stream)
    bytes_alg = 2 * 8 * d
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    # a plain copy of one vector (read 8 d, write 8 d bytes): the bandwidth a
    # streaming kernel reaches on this GPU, beside the published peak
    ms_copy, _ = time_calls(torch, lambda: w.copy_(v), args.steps, args.warmup, stream)
    copy_gbs = bytes_alg / (ms_copy * 1e-3) / 1e9

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
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.U),
                     "kernel": "H.v (k_hv_inrow_tile + k_hv_down_acc)",
                     "bytes_per_launch": bytes_alg,
                     "copy_kernel_GBps": round(copy_gbs, 1),
                     "frac_of_copy_kernel": round(gbs / copy_gbs, 4)},
    }

    if not args.no_extra:
        v32 = v.float()
        w32 = torch.empty_like(v32)
        plan32 = q.HvPlan(m, b, "fp32v")

        def hv32():
            plan32(v32, w32)

        ms32, _ = time_calls(torch, hv32, max(3, args.steps // 2), 2, stream)
        gbs32 = 2 * 4 * d / (ms32 * 1e-3) / 1e9
        out["fp32v_hv"] = {"ms": round(ms32, 4), "GBps": round(gbs32, 2),
                           "frac_of_hbm_peak": round(gbs32 / HBM_PEAK_GBS, 4)}
        del v32, w32
        # 300-step Lanczos on the same sector, FP64 and FP32 vectors
        gold = os.path.join(ROOT, "tests", "golden", "cluster_4x4.json")
        e_ref = json.load(open(gold))["e0"] if (os.path.exists(gold) and args.U == 8.0) else None
        for prec in ("fp64", "fp32v"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = q.lanczos_gs(m, b, fixed_steps=args.lanczos_steps, want_vector=False, prec=prec,
                             reorth=1 if prec == "fp32v" else 0, check_every=args.lanczos_steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s_el = 8 if prec == "fp64" else 4
            rec = {"steps": r["n_iter"], "s_per_step": round(dt / r["n_iter"], 5),
                   "e0": r["e0"], "residual_est": r["residual_est"],
                   # algorithmic bytes per step: the product (read v, write w)
                   # and the recurrence's floor (read v_n, v_n-1, write v_n+1)
                   "GBps_algorithmic_5sd": round(5 * s_el * d / (dt / r["n_iter"]) / 1e9, 1)}
            if e_ref is not None:
                rec["e0_rel_err_vs_oracle_converged"] = abs(r["e0"] - e_ref) / abs(e_ref)
            out[f"lanczos_{prec}"] = rec

    if not args.no_context:
        out["context_chain14"] = context_section(args, torch, q, synth, np)
    if not args.no_cdmft:
        out["cdmft"] = cdmft_section(args, torch, q, synth, np)
    if not args.no_vca:
        out["vca"] = vca_section(args, torch, q, synth, np)
    if not args.no_sym:
        out["sym_4x4_a1"] = sym_section(args, torch, q, synth, np, stream)
    if not args.no_batch:
        out["batched"] = batched_section(args, torch, q, synth, np)
    if not args.no_serve:
        out["serving"] = serving_section(args, torch, q, synth, np)

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
        # one core, on every 32nd row
        rows1 = np.arange(d // 32, dtype=np.int64) * 32
        t1 = time.perf_counter()
        oracle.hv_rows(m.t, m.U, 8, 8, vh, rows1, nthreads=1)
        dt1 = time.perf_counter() - t1
        cpu = cpu_info()
        out["cpu_baseline"] = {"value": round(cpu_gbs, 4), "unit": "GB/s", "cores": threads,
                               "kind": "oracle", "cpu_model": cpu.get("model"),
                               "physical_cores": cpu.get("physical_cores"),
                               "logical_cpus": cpu.get("logical_cpus"),
                               "threads_used": threads,
                               "sample": f"{nrows} of {d} rows of the same sector (one full "
                                         f"product when equal), FP64, {dt:.1f} s; GB/s counts "
                                         f"16 bytes per row like the GPU figure",
                               "one_core": {"value": round(2 * 8 * len(rows1) / dt1 / 1e9, 4),
                                            "unit": "GB/s",
                                            "sample": f"every 32nd row ({len(rows1)} rows), "
                                                      f"{dt1:.1f} s"}}
        del vh
    print(json.dumps(out), flush=True)


Z_GRID = None


def _z(synth):
    global Z_GRID
    if Z_GRID is None:
        Z_GRID = synth.omega_grid()
    return Z_GRID


def solve_single_fp64(q, m, z, gf_steps, stream=None):
    """One request through the single-solve calls in plain FP64."""
    b = q.sector_basis(m.L, m.nup, m.ndn)
    r = q.lanczos_gs((m.t, m.U), b)
    g = q.green_cf((m.t, m.U), b, r["psi"], r["e0"], [0, 1, 2, 3], z, max_steps=gf_steps)
    return r["e0"], g["G"]


def floor_bytes(m, r, s_el):
    """Bytes of one solve at the Lanczos step's floor of 3 s d (read v_n and
    v_{n-1}, write v_{n+1}): the ground-state recurrence and its replay for
    the vector (2 n_iter steps on the ground-state sector), then every chain
    step on its own sector (electron chains add an up electron, hole chains
    remove one)."""
    from math import comb
    L, nu, nd = m.L, m.nup, m.ndn
    d_gs = comb(L, nu) * comb(L, nd)
    d_e = comb(L, nu + 1) * comb(L, nd) if nu < L else 0
    d_h = comb(L, nu - 1) * comb(L, nd) if nu > 0 else 0
    steps = 2 * int(r["n_iter"]) * d_gs
    if r.get("len") is not None:
        steps += int(r["len"][:, 0].sum()) * d_e + int(r["len"][:, 1].sum()) * d_h
    return 3 * s_el * steps


def engine_opts_for(prec):
    # residual test: the engine's automatic tolerance (1e-12 in FP64, 1e-7
    # with FP32 vectors, whose rounding floors the residual estimate)
    if prec == "fp64":
        return dict(prec="fp64", reorth=0)
    return dict(prec="fp32v", reorth=1)


MOMENT_FLOORS = 5


def _moments(b0sq, a, b2, kmax, np):
    """mu_k = b0^2 (T^k)_00, k = 0..kmax, T the tridiagonal matrix of the
    floors given (exact for k <= 2 len(a) - 1)."""
    K = len(a)
    T = np.diag(np.asarray(a, dtype=float))
    if K > 1:
        off = np.sqrt(np.maximum(np.asarray(b2, dtype=float), 0.0))
        T += np.diag(off, 1) + np.diag(off, -1)
    e = np.zeros(K)
    e[0] = 1.0
    out = []
    x = e.copy()
    for _ in range(kmax + 1):
        out.append(b0sq * x[0])
        x = T @ x
    return np.array(out)


def oracle_accuracy(models, results_by_prec, idx, z, np, gf_steps=100):
    """Per-result errors of GPU solves against the CPU FP64 oracle (plain
    recurrence, the same start vector): relative |dE0|, max |dG| over the 4x4
    block on the grid, max |d b0^2| of the 20 chains, the degeneracy flag and
    whether every chain of the oracle ended by exhausting its Krylov space
    (only then is the 100-floor G independent of rounding; truncated chains
    without reorthogonalisation differ run to run, in either precision).
    Also the well-conditioned part of every chain: the spectral moments
    mu_k = <phi| H^k |phi> = b0^2 (T^k)_00, k <= 8, which its first five floors
    fix exactly (T their tridiagonal matrix), relative to b0^2 S^k with S the
    largest |a_n| or b_n of those floors.  The coefficients themselves are
    not: where a chain starts in a cluster of close eigenvalues they amplify a
    start-vector change about tenfold per floor (FP32 storage, 1e-7, moves a_4
    by 2e-4 on a 7-orbital request; the FP64 chains agree with the oracle to
    1e-9 through floor 11 on the 3x4 cluster)."""
    import oracle
    from oracle import cf
    recs = []
    for i in idx:
        m = models[i]
        d = oracle.binom(m.L, m.nup) * oracle.binom(m.L, m.ndn)
        th = 1 if d <= 100000 else oracle.default_threads()
        ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True, nthreads=th)
        ch = oracle.green_cf(m.t, m.U, m.nup, m.ndn, ro["psi"], [0, 1, 2, 3], max_steps=gf_steps,
                             nthreads=th)
        Go = cf.green_matrix(ch, 4, z, ro["e0"])
        exhausted = all(len(a) < gf_steps for (_, a, _) in ch.values())
        rec = {"job": int(i), "orbitals": m.L, "dim": int(d), "oracle_chains_exhausted": exhausted}
        keys = [(a, b, part) for a in range(4) for b in range(a, 4) for part in (0, 1)]
        for prec, res in results_by_prec.items():
            r = res[i]
            b0 = [r["coef"][p, part, 0] for p in range(10) for part in (0, 1)]
            b0o = [ch[k][0] for k in keys]
            # spectral moments from the first floors of each chain, both sides
            dmom = 0.0
            for n, k in enumerate(keys):
                p, part = n // 2, n % 2
                bo, ao, b2o = ch[k]
                K = min(MOMENT_FLOORS, int(r["len"][p, part]), len(ao))
                if K == 0 or bo == 0.0:
                    continue
                mg = _moments(r["coef"][p, part, 0], r["coef"][p, part, 1:1 + K],
                              r["coef"][p, part, 1 + gf_steps:gf_steps + K], 2 * K - 2, np)
                mo = _moments(bo, ao[:K], b2o[:K - 1], 2 * K - 2, np)
                S = max(1.0, float(np.abs(ao[:K]).max()), float(np.sqrt(np.max(b2o[:K - 1]))) if K > 1 else 0.0)
                scale = bo * S ** np.arange(mo.shape[0])
                dmom = max(dmom, float(np.max(np.abs(mg - mo) / scale)))
            rec[prec] = {"rel_dE0": abs(r["e0"] - ro["e0"]) / abs(ro["e0"]),
                         "max_dG": float(np.abs(r["G"] - Go).max()),
                         "max_db0sq": float(np.max(np.abs(np.array(b0) - np.array(b0o)))),
                         "max_rel_dmoment": dmom,
                         "degenerate_suspect": bool(r["degenerate_suspect"])}
        recs.append(rec)
    summ = {}
    for prec in results_by_prec:
        for key, sel in (("all", recs), ("exhausted", [r for r in recs if r["oracle_chains_exhausted"]]),
                         ("truncated", [r for r in recs if not r["oracle_chains_exhausted"]])):
            if not sel:
                continue
            summ[f"{prec}_{key}"] = {
                "jobs": len(sel),
                "max_rel_dE0": max(r[prec]["rel_dE0"] for r in sel),
                "max_dG": max(r[prec]["max_dG"] for r in sel),
                "median_dG": float(np.median([r[prec]["max_dG"] for r in sel])),
                "max_db0sq": max(r[prec]["max_db0sq"] for r in sel),
                "max_rel_dmoment_k8": max(r[prec]["max_rel_dmoment"] for r in sel),
                "degenerate_suspect_jobs": sum(r[prec]["degenerate_suspect"] for r in sel)}
    return summ, recs


def context_section(args, torch, q, synth, np):
    """The paper's timed workload (Table performance): the 14-site open chain,
    t = -1, U = 4, mu = 2, at half filling.  Here the full (7,7) sector
    (11,778,624 states; the paper used the 5,889,312-state reflection-even
    half), FP64: ground state to the residual test, then the 14 x 14 up-spin
    G from 200-floor continued fractions and by band Lanczos (the paper's
    method); and the ground state in the paper's own sector, the
    reflection-even half, through the stored (packed) matrix."""
    m = synth.chain(14, U=4.0, mu=2.0, nup=7, ndn=7)
    z = _z(synth)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = q.sector_basis(14, 7, 7)
    r = q.lanczos_gs((m.t, m.U), b)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t0
    gcf = q.green_cf((m.t, m.U), b, r["psi"], r["e0"], list(range(14)), z, max_steps=200)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    # the paper's method for G: band Lanczos over the 14 start states, stopped
    # by the convergence of the lowest eigenvalue of T (1e-10)
    t1 = time.perf_counter()
    gb = q.green_band((m.t, m.U), b, r["psi"], r["e0"], list(range(14)), z, max_basis=1000,
                      etol=1e-10)
    torch.cuda.synchronize()
    t_band = time.perf_counter() - t1
    gb_R = [int(x) for x in gb["R"]]
    gs_steps = r["n_iter"]
    dg = float((gb["G"] - gcf["G"]).abs().max().item())
    e0_full = r["e0"]
    del gcf, gb, r, b
    torch.cuda.empty_cache()
    # the paper's own sector: the reflection-even half (irrep A of the
    # chain's mirror; with 7 particles per spin no state is its own mirror
    # image, so A holds exactly half the states), stored matrix built on the
    # GPU and packed, then the ground state
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bs = q.sector_basis(14, 7, 7)
    sec = q.sym_sector(bs, synth.c2_chain(14), synth.C2_IRREPS["A"])
    Hs = q.sym_hamiltonian((m.t, m.U), sec)
    Hs.pack()
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t2
    t3 = time.perf_counter()
    rs = q.sym_lanczos_gs(Hs, want_vector=True)
    torch.cuda.synchronize()
    t_gs_a = time.perf_counter() - t3
    sym = {"sector_dim": sec.dim, "nnz": Hs.nnz, "values": Hs.n_values,
           "build_s": round(t_build, 3), "gs_s": round(t_gs_a, 3), "gs_steps": rs["n_iter"],
           "e0": rs["e0"], "e0_minus_full_sector": rs["e0"] - e0_full,
           "true_residual": rs["true_residual"]}
    del Hs, sec, bs
    torch.cuda.empty_cache()
    print(f"context chain14: GS {t_gs:.2f} s, GS + G {t_all:.2f} s, band G {t_band:.2f} s "
          f"(R {list(gb_R)}); reflection-even sector (dim {sym['sector_dim']}): build "
          f"{t_build:.2f} s, GS {t_gs_a:.2f} s, E0 - full {sym['e0_minus_full_sector']:.1e}",
          file=sys.stderr, flush=True)
    return {"workload": "14-site chain t=-1 U=4 mu=2, sector (7,7) d=11778624, FP64; GS to "
                        "tol 1e-12, then 14x14 G (105 pairs x 2 chains x 200 floors), and the "
                        "14x14 G by band Lanczos (lowest Ritz value converged to 1e-10)",
            "gs_s": round(t_gs, 3), "gs_steps": gs_steps, "e0": e0_full,
            "gs_plus_g_s": round(t_all, 3),
            "band_g_s": round(t_band, 3), "band_R": gb_R,
            "gs_plus_band_g_s": round(t_gs + t_band, 3),
            "max_abs_G_band_minus_cf": dg,
            "reflection_even_sector": sym,
            "paper": {"hardware": "Apple M2 Max, 8 OpenMP threads", "sector_dim": 5889312,
                      "lanczos_s": 26.8, "gs_plus_gf_s": 86.0, "gf_method": "band Lanczos"}}


def cdmft_section(args, torch, q, synth, np):
    """The CDMFT loop of the paper's 1D example: Hubbard chain U = 4, mu = 2,
    4-site clusters with 4 bath orbitals (parameters eb1, eb2, tb1, tb2 from
    (1, -1, 1, 1)), sector (4,4) of the 8-orbital impurity, 64 wave-vectors,
    Matsubara grid beta = 50 up to omega = 2, uniform weights, stopped when
    no parameter moves by more than 1e-6.  One iteration of the CPU oracle is
    timed beside it (context)."""
    s = synth.cdmft_chain_4_4b()
    z = synth.matsubara_grid(s.beta, s.wc)
    w = np.full(z.shape[0], 1.0 / z.shape[0])
    ks = synth.k_grid_1d(64)
    q.cdmft(s, s.p0, ks, z, w, max_iter=1)          # warm-up (library and kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = q.cdmft(s, s.p0, ks, z, w, max_iter=40, tol=1e-6)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": "1D Hubbard U=4 mu=2, 4-site clusters + 4 bath orbitals, impurity sector "
                       "(4,4) d=4900, 64 k, beta=50, wc=2 (16 frequencies), tol 1e-6",
           "iterations": r["iterations"], "converged": bool(r["converged"]),
           "loop_s": round(dt, 4), "s_per_iteration": round(dt / r["iterations"], 5),
           "bath": [float(x) for x in r["p"]], "distance": r["distance"]}
    msg = f"cdmft: {r['iterations']} iterations in {dt:.2f} s"
    if not args.no_cpu:
        # CPU baseline: one iteration of the oracle (its Lanczos and continued
        # fractions on one thread, then NumPy / SciPy)
        from oracle import cdmft as C
        t1 = time.perf_counter()
        Gc, _ = C.cluster_green(s, s.p0, z)
        sig = C.sigma(s, s.p0, z, Gc)
        G0i = C.g0inv(C.gbar(s, z, sig, ks), sig)
        C.fit(s, s.p0, z, w, G0i)
        t_cpu = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(t_cpu, 3), "unit": "s per iteration", "cores": 1,
                               "kind": "oracle", "sample": "one CDMFT iteration from p0"}
        msg += f"; one oracle iteration {t_cpu:.2f} s"
    print(msg, file=sys.stderr, flush=True)
    return out


def vca_section(args, torch, q, synth, np):
    """The Potthoff functional of the 2x2 plaquette reference system for the
    square-lattice Hubbard model (U = 8, mu = 4, half filling), scanned over
    the reference hopping t' (9 values in [-1.4, -0.6]) on a 32 x 32 grid of
    the reduced zone: per value a GPU ground state, a GPU band Lanczos to
    exhaustion and the GPU pole formula.  The CPU oracle's pole formula for
    one value is timed beside it."""
    tps = np.linspace(-1.4, -0.6, 9)
    ks = synth.k_grid_2d(32)
    q.vca.omega(synth.vca_plaquette(tp=-1.0), ks)        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om = [q.vca.omega(synth.vca_plaquette(tp=tp), ks) for tp in tps]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    i = int(np.argmin(om))
    stat = None
    if 0 < i < len(tps) - 1:       # vertex of the parabola through the three points
        a, b, c = np.polyfit(tps[i - 1:i + 2], om[i - 1:i + 2], 2)
        stat = float(-b / (2 * a))
    # the same scan by the adaptive frequency integral (eq. (sef4))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    omq = [q.vca.omega(synth.vca_plaquette(tp=tp), ks, method="quad") for tp in tps]
    torch.cuda.synchronize()
    dtq = time.perf_counter() - t0
    out = {"workload": "2x2 plaquette reference, square lattice t=-1 U=8 mu=4 (2,2); 32x32 k; "
                       "t' scan of 9 values in [-1.4, -0.6]",
           "s_per_evaluation": round(dt / len(tps), 4), "omega": [float(x) for x in om],
           "tp": [float(x) for x in tps], "tp_stationary": stat,
           "quad": {"s_per_evaluation": round(dtq / len(tps), 4),
                    "max_abs_diff_vs_pole_formula": float(np.max(np.abs(np.array(omq) - om)))}}
    msg = (f"vca: {len(tps)} evaluations in {dt:.2f} s (quadrature {dtq:.2f} s, max diff "
           f"{out['quad']['max_abs_diff_vs_pole_formula']:.1e}), stationary t' ~ {stat}")
    if not args.no_cpu:
        from oracle import vca as O
        s = synth.vca_plaquette(tp=-1.0)
        t1 = time.perf_counter()
        e0, poles, Q = O.cluster_lehmann(s.t_ref, s.U, s.nup, s.ndn)
        O.omega_poles(e0, poles, Q, s.dt, s.bonds, ks)
        t_cpu = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(t_cpu, 3), "unit": "s per evaluation", "cores": 1,
                               "kind": "oracle", "sample": "one functional value (t' = -1)"}
        msg += f"; one oracle evaluation {t_cpu:.2f} s"
    print(msg, file=sys.stderr, flush=True)
    return out


def sym_section(args, torch, q, synth, np, stream):
    """The 4x4 cluster's A1 sector of C2v (the rectangle's rotation by pi
    and its two mirrors; U as the main figure, mu = U/2, (8,8)): the stored
    matrix is built on the GPU, then timed: the product w = H v over the
    stored rows (HBM roofline: the matrix streamed once, 12 bytes per
    element, the row pointers, v read and w written once) and fixed-step
    Lanczos.  The oracle's one-column routine is timed on a sample of
    columns beside it."""
    m = synth.cluster_4x4(args.U)
    perms, chi = synth.c2v_rectangle(4, 4), synth.C2V_IRREPS["A1"]
    b = q.sector_basis(16, 8, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sec = q.sym_sector(b, perms, chi)
    H = q.sym_hamiltonian(m, sec)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    n, nnz = sec.dim, H.nnz
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    v = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    w = torch.empty_like(v)
    ms, _ = time_calls(torch, lambda: H(v, w), args.steps, args.warmup, stream)
    bytes_alg = 12 * nnz + 8 * (n + 1) + 16 * n
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    steps = args.lanczos_steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = q.sym_lanczos_gs(H, fixed_steps=steps, want_vector=False, check_every=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    # the packed form: one index per distinct value (4 bytes per element)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    nvals = H.pack()
    torch.cuda.synchronize()
    t_pack = time.perf_counter() - t3
    packed = None
    if nvals:
        ms_p, _ = time_calls(torch, lambda: H(v, w), args.steps, args.warmup, stream)
        bytes_p = 4 * nnz + 8 * (n + 1) + 16 * n
        gbs_p = bytes_p / (ms_p * 1e-3) / 1e9
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rp = q.sym_lanczos_gs(H, fixed_steps=steps, want_vector=False, check_every=steps)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t1
        packed = {"values": nvals, "pack_s": round(t_pack, 3), "ms": round(ms_p, 4),
                  "GBps": round(gbs_p, 2), "frac_of_hbm_peak": round(gbs_p / HBM_PEAK_GBS, 4),
                  "bytes_per_launch": bytes_p, "kernel": "k_sym_spmv_pk",
                  "traffic": measured_traffic(args.U, "sym_4x4_a1_hbm_traffic.txt", ("sym.hip",),
                                              "traffic_bytes_per_hv_packed"),
                  "lanczos_s_per_step": round(dtp / rp["n_iter"], 5),
                  "e0_rel_diff_vs_explicit": abs(rp["e0"] - r["e0"]) / abs(r["e0"])}
    del v, w
    gold = os.path.join(ROOT, "tests", "golden", "cluster_4x4.json")
    e_ref = json.load(open(gold))["e0"] if (os.path.exists(gold) and args.U == 8.0) else None
    out = {"workload": f"4x4 Hubbard cluster t=-1 U={args.U:g} mu=U/2 (8,8), C2v irrep A1",
           "dim": n, "nnz": nnz, "build_s": round(t_build, 3),
           "hv": {"ms": round(ms, 4), "GBps": round(gbs, 2),
                  "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": bytes_alg,
                  "kernel": "k_sym_spmv",
                  "traffic": measured_traffic(args.U, "sym_4x4_a1_hbm_traffic.txt", ("sym.hip",))},
           "lanczos": {"steps": r["n_iter"], "s_per_step": round(dt / r["n_iter"], 5),
                       "e0": r["e0"]},
           "packed": packed}
    if e_ref is not None:
        out["lanczos"]["e0_rel_diff_vs_full_sector_oracle"] = abs(r["e0"] - e_ref) / abs(e_ref)
    msg = (f"sym 4x4 A1: dim {n}, nnz {nnz}, build {t_build:.2f} s, H.v {ms:.3f} ms "
           f"({gbs:.0f} GB/s), Lanczos {dt / r['n_iter'] * 1e3:.2f} ms/step, E0 {r['e0']:.12f}")
    if packed:
        msg += (f"; packed ({nvals} values, {t_pack:.2f} s): H.v {packed['ms']:.3f} ms "
                f"({packed['GBps']:.0f} GB/s), Lanczos {packed['lanczos_s_per_step'] * 1e3:.2f} ms/step")
    if not args.no_cpu:
        from math import comb
        from oracle import sym as S
        Su = S.strings(16, 8)
        rep = H.rep[:n]
        # exact int64 positions 0 .. n-1, made on the host
        idx = torch.from_numpy(np.arange(200, dtype=np.int64) * (n - 1) // 199).to("cuda")
        labs = (rep[idx].cpu().numpy().astype(np.int64) & 0xFFFFFFFF).tolist()
        d_up = comb(16, 8)
        t2 = time.perf_counter()
        for lab in labs:
            S.sym_column(m.t, m.U, int(Su[lab % d_up]), int(Su[lab // d_up]), perms, chi)
        per = (time.perf_counter() - t2) / len(labs)
        out["cpu_baseline"] = {"value": round(per * n, 1), "unit": "s per stored matrix",
                               "cores": 1, "kind": "oracle",
                               "sample": f"the one-column routine on 200 of {n} columns "
                                         f"({per * 1e3:.2f} ms each), scaled to all columns"}
        msg += f"; oracle {per * 1e3:.2f} ms per column ({per * n:.0f} s for the matrix)"
    print(msg, file=sys.stderr, flush=True)
    del H, sec
    torch.cuda.empty_cache()
    return out


def batched_section(args, torch, q, synth, np):
    """256 impurity solves (4-site cluster + 2..10 bath orbitals, seed 18643):
    ground state to convergence plus the 4x4 cluster G with 100-floor chains
    on the 64-point grid.  Engine in FP32V and FP64 with every solve in flight
    at once, against the same solves run one at a time through the
    single-solve calls in FP64."""
    z = _z(synth)
    ms = synth.batched_solves(18643, args.batch_count)
    out = {"workload": f"{len(ms)} impurity solves, seed 18643, n = 6..14 orbitals, GS + 4x4 G "
                       "(M_G = 100, 64 frequencies)"}
    res = {}
    for prec in ("fp32v", "fp64"):
        specs = [q.JobSpec((m.t, m.U), m.nup, m.ndn, orbs=range(4), tag=i) for i, m in enumerate(ms)]
        kw = dict(gf_steps=100, z=z, max_jobs=len(ms), **engine_opts_for(prec))
        need = q.batch_bytes(specs, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rr = q.batch_solve(specs, ws_bytes=need, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = rr
        fb = sum(floor_bytes(m, r, 4 if prec == "fp32v" else 8) for m, r in zip(ms, rr))
        out[f"engine_{prec}"] = {"s": round(dt, 3), "solves_per_s": round(len(ms) / dt, 2),
                                 "pool_GB": round(need / 1e9, 2),
                                 "gs_steps_mean": round(float(np.mean([r["n_iter"] for r in rr])), 1),
                                 "floor_GB": round(fb / 1e9, 1),
                                 "GBps_floor": round(fb / dt / 1e9, 1)}
        print(f"batched engine {prec}: {dt:.2f} s", file=sys.stderr, flush=True)
    # accuracy of FP32V against the FP64 engine
    e64 = np.array([r["e0"] for r in res["fp64"]])
    e32 = np.array([r["e0"] for r in res["fp32v"]])
    dG = max(float(np.abs(a["G"] - b["G"]).max()) for a, b in zip(res["fp32v"], res["fp64"]))
    out["fp32v_vs_fp64"] = {"max_rel_dE0": float(np.max(np.abs(e32 - e64) / np.abs(e64))),
                            "max_abs_dG": dG}
    # accuracy of both engines against the CPU oracle, per result: every job of
    # 8 orbitals or fewer, and a stated sample of the larger ones
    if not args.no_cpu:
        small = [i for i, m in enumerate(ms) if m.L <= 8]
        sample = []
        for L in (9, 10, 11):
            sample += [i for i, m in enumerate(ms) if m.L == L][:2]
        t0 = time.perf_counter()
        summ, recs = oracle_accuracy(ms, res, small + sample, z, np)
        out["vs_oracle"] = {"jobs": f"all {len(small)} jobs with <= 8 orbitals and the first two "
                                    f"of 9, 10 and 11 orbitals ({len(sample)})",
                            "summary": summ, "per_job": recs,
                            "oracle_s": round(time.perf_counter() - t0, 1)}
        print(f"batched accuracy vs oracle: {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    # baseline: the same solves one at a time, FP64 single-solve calls
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    base = []
    for i, m in enumerate(ms):
        base.append(solve_single_fp64(q, m, z, 100))
        if (i + 1) % 32 == 0:
            print(f"  one-at-a-time fp64: {i + 1} solves, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the single calls take the FP64 engine's steps (equal bit for bit, below)
    fb = sum(floor_bytes(m, r, 8) for m, r in zip(ms, res["fp64"]))
    out["one_at_a_time_fp64"] = {"s": round(dt, 3), "solves_per_s": round(len(ms) / dt, 2),
                                 "GBps_floor": round(fb / dt / 1e9, 1)}
    out["floor_bytes"] = ("3 s d per Lanczos step (read v_n, v_{n-1}, write v_{n+1}) over the "
                          "ground-state recurrence and its replay and every chain step, summed "
                          "over the solves and divided by the wall time")
    out["speedup_fp32v_engine"] = round(dt / out["engine_fp32v"]["s"], 2)
    out["speedup_fp64_engine"] = round(dt / out["engine_fp64"]["s"], 2)
    # the FP64 engine equals the single-solve calls bit for bit
    out["fp64_engine_equals_single_calls"] = bool(all(
        r["e0"] == e0 and np.array_equal(r["G"], G.cpu().numpy())
        for r, (e0, G) in zip(res["fp64"], base)))
    print(f"batched one-at-a-time fp64: {dt:.2f} s", file=sys.stderr, flush=True)
    return out


def serving_section(args, torch, q, synth, np):
    """Poisson streams of serving requests (seed 2305: 4..14-orbital chains
    and ladders, GS + 4x4 G, M_G = 100) at multiples of the one-at-a-time
    FP64 rate R1, through the continuously batched FP32V engine with a pool
    budget; the baseline is the FIFO one-at-a-time FP64 queue on the same
    arrivals, from each request's measured service time."""
    from paper_2305_18643_amd import serving
    z = _z(synth)
    n = args.serve_count
    reqs = synth.serving_requests(2305, n)
    # service time of each request alone, FP64 single-solve calls
    svc = []
    solve_single_fp64(q, reqs[0], z, 100)   # warm-up
    for i, m in enumerate(reqs):
        if i % 20 == 0:
            print(f"  serving baseline: request {i}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve_single_fp64(q, m, z, 100)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t0)
    svc = np.array(svc)
    r1 = n / svc.sum()
    out = {"workload": f"{n} requests per rate, seed 2305, n = 4..14 orbitals, GS + 4x4 G "
                       "(M_G = 100), Poisson arrivals",
           "R1_fp64_one_at_a_time_solves_per_s": round(r1, 3),
           "budget_GiB": args.serve_budget_gib, "rates": []}
    budget = int(args.serve_budget_gib * (1 << 30))
    eng = q.Engine(budget, gf_steps=100, z=z, max_jobs=256, **engine_opts_for("fp32v"))
    for k, mult in enumerate(float(x) for x in args.serve_rates.split(",")):
        lam = mult * r1
        arr = serving.poisson_arrivals(lam, n, seed=2305 + k)
        specs = [q.JobSpec((m.t, m.U), m.nup, m.ndn, orbs=range(4), tag=i)
                 for i, m in enumerate(reqs)]
        rep = serving.serve(eng, specs, arr, progress=lambda c: print(
            f"  serving x{mult}: {c} of {n} done", file=sys.stderr, flush=True))
        base = serving.fifo_one_at_a_time(svc, arr)
        if k == 0 and not args.no_cpu:
            # per-result accuracy of the served (FP32V) solves against the CPU
            # oracle, on a 50-request sample: the first 50 requests whose sector
            # has at most 100,000 states
            import oracle as _o
            samp = [i for i, m in enumerate(reqs)
                    if _o.binom(m.L, m.nup) * _o.binom(m.L, m.ndn) <= 100000][:50]
            summ, recs = oracle_accuracy(reqs, {"fp32v": rep.results}, samp, z, np)
            out["vs_oracle"] = {"sample": f"the first {len(samp)} requests with at most 100,000 "
                                          "states, at the first rate", "summary": summ,
                                "per_request": recs}
        warm = min(max(args.serve_warmup, 0), n - 1)
        meas = [t for t in range(warm, n)]
        lat = np.array([rep.latency[t] for t in meas])
        done_at = max(arr[t] + rep.latency[t] for t in meas)
        bl = np.asarray(base)[warm:]
        out["rates"].append({
            "x_R1": mult, "rate_per_s": round(lam, 3), "measured_requests": len(meas),
            "warmup_requests": warm,
            "engine_fp32v": {"p50_s": round(serving.nearest_rank(lat, 50), 4),
                             "p99_s": round(serving.nearest_rank(lat, 99), 4),
                             "solves_per_s": round(len(meas) / (done_at - arr[warm]), 3),
                             "GBps_floor": round(sum(floor_bytes(reqs[t], rep.results[t], 4)
                                                     for t in meas) / (done_at - arr[warm]) / 1e9, 1),
                             "max_in_flight": rep.max_in_flight},
            "fifo_fp64": {"p50_s": round(serving.nearest_rank(bl, 50), 4),
                          "p99_s": round(serving.nearest_rank(bl, 99), 4),
                          "solves_per_s": round(len(meas) / (arr[-1] + base[-1] - arr[warm]), 3)}})
        print(f"serving x{mult}: p99 {serving.nearest_rank(lat, 99):.3f} s", file=sys.stderr,
              flush=True)
    out["peak_pool_GB"] = round(eng.info()["peak_in_use"] / 1e9, 3)
    torch.cuda.empty_cache()   # blocks cached by earlier sections are not the engine's
    free, total = torch.cuda.mem_get_info()
    out["device_memory_in_use_GB"] = round((total - free) / 1e9, 3)
    out["device_memory_GB"] = round(total / 1e9, 3)
    eng.close()
    return out


if __name__ == "__main__":
    main()
