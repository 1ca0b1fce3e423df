#!/usr/bin/env python3
"""Benchmark of the plane-wave H.psi / block-Davidson hot path on one MI355X.

Default workload (cell512): the largest served cell -- cubic a = 41 bohr,
Gamma, ecutwfc 30 Ry (191,471 plane waves), FFT grid 144^3, 512 atoms with
2048 s/p projectors, 1024 bands.  A step is one mixed-precision hpsi_apply of
the 1024-band block (float32 transforms and projector products with float32
accumulation; complex128 in and out); value = band-H.psi/s.  The same
product in plain float64 on the same GPU is the metric's baseline
(vs_baseline = mixed / float64).  Beside it: the 64-atom cell's Davidson
solves (float64 and mixed, solves/s and the largest eigenvalue error against
the dense oracle's golden values), the live roofline of the dominant kernel,
and the CPU baselines (dense oracle rows, and the CPU FFT method), whose
sampled rows also give the GPU products' parity on this cell.

Other workloads: cell64 (a step is one Davidson solve of the 64-atom cell),
batch (32 cells x 4 k-points), serve (Poisson request trace, p50/p99),
solve512 (a step is one Davidson solve of the 512-atom cell).
Inputs are synthetic and resident in HBM before timing starts.
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

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TF = 78.6     # MFMA and vector
FP32_MFMA_PEAK_TF = 157.3

HBM_KERNELS = {"k_zinv", "k_plane", "k_zfwd", "calbec_reduce_dapply", "zgemm_cn_reduce", "vector_ops"}
MFMA_KERNELS = {"calbec_gemm", "add_nl_gemm", "zgemm_cn", "zgemm_nn"}
ALU_KERNELS = {"k_chol", "k_trinv", "k_tridiag", "k_backtr", "k_bisect", "k_invit"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20 for cell512, 3 otherwise)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 3 for cell512, 1 otherwise)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="default: fp64 for the cell64 solves, mixed for batch and serve")
    ap.add_argument("--ndim", type=int, default=None,
                    help="Davidson basis cap (x nb); default: 3 for the float64 cell solve, 2 otherwise "
                         "(the fastest settings measured for the bench cell)")
    ap.add_argument("--hpsi-reps", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gamma", action="store_true", help="cell512: skip the Gamma-point path rates")
    ap.add_argument("--no-stages", action="store_true",
                    help="skip the per-stage H.psi measurement (keeps kernel profiles to the timed steps)")
    ap.add_argument("--workload", choices=["cell512", "cell64", "batch", "serve", "solve512"], default="cell512",
                    help="cell512: mixed H.psi of the 512-atom 144^3 cell vs plain float64 (default line); "
                         "cell64: Davidson solves of the 64-atom cell; batch: 32 cells x 4 k-points solved "
                         "concurrently vs one at a time in FP64; serve: Poisson request trace through the "
                         "serving loop (p50/p99 latency); solve512: Davidson solves of the 512-atom cell "
                         "(mixed: and one float64 solve beside it)")
    ap.add_argument("--nbands", type=int, default=1024, help="cell512: bands of the H.psi block")
    ap.add_argument("--solves", type=int, default=3,
                    help="cell512: Davidson solves of the 64-atom cell per precision (0: skip)")
    ap.add_argument("--workers", type=int, default=None,
                    help="batch/serve: concurrent solves (default 12 for batch, 8 for serve)")
    ap.add_argument("--requests", type=int, default=32, help="serve: requests per trace")
    ap.add_argument("--max-atoms", type=int, default=512, help="serve: largest request (atoms)")
    ap.add_argument("--ecut", type=float, default=30.0, help="serve: cutoff in Ry")
    ap.add_argument("--plane-mode", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="cell512: plane pass form (plan option plane_mode: 0 auto, 1 three kernels, "
                         "2 the 16-lane-group kernel wherever it applies, 3 measured at plan creation, "
                         "4 the register (quad) kernel wherever it applies)")
    ap.add_argument("--nl-overlap", type=int, default=0, choices=[0, 1, 2],
                    help="cell512: projector GEMMs beside the transforms (plan option nl_overlap: 0 auto, "
                         "1 always beside, 2 always after)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy 1 GiB device to device once (reference kernel "
                         "for the FETCH_SIZE / WRITE_SIZE counter scale)")
    ap.add_argument("--gamma", action="store_true",
                    help="solve512: the same cell at Gamma on the half sphere with real wavefunctions "
                         "(two bands per transform, real products)")
    ap.add_argument("--class-profile", action="store_true",
                    help="solve512: after the timed solves, one more float64 solve with every kernel class "
                         "timed (HIP events around each class's launches); reports each class's time and "
                         "rate, the subspace products' fraction of the FP64 MFMA peak among them")
    ap.add_argument("--mode", choices=["solve", "hpsi"], default="solve",
                    help="solve: a step is one Davidson solve; hpsi: a step is one hpsi_apply of the "
                         "128-band block (for kernel profiles of H.psi alone)")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = "mixed" if args.workload in ("batch", "serve", "solve512") else "fp64"
    if args.steps is None:
        args.steps = {"cell512": 20, "solve512": 1}.get(args.workload, 3)
    if args.warmup is None:
        args.warmup = {"cell512": 3, "solve512": 0}.get(args.workload, 1)
    if args.ndim is None:
        args.ndim = 3 if (args.workload == "cell64" and args.precision == "fp64") else 2
    return args


def roofline(prof, dtype):
    name, (n, ms, units) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_s = ms / max(n, 1) / 1e3
    per_launch = units / max(n, 1)
    if name in HBM_KERNELS:
        achieved = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif name in MFMA_KERNELS:
        peak = FP32_MFMA_PEAK_TF if dtype == "f32" else FP64_PEAK_TF
        achieved = per_launch / avg_s / 1e12 if avg_s > 0 else 0.0
        out = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
        if name in COMPLEX3_KERNELS:
            # the conventional complex count is 8 M N K; the complex GEMMs run
            # Gauss's three-product form, 6 M N K on the matrix cores
            out["flops_counted_as"] = "8 M N K (conventional complex GEMM count)"
            out["mfma_flops_per_launch"] = 0.75 * per_launch
            out["mfma_pipe_frac"] = 0.75 * achieved / peak
    else:
        achieved = per_launch / avg_s / 1e12 if avg_s > 0 else 0.0
        out = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TF, "unit": "TFLOP/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = None
    out["kernel"] = name
    out["launches"] = n
    out["avg_us"] = avg_s * 1e6
    out["units_per_launch"] = per_launch
    return out


FFT_KERNELS = ("k_zinv", "k_plane", "k_zfwd")
PLANE_FORMS = {0: "one kernel per plane, a quad of lanes per 1D transform", 1: "three kernels",
               2: "one kernel per plane, 16-lane groups", 3: "one kernel per plane, generic LDS FFT"}
COMPLEX3_KERNELS = ("calbec_gemm", "add_nl_gemm", "zgemm_cn", "zgemm_nn")
NL_KERNELS = ("calbec_gemm", "add_nl_gemm")


def hpsi_graph_rates(ctx, p, plan, psi0, prec, reps):
    """band-H.psi/s of hpsi_apply launched eagerly and replayed from a HIP graph
    (one capture, `reps` replays), for this cell and for the small 8-atom cell
    (a = 10 bohr, 15 Ry, 16 bands), where launch latency dominates."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen

    def rates(pl, x, nb, pr):
        y = torch.empty_like(x)
        for _ in range(3):
            pl.hpsi(x, y, prec=pr)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            pl.hpsi(x, y, prec=pr)
        torch.cuda.synchronize()
        eager = nb * reps / (time.perf_counter() - a)
        g = pl.hpsi_graph(x, y, prec=pr)
        g.replay()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        graph = nb * reps / (time.perf_counter() - a)
        del g
        return {"eager": eager, "graph": graph}

    precs = [("fp64", pwdft.PW_FP64)] + ([("mixed", pwdft.PW_MIXED)] if prec == pwdft.PW_MIXED else [])
    out = {"cell64": {n: rates(plan, psi0, p.nb, pr) for n, pr in precs}}
    q = pwgen.config1()
    small = pwdft.Plan(ctx, q, precision=prec, nb_max=q.nb, ndim_max=0)
    try:
        x = torch.from_numpy(q.psi0).to(psi0.device)
        out["cell8"] = {n: rates(small, x, q.nb, pr) for n, pr in precs}
    finally:
        small.close()
    out["unit"] = "band-H·ψ/s"
    return out


def hpsi_stages(ctx, p, plan, psi0, prec, reps):
    """Per-stage rates of one H.psi of the band block: the transform stage (sphere -> sticks ->
    planes -> sticks -> sphere) against HBM, the projector products against the
    matrix cores.  "in_hpsi": the full product, where the projector products run on
    a side stream beside the transforms; "fft_alone": the same transforms of a plan
    without projectors (no contention)."""
    import dataclasses
    import torch
    from paper_0906_2569_amd import pwdft

    def measure(pl, pr):
        x = psi0.clone()
        y = torch.empty_like(x)
        for _ in range(3):
            pl.hpsi(x, y, prec=pr)
        torch.cuda.synchronize()
        pwdft.profile_enable(True)
        for _ in range(reps):
            pl.hpsi(x, y, prec=pr)
        torch.cuda.synchronize()
        prof = pwdft.profile_read()
        pwdft.profile_enable(False)
        return prof

    def summarize(prof, pr):
        out = {}
        calls = reps   # H.psi calls (a call launches each pass once per band chunk)
        t_fft = sum(prof[k][1] for k in FFT_KERNELS if k in prof) / calls * 1e-3
        b_fft = sum(prof[k][2] for k in FFT_KERNELS if k in prof) / calls
        if t_fft > 0:
            gbs = b_fft / t_fft / 1e9
            out["fft"] = {"us_per_hpsi": t_fft * 1e6, "alg_bytes": b_fft, "GB_per_s": gbs,
                          "hbm_frac": gbs / HBM_PEAK_GBS}
        ks = [k for k in NL_KERNELS if k in prof and prof[k][0]]
        if ks:
            t_nl = sum(prof[k][1] for k in ks) / calls * 1e-3
            f_nl = sum(prof[k][2] for k in ks) / calls
            peak = FP64_PEAK_TF if pr == pwdft.PW_FP64 else FP32_MFMA_PEAK_TF
            tf = f_nl / t_nl / 1e12
            out["nl_gemms"] = {"us_per_hpsi": t_nl * 1e6, "flops": f_nl, "TFLOP_per_s": tf, "peak": peak,
                               "mfma_frac": tf / peak}
        return out

    precs = [pwdft.PW_FP64] + ([pwdft.PW_MIXED] if prec == pwdft.PW_MIXED else [])
    res = {}
    q = dataclasses.replace(p, beta=np.zeros((0, p.npw), np.complex128), blk_off=np.zeros(1, np.int32),
                            dmat=np.zeros(0, np.complex128), tau=np.zeros((0, 3)))
    bare = pwdft.Plan(ctx, q, precision=prec, nb_max=p.nb, ndim_max=0)
    try:
        for pr in precs:
            key = "fp64" if pr == pwdft.PW_FP64 else "fp32"
            res[key] = {"in_hpsi": summarize(measure(plan, pr), pr),
                        "fft_alone": summarize(measure(bare, pr), pr).get("fft")}
    finally:
        bare.close()
    return res


def cpu_baseline(p, band_hpsi_per_solve, seconds):
    """The CPU oracle (dense rows of H applied to the band block) on a sample of rows."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    vt = oracle.vtilde_table(p.vloc_r)
    rng = np.random.default_rng(0)
    order = rng.permutation(p.npw)
    done, t0 = 0, time.perf_counter()
    chunk = 256
    while time.perf_counter() - t0 < seconds and done < p.npw:
        rows = np.sort(order[done:done + chunk])
        hr = oracle.h_rows(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat, rows, vt=vt)
        _ = p.psi0 @ hr.T
        done += len(rows)
    dt = time.perf_counter() - t0
    t_full = dt * p.npw / done                      # one dense H.psi of all 128 bands
    band_hpsi_s = p.nb / t_full
    solves_s = band_hpsi_s / band_hpsi_per_solve
    return {
        "value": solves_s, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"dense H rows (kinetic + direct-DFT V + projector term) built and applied to the "
                   f"128-band block for {done} of {p.npw} rows in {dt:.1f} s; full H.psi extrapolated "
                   f"({t_full:.1f} s, {band_hpsi_s:.3g} band-H.psi/s) and divided by the "
                   f"{band_hpsi_per_solve:.0f} band-H.psi one GPU solve needs; the reduced "
                   f"eigenproblems are not counted (upper bound on the oracle's solves/s)"),
        "band_hpsi_per_s": band_hpsi_s,
    }


def percentile(xs, q):
    """Nearest-rank percentile."""
    xs = sorted(xs)
    k = max(1, int(np.ceil(q / 100.0 * len(xs))))
    return xs[k - 1]


def bench_batch(args):
    """32 cells x 4 k-points: every problem solved one at a time in FP64, then all of
    them through davidson_solve_batched (mixed precision, concurrent workers)."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen
    dev = torch.device("cuda", 0)
    ps = pwgen.config4()
    ctx = pwdft.Context(0)
    opts = pwdft.default_opts(ndim=args.ndim, max_iter=400)
    psi0 = [torch.from_numpy(p.psi0).to(dev) for p in ps]
    nbands = sum(p.nb for p in ps)

    def run_seq(plans):
        xs = [x.clone() for x in psi0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, nh = [], 0
        for pl, x in zip(plans, xs):
            s, _, _, stt = pl.davidson(x, opts=opts)
            st.append(s)
            nh += stt.n_hpsi_fp64 + stt.n_hpsi_fp32
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st, nh

    def run_batch(plans):
        xs = [x.clone() for x in psi0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, sts, eigs, res, stats = pwdft.davidson_batched(ctx, plans, xs, opts=opts, nworkers=args.workers)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sts, sum(s.n_hpsi_fp64 + s.n_hpsi_fp32 for s in stats), eigs

    def hpsi_rate(plans, prec, batched):
        xs = psi0
        ys = [torch.empty_like(x) for x in xs]
        reps = 5
        for _ in range(2):
            pwdft.hpsi_batched(ctx, plans, xs, ys, prec=prec, nstreams=args.workers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if batched:
                pwdft.hpsi_batched(ctx, plans, xs, ys, prec=prec, nstreams=args.workers)
            else:
                for pl, x, y in zip(plans, xs, ys):
                    pl.hpsi(x, y, prec=prec)
        torch.cuda.synchronize()
        return nbands * reps / (time.perf_counter() - t0)

    plans64 = [pwdft.Plan(ctx, p, precision=pwdft.PW_FP64, nb_max=p.nb, ndim_max=args.ndim) for p in ps]
    run_seq(plans64[:4])
    t_seq, st_seq, nh_seq = run_seq(plans64)
    hp_seq = hpsi_rate(plans64, pwdft.PW_FP64, False)
    hp_b64 = hpsi_rate(plans64, pwdft.PW_FP64, True)
    for pl in plans64:
        pl.close()
    prec = pwdft.PW_MIXED if args.precision == "mixed" else pwdft.PW_FP64
    plans = [pwdft.Plan(ctx, p, precision=prec, nb_max=p.nb, ndim_max=args.ndim) for p in ps]
    run_batch(plans)
    times, last = [], None
    for _ in range(max(1, args.steps)):
        t, sts, nh_b, eigs = run_batch(plans)
        times.append(t)
        last = (sts, nh_b)
    t_b = float(np.median(times))
    hp_bm = hpsi_rate(plans, pwdft.PW_MIXED, True) if prec == pwdft.PW_MIXED else None
    for pl in plans:
        pl.close()
    line = {
        "metric": "band H·ψ/s and Davidson solves/s vs plain FP64 at 1e-8 Ry; p50/p99 latency",
        "value": len(ps) / t_b, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if prec == pwdft.PW_MIXED else "f64",
        "data": "synthetic (32 seeded cells a~U[10,20] bohr, 8-64 atoms, 25 Ry, k=(+-1/4,+-1/4,0))",
        "config": {"workload": "batch of 128 problems: 32 cells x 4 k-points, npw 2157-16382, nb 20-128, "
                               "Davidson to 1e-8 Ry", "problems": len(ps), "workers": args.workers,
                               "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "ndim": args.ndim, "precision": args.precision},
        "sequential_fp64_solves_per_s": len(ps) / t_seq,
        "speedup_vs_sequential_fp64": t_seq / t_b,
        "band_hpsi_per_s": {"fp64_sequential": hp_seq, "fp64_batched": hp_b64, "mixed_batched": hp_bm},
        "band_hpsi_per_solve": {"sequential_fp64": nh_seq / len(ps), "batched": last[1] / len(ps)},
        "status": {"sequential_fp64_ok": int(sum(s == 0 for s in st_seq)), "batched_ok": int(sum(s == 0 for s in last[0]))},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_serve(args):
    """Open-loop Poisson traces of requests (log-uniform atom counts 8..max at
    constant density, up to the 512-atom, 144^3, 1024-band cell) through the
    serving loop: a closed burst of one request set measures the capacity;
    a second set then arrives at 20 req/s (the configured rate, above
    capacity: queueing dominates the latency) and at 0.7 x capacity."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen
    dev = torch.device("cuda", 0)
    ctx = pwdft.Context(0)
    opts = pwdft.default_opts(ndim=args.ndim, max_iter=400)
    nreq = args.requests
    t0 = time.perf_counter()
    reqs = [pwgen.serving_request(i, ecut_ry=args.ecut, max_atoms=args.max_atoms) for i in range(2 * nreq)]
    t_gen = time.perf_counter() - t0
    print(f"bench: {2 * nreq} requests generated in {t_gen:.0f} s", file=sys.stderr, flush=True)
    prec = pwdft.PW_MIXED if args.precision == "mixed" else pwdft.PW_FP64

    def run(batch, arrivals):
        srv = pwdft.Server(ctx, nworkers=args.workers, precision=prec)
        start = srv.clock()
        subs = []
        for p, ta in zip(batch, arrivals):
            while srv.clock() - start < ta:
                time.sleep(min(0.002, max(0.0, ta - (srv.clock() - start))))
            x = torch.from_numpy(p.psi0).to(dev)
            subs.append(srv.submit(p, x, opts=opts))
        res = [srv.wait(t) for t, _, _ in subs]
        pools.append(srv.info())
        srv.close()
        lat = [r[2][2] - r[2][0] for r in res]
        t_end = max(r[2][2] for r in res) - start
        ok = sum(r[0] == 0 for r in res)
        return lat, t_end, ok, res

    pools = []

    def poisson(rate, seed):
        rng = np.random.default_rng(seed)
        return np.cumsum(rng.exponential(1.0 / rate, size=nreq)).tolist()

    # warm-up, then capacity: the first request set submitted at once
    run(reqs[:4], [0.0] * 4)
    lat_b, t_b, ok_b, _ = run(reqs[:nreq], [0.0] * nreq)
    capacity = nreq / t_b
    print(f"bench: burst capacity {capacity:.3g} solves/s", file=sys.stderr, flush=True)
    traces = {}
    for key, lam, seed in (("offered_20_per_s", 20.0, 20090605), ("offered_0.7_capacity", 0.7 * capacity, 20090606)):
        lat, t_end, ok, res = run(reqs[nreq:], poisson(lam, seed))
        big = [(int(p.nbeta // 4), r[2][2] - r[2][1]) for p, r in zip(reqs[nreq:], res)]
        traces[key] = {"offered_req_per_s": lam, "solves_per_s": nreq / t_end,
                       "latency_s": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "max": max(lat)},
                       "ok": int(ok), "largest_request": max(big)}
        print(f"bench: {key}: {nreq / t_end:.3g} solves/s, p50 {percentile(lat, 50):.2f} s, "
              f"p99 {percentile(lat, 99):.2f} s", file=sys.stderr, flush=True)
    nat = [int(p.nbeta // 4) for p in reqs[nreq:]]
    main = traces["offered_20_per_s"]
    line = {
        "metric": "band H·ψ/s and Davidson solves/s vs plain FP64 at 1e-8 Ry; p50/p99 latency",
        "value": main["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": nreq, "warmup": 4,
        "ms_per_step": 1e3 / main["solves_per_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if prec == pwdft.PW_MIXED else "f64",
        "data": "synthetic requests: atoms log-uniform 8..max, a = 41 (n/512)^(1/3) bohr, k = t b1",
        "config": {"workload": f"served requests, {args.ecut:g} Ry, 8-{args.max_atoms} atoms (nb = 2 atoms), "
                               f"Poisson arrivals at 20 req/s and at 0.7 x measured capacity", "requests": nreq,
                   "workers": args.workers, "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "ndim": args.ndim, "precision": args.precision},
        "latency_s": main["latency_s"],
        "traces": traces,
        "capacity_solves_per_s": capacity,
        "burst_latency_s": {"p50": percentile(lat_b, 50), "p99": percentile(lat_b, 99)},
        "atoms": {"min": min(nat), "median": int(np.median(nat)), "max": max(nat)},
        "memory_pool": {"pool_bytes": pools[-1]["pool_bytes"], "peak_use": max(q["pool_peak"] for q in pools),
                        "allocations_outside_pool": sum(q["pool_fallbacks"] for q in pools),
                        "requests_served": sum(q["served"] for q in pools)},
        "input_generation_s": t_gen,
    }
    print(json.dumps(line), flush=True)
    return 0


# HBM bytes per launch of a kernel class, from the rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters (each scaled by a device-to-device copy of known size:
# fetched bytes = 2.0 x FETCH_SIZE KiB x 1024, written = 1.0 x WRITE_SIZE KiB
# x 1024), keyed by (workload, kernel class).  Summaries under profiles/.
# An entry is removed whenever its kernel changes.
TRAFFIC_BYTES = {
    # calibrated FETCH_SIZE + WRITE_SIZE bytes per launch of the dominant
    # kernel, taken with the kernel as it now stands; an entry is removed
    # whenever that kernel changes, until its counters are taken again.
    # k_gemm_cn<float, float, double> (three-product form, 128 x 64 tiles),
    # 8 K chunks: 56.085 GB read + 0.134 GB written
    # (profiles/hpsi_mixed_512atom_144cubed.md)
    ("cell512_mixed", "calbec_gemm"): 56.219e9,
}


def golden_config2():
    """Lowest 128 eigenvalues of the 64-atom cell's dense Hamiltonian, as the
    CPU oracle wrote them (tests/golden/make_config2_eigenvalues.py)."""
    return np.loadtxt(os.path.join(ROOT, "tests", "golden", "config2_eigenvalues.txt"))


def cell64_solves(ctx, nsolves):
    """Davidson solves of the 64-atom cell (npw 18277, 72^3, 256 beta, 128 bands)
    in float64 (basis 3 nb) and in mixed precision (basis 2 nb, the ladder);
    locking on, to 1e-8 Ry; every solve's eigenvalues against the golden
    dense-oracle values."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen
    p = pwgen.config2()
    w = golden_config2()
    dev = torch.device("cuda", 0)
    psi0 = torch.from_numpy(p.psi0).to(dev)
    out = {}
    for key, prec, ndim in (("fp64", pwdft.PW_FP64, 3), ("mixed", pwdft.PW_MIXED, 2)):
        plan = pwdft.Plan(ctx, p, precision=prec, nb_max=p.nb, ndim_max=ndim)
        try:
            psi = torch.empty_like(psi0)
            eig = torch.empty(p.nb, dtype=torch.float64, device=dev)
            resid = torch.empty_like(eig)
            opts = pwdft.default_opts(ndim=ndim, max_iter=400)
            psi.copy_(psi0)
            plan.davidson(psi, eig, resid, opts=opts)        # untimed
            torch.cuda.synchronize()
            t_tot, errs, sts, stats, rmax = 0.0, [], [], None, 0.0
            for _ in range(nsolves):
                psi.copy_(psi0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, _, _, stats = plan.davidson(psi, eig, resid, opts=opts)
                torch.cuda.synchronize()
                t_tot += time.perf_counter() - t0
                e = np.abs(eig.cpu().numpy() - w)
                errs.append(e)
                sts.append(st)
                rmax = max(rmax, float(resid.max()))
            out[key] = {
                "solves_per_s": nsolves / t_tot, "ms_per_solve": t_tot * 1e3 / nsolves, "ndim": ndim,
                "max_abs_eig_err_ha": float(max(e.max() for e in errs)),
                "eig_err_ha_last_solve": [float(f"{x:.2e}") for x in errs[-1]],
                "max_resid_ha": rmax, "status": sts, "stats": stats.asdict(),
                "band_hpsi_per_solve": stats.n_hpsi_fp64 + stats.n_hpsi_fp32,
            }
        finally:
            plan.close()
    # the same cell on the Gamma-point real-wavefunction path (half sphere; the
    # -i of its p projectors leaves H unchanged for diagonal D, so the same
    # golden eigenvalues apply)
    g = pwgen.gamma_cell(20.5, 25.0, 64, 128, pwgen.SEED_BASE + 2, nr=(72, 72, 72))
    plan = pwdft.Plan(ctx, g, precision=pwdft.PW_FP64, nb_max=g.nb, ndim_max=3, gamma=1)
    try:
        gpsi0 = torch.from_numpy(g.psi0).to(dev)
        psi = torch.empty_like(gpsi0)
        eig = torch.empty(g.nb, dtype=torch.float64, device=dev)
        resid = torch.empty_like(eig)
        opts = pwdft.default_opts(ndim=3, max_iter=400)
        psi.copy_(gpsi0)
        plan.davidson(psi, eig, resid, opts=opts)
        torch.cuda.synchronize()
        t_tot, emax, sts = 0.0, 0.0, []
        for _ in range(nsolves):
            psi.copy_(gpsi0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _, _, stats = plan.davidson(psi, eig, resid, opts=opts)
            torch.cuda.synchronize()
            t_tot += time.perf_counter() - t0
            emax = max(emax, float(np.abs(eig.cpu().numpy() - w).max()))
            sts.append(st)
        out["gamma_fp64"] = {"solves_per_s": nsolves / t_tot, "ms_per_solve": t_tot * 1e3 / nsolves, "ndim": 3,
                             "max_abs_eig_err_ha": emax, "status": sts, "stats": stats.asdict(),
                             "npw_half": g.npw}
    finally:
        plan.close()
    out["mixed_over_fp64_solves"] = out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    out["gamma_over_complex_fp64_solves"] = out["gamma_fp64"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    out["reference"] = ("lowest 128 eigenvalues of the dense 18277^2 oracle Hamiltonian "
                        "(tests/golden/config2_eigenvalues.txt); target 5e-9 Ha = 1e-8 Ry")
    return out


def cpu_baseline_rows(p, got, seconds):
    """The CPU oracle on a bounded sample of the workload: dense rows of H
    (kinetic + direct-DFT V + projector term) built and applied to the whole
    band block, 32 rows at a time for about `seconds`.  The same rows are the
    parity sample of the GPU products `got` ({name: [nb][npw] device tensor}):
    per band, ||(H psi)_gpu - (H psi)_oracle|| / ||(H psi)_oracle|| over the
    sampled rows.  Then the CPU FFT method (3D FFTs + BLAS, float64) on a few
    bands, checked on the same rows."""
    import torch
    import oracle
    from oracle import fft_method
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    rng = np.random.default_rng(0)
    order = rng.permutation(p.npw)
    vt = oracle.vtilde_table(p.vloc_r)
    done, t_rows = 0, 0.0
    chunk = 32
    parity = None
    while (t_rows < seconds or done == 0) and done < p.npw:
        rows = np.sort(order[done:done + chunk])
        t0 = time.perf_counter()
        hr = oracle.h_rows(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat, rows, vt=vt)
        ref = p.psi0 @ hr.T                                   # [nb][rows]
        t_rows += time.perf_counter() - t0
        if parity is None:
            idx = torch.from_numpy(rows).to(next(iter(got.values())).device)
            parity = {"rows": int(len(rows))}
            for name, y in got.items():
                g = y.index_select(1, idx).cpu().numpy()
                rel = np.linalg.norm(g - ref, axis=1) / np.linalg.norm(ref, axis=1)
                parity[name] = {"max_band_rel_err": float(rel.max()), "median_band_rel_err": float(np.median(rel))}
            ref_rows, rows0 = ref, rows
        done += len(rows)
    band_hpsi_s = p.nb * done / (t_rows * p.npw)
    out = {
        "value": band_hpsi_s, "unit": "band-H·ψ/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"dense H rows of the oracle built and applied to all {p.nb} bands for {done} of {p.npw} "
                   f"rows in {t_rows:.1f} s; rate = bands x sampled rows / (time x npw)"),
    }
    # CPU FFT method on the first few bands (all host cores)
    nbf = min(4, p.nb)
    t0 = time.perf_counter()
    hf = fft_method.hpsi(p.miller, p.kpg, p.vloc_r, p.beta, p.blk_off, p.dmat, p.psi0[:nbf])
    t_fft = time.perf_counter() - t0
    chk = np.linalg.norm(hf[:, rows0] - ref_rows[:nbf], axis=1) / np.linalg.norm(ref_rows[:nbf], axis=1)
    fftm = {"value": nbf / t_fft, "unit": "band-H·ψ/s", "cores": int(os.cpu_count() or 1),
            "kind": "cpu_fft_method_fp64",
            "sample": f"{nbf} bands through scipy.fft 3D transforms and BLAS products in {t_fft:.1f} s",
            "max_band_rel_err_vs_oracle_rows": float(chk.max())}
    return out, fftm, parity


def gamma_rates(ctx, p, reps, mixed_complex, fp64_complex):
    """band-H.psi/s of the same cell on the Gamma-point real-wavefunction path
    (half sphere, two bands per transform, real projector products), mixed and
    float64, against the complex path."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen
    g = pwgen.gamma_cell(p.a, p.ecut_ry, p.natoms, p.nb, p.meta.get("seed") or pwgen.SEED_BASE + 5, nr=p.nr)
    plan = pwdft.Plan(ctx, g, precision=pwdft.PW_MIXED, nb_max=g.nb, ndim_max=0, gamma=1)
    try:
        x = torch.from_numpy(g.psi0).cuda()
        y = torch.empty_like(x)
        out = {"npw_half": g.npw}
        for key, pr in (("mixed", pwdft.PW_MIXED), ("fp64", pwdft.PW_FP64)):
            plan.hpsi(x, y, prec=pr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.hpsi(x, y, prec=pr)
            torch.cuda.synchronize()
            out[key] = g.nb * reps / (time.perf_counter() - t0)
        out["mixed_over_complex_mixed"] = out["mixed"] / mixed_complex
        out["fp64_over_complex_fp64"] = out["fp64"] / fp64_complex
        out["unit"] = "band-H·ψ/s"
        return out
    finally:
        plan.close()


def bench_solve512(args):
    """Davidson solves of the 512-atom cell (npw 191,471, 144^3 grid, 2048
    projectors, 1024 bands; basis 2 nb, locking, residuals to 1e-6 Ha) in the
    chosen precision, timed one solve per step.  A mixed run also solves in
    float64 once, for the ratio and the largest eigenvalue difference."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    if args.gamma:
        # the same cell (a = 41 bohr, 30 Ry, 512 atoms, seed of the full-sphere form) at Gamma
        p = pwgen.gamma_cell(41.0, 30.0, 512, 1024, pwgen.SEED_BASE + 5, name="cfg5_gamma")
    else:
        p = pwgen.config5_largest(nb=1024)
    print(f"bench: cell generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = pwdft.Context(0)
    opts = pwdft.default_opts(ndim=args.ndim, max_iter=400)
    psi0 = torch.from_numpy(np.ascontiguousarray(p.psi0)).to(dev)
    gam = 1 if args.gamma else 0

    prof_out = {}

    def solves(prec, nsteps, nwarm, profile=False):
        plan = pwdft.Plan(ctx, p, precision=prec, nb_max=p.nb, ndim_max=args.ndim, gamma=gam)
        try:
            psi = torch.empty_like(psi0)
            eig = torch.empty(p.nb, dtype=torch.float64, device=dev)
            resid = torch.empty_like(eig)
            out = []
            for i in range(nwarm + nsteps):
                psi.copy_(psi0)
                torch.cuda.synchronize()
                if profile:
                    pwdft.profile_enable(True)
                t = time.perf_counter()
                st, _, _, stats = plan.davidson(psi, eig, resid, opts=opts)
                torch.cuda.synchronize()
                if i >= nwarm:
                    out.append((time.perf_counter() - t, st, stats.asdict()))
            return out, eig.cpu().numpy(), resid.cpu().numpy()
        finally:
            if profile:
                prof_out.update({k: v for k, v in pwdft.profile_read().items() if v[0] > 0})
                pwdft.profile_enable(False)
            plan.close()

    prec = pwdft.PW_MIXED if args.precision == "mixed" else pwdft.PW_FP64
    runs, e, r = solves(prec, args.steps, args.warmup)
    secs = [t for t, _, _ in runs]
    sec = sum(secs) / len(secs)
    line = {"metric": "solves/s", "value": 1.0 / sec, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
            "config": {"workload": ("Davidson solve of the 512-atom cell (npw 191,471, 144^3, 2048 projectors, "
                                    "1024 bands)" + (" at Gamma: half sphere of " + f"{p.npw:,}" +
                                                     " coefficients, real wavefunctions" if gam else "")),
                       "ndim": args.ndim, "precision": args.precision, "gamma": bool(gam)},
            "status": [st for _, st, _ in runs], "solve_stats": runs[-1][2],
            "eig_range_ha": [float(e[0]), float(e[-1])], "max_resid_ha": float(r.max())}
    if args.precision == "mixed":
        runs64, e64, _ = solves(pwdft.PW_FP64, 1, 0)
        line["fp64_seconds"] = runs64[0][0]
        line["fp64_status"] = runs64[0][1]
        line["mixed_over_fp64"] = runs64[0][0] / sec
        line["max_abs_eig_diff_vs_fp64_ha"] = float(np.abs(e - e64).max())
    if args.class_profile:
        # every class timed with events in one more float64 solve (kept out of
        # the figures above); flops for the products and factorizations, bytes
        # for the transform passes and vector kernels
        runs_p, _, _ = solves(pwdft.PW_FP64, 1, 0, profile=True)
        flop_classes = {"calbec_gemm", "add_nl_gemm", "zgemm_cn", "zgemm_nn", "k_chol", "k_trinv", "k_tridiag",
                        "k_backtr"}
        cls = {}
        for k, (n, ms, units) in sorted(prof_out.items(), key=lambda kv: -kv[1][1]):
            rec = {"launches": n, "ms": round(ms, 2)}
            if units > 0 and ms > 0:
                if k in flop_classes:
                    rec["tflops"] = round(units / ms * 1e-9, 2)
                else:
                    rec["gbs"] = round(units / ms * 1e-6, 1)
            cls[k] = rec
        line["fp64_solve_profiled_seconds"] = runs_p[0][0]
        line["fp64_solve_classes"] = cls
        line["fp64_solve_classes_note"] = ("one float64 solve with events around every kernel class; zgemm_cn: "
                                           "the projections phi^H H phi, phi^H phi and the locked-band "
                                           "projections; zgemm_nn: Ritz rotations, locked-band updates and the "
                                           "Cholesky trailing updates (also inside k_chol); peak FP64 MFMA "
                                           f"{FP64_PEAK_TF} TFLOP/s")
    print(json.dumps(line), flush=True)
    return 0 if all(st == 0 for _, st, _ in runs) else 1


def bench_cell512(args):
    """Mixed-precision H.psi of the 1024-band block of the 512-atom 144^3 cell,
    against the same product in plain float64."""
    import torch
    from paper_0906_2569_amd import pwdft, pwgen
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    p = pwgen.config5_largest(nb=args.nbands)
    t_gen = time.perf_counter() - t0
    print(f"bench: cell generated in {t_gen:.1f} s (npw {p.npw}, grid {p.nr}, {p.nbeta} beta, {p.nb} bands)",
          file=sys.stderr, flush=True)
    ctx = pwdft.Context(0)
    plan = pwdft.Plan(ctx, p, precision=pwdft.PW_MIXED, nb_max=p.nb, ndim_max=0, plane_mode=args.plane_mode,
                      nl_overlap=args.nl_overlap)
    info = plan.info()
    psi0 = torch.from_numpy(p.psi0).to(dev)
    y = torch.empty_like(psi0)
    torch.cuda.synchronize()
    # warm-up: every kernel class profiled (the kernel_ms breakdown)
    pwdft.profile_enable(True)
    for _ in range(args.warmup):
        plan.hpsi(psi0, y, prec=pwdft.PW_MIXED)
    torch.cuda.synchronize()
    prof_all = {k: v for k, v in pwdft.profile_read().items() if v[0] > 0}
    dominant = max(prof_all.items(), key=lambda kv: kv[1][1])[0]
    # timed steps: events around the dominant class only
    pwdft.profile_only(dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.hpsi(psi0, y, prec=pwdft.PW_MIXED)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: v for k, v in pwdft.profile_read().items() if v[0] > 0}
    pwdft.profile_enable(False)
    value = p.nb * args.steps / (t1 - t0)
    print(f"bench: mixed H.psi {value:.4g} band-H.psi/s", file=sys.stderr, flush=True)
    # plain float64 on the same GPU and plan (the metric's baseline)
    y64 = torch.empty_like(psi0)
    plan.hpsi(psi0, y64, prec=pwdft.PW_FP64)
    torch.cuda.synchronize()
    reps64 = max(3, args.steps // 4)
    a = time.perf_counter()
    for _ in range(reps64):
        plan.hpsi(psi0, y64, prec=pwdft.PW_FP64)
    torch.cuda.synchronize()
    rate64 = p.nb * reps64 / (time.perf_counter() - a)
    print(f"bench: float64 H.psi {rate64:.4g} band-H.psi/s", file=sys.stderr, flush=True)
    stages = None
    if not args.no_stages:
        stages = hpsi_stages(ctx, p, plan, psi0, pwdft.PW_MIXED, 3)
    gamma = None if args.no_gamma else gamma_rates(ctx, p, max(3, args.steps // 4), value, rate64)
    solves = cell64_solves(ctx, args.solves) if args.solves > 0 else None
    rl = roofline(prof, "f32")
    tb = TRAFFIC_BYTES.get(("cell512_mixed", rl["kernel"]))
    rl["traffic"] = tb
    line = {
        "metric": "band H·ψ/s and Davidson solves/s vs plain FP64 at 1e-8 Ry; p50/p99 latency",
        "value": value, "unit": "band-H·ψ/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": value / rate64,
        "vs_baseline_is": "mixed-precision H.psi over plain float64 H.psi of the same cell on the same GPU "
                          "(the metric's baseline; the paper reports no number for this path)",
        "dtype": "f32 (transforms, projector GEMMs; complex128 in/out)",
        "data": "synthetic (seeded cell, V(G), projectors, D, trial block)",
        "config": {"workload": f"largest served cell: cubic a=41 bohr, Gamma, ecutwfc 30 Ry (npw {p.npw}), "
                               f"FFT {p.nr[0]}^3, 512 atoms, {p.nbeta} beta, {p.nb} bands; one mixed-precision "
                               f"hpsi_apply per step",
                   "npw": p.npw, "fft": list(p.nr), "nbeta": p.nbeta, "nbands": p.nb, "precision": "mixed",
                   "band_chunk": info["band_chunk"],
                   "plane_pass": {k: PLANE_FORMS[info[k]] for k in ("plane64", "plane32")}},
        "band_hpsi_per_s_mixed": value,
        "band_hpsi_per_s_fp64": rate64,
        "ms_per_hpsi": {"mixed": 1e3 * p.nb / value, "fp64": 1e3 * p.nb / rate64},
        "roofline": rl,
        "hpsi_stages": stages,
        "gamma_real_path": gamma,
        "cell64_solves": solves,
        "kernel_ms": {k: round(v[1] / max(args.warmup, 1), 3)
                      for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1][1])},
        "kernel_ms_from": "the warm-up steps, every kernel class timed (per step)",
        "input_generation_s": t_gen,
    }
    if not args.no_cpu_baseline:
        cpu, fftm, parity = cpu_baseline_rows(p, {"mixed": y, "fp64": y64}, args.cpu_seconds)
        line["cpu_baseline"] = cpu
        line["cpu_fft_method"] = fftm
        line["parity_sampled_rows"] = parity
        line["speedup_vs_cpu_fft_method"] = value / fftm["value"]
    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 2 * src.numel() * 8
    print(json.dumps(line), flush=True)
    plan.close()
    return 0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(independent cells and k-points would shard one group per GPU)", file=sys.stderr)
        return 2
    if args.workload in ("batch", "serve"):
        # every solve drives two streams (transforms and the projector side
        # stream): 16 hardware queues keep 8 and more workers from sharing
        # them (HIP's default is 4).  Set before the GPU runtime starts.
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 16:
            os.environ["GPU_MAX_HW_QUEUES"] = "16"
        if args.workers is None:
            args.workers = 12 if args.workload == "batch" else 8
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "cell512":
        return bench_cell512(args)
    if args.workload == "solve512":
        return bench_solve512(args)
    import torch
    from paper_0906_2569_amd import pwdft, pwgen

    dev = torch.device("cuda", 0)
    p = pwgen.config2()
    prec = pwdft.PW_MIXED if args.precision == "mixed" else pwdft.PW_FP64
    ctx = pwdft.Context(0)
    plan = pwdft.Plan(ctx, p, precision=prec, nb_max=p.nb, ndim_max=args.ndim)
    psi0 = torch.from_numpy(p.psi0).to(dev)
    psi = torch.empty_like(psi0)
    eig = torch.empty(p.nb, dtype=torch.float64, device=dev)
    resid = torch.empty_like(eig)
    opts = pwdft.default_opts(ndim=args.ndim, max_iter=400)

    def step():
        if args.mode == "hpsi":
            plan.hpsi(psi0, psi, prec=prec)
            return 0, None, None, None
        psi.copy_(psi0)
        return plan.davidson(psi, eig, resid, opts=opts)

    # the warm-up steps are profiled in full (every kernel class: the kernel_ms
    # breakdown); the timed steps bracket only the dominant class with events,
    # so that the events add no gaps between the other kernels
    pwdft.profile_enable(True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prof_all = {k: v for k, v in pwdft.profile_read().items() if v[0] > 0}
    dominant = max(prof_all.items(), key=lambda kv: kv[1][1])[0] if prof_all else None
    pwdft.profile_only(dominant)
    stats_all = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, _, _, stats = step()
        stats_all.append((st, stats.asdict() if stats is not None else {"n_hpsi_fp64": p.nb, "n_hpsi_fp32": 0}))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pwdft.profile_read()
    pwdft.profile_enable(False)
    if not prof_all:
        prof_all = {k: v for k, v in prof.items() if v[0] > 0}
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solves_s = args.steps / (t1 - t0)
    hpsi_per_solve = float(np.mean([s["n_hpsi_fp64"] + s["n_hpsi_fp32"] for _, s in stats_all]))

    # band-H.psi/s of hpsi_apply alone (float64, and float32 arithmetic if the plan allows)
    def hpsi_rate(pr):
        x = psi0.clone()
        y = torch.empty_like(x)
        for _ in range(3):
            plan.hpsi(x, y, prec=pr)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.hpsi_reps):
            plan.hpsi(x, y, prec=pr)
        torch.cuda.synchronize()
        return p.nb * args.hpsi_reps / (time.perf_counter() - a)

    rate64 = hpsi_rate(pwdft.PW_FP64)
    rate_mixed = None
    if prec == pwdft.PW_MIXED:
        rate_mixed = hpsi_rate(pwdft.PW_MIXED)
    stages = None if args.no_stages else hpsi_stages(ctx, p, plan, psi0, prec, args.hpsi_reps)
    graphs = None if args.no_stages else hpsi_graph_rates(ctx, p, plan, psi0, prec, args.hpsi_reps)

    dtype = "f64" if prec == pwdft.PW_FP64 else "f64+f32"
    if args.mode == "hpsi":
        value, unit = p.nb * args.steps / (t1 - t0), "band-H·ψ/s"
    else:
        value, unit = solves_s, "solves/s"
    line = {
        "metric": "band H·ψ/s and Davidson solves/s vs plain FP64 at 1e-8 Ry; p50/p99 latency",
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded cell, V(G), projectors, D, trial block)",
        "config": {"workload": "cubic 64-atom cell a=20.5 bohr, Gamma, ecutwfc 25 Ry (npw 18277), "
                               "FFT 72^3, 256 beta, 128 bands, Davidson to 1e-8 Ry",
                   "npw": p.npw, "fft": list(p.nr), "nbeta": p.nbeta, "nbands": p.nb,
                   "ndim": args.ndim, "precision": args.precision},
        "band_hpsi_per_s_fp64": rate64,
        "band_hpsi_per_s_mixed": rate_mixed,
        "band_hpsi_per_solve": hpsi_per_solve,
        "mode": args.mode,
        "solve_stats": stats_all[-1][1],
        "solve_status": [s for s, _ in stats_all],
        "eig_min_max_ha": [float(eig.min()), float(eig.max())] if args.mode == "solve" else None,
        "max_resid_ha": float(resid.max()) if args.mode == "solve" else None,
        "roofline": roofline({k: v for k, v in prof.items() if v[0] > 0}, "f64" if prec == 0 else "f32"),
        "hpsi_stages": stages,
        "hpsi_graph": graphs,
        "kernel_ms": {k: round(v[1], 3) for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1][1]) if v[0]},
        # matrix-core products of the solve (subspace projections, Ritz
        # rotations, reduced products, projector terms): conventional
        # 8 M N K flops over their time, against the peak of the precision
        "gemm_rates_fp64": ({k: {"TFLOP_per_s": v[2] / (v[1] * 1e-3) / 1e12,
                                 "frac_of_fp64_peak": v[2] / (v[1] * 1e-3) / 1e12 / FP64_PEAK_TF}
                             for k, v in prof_all.items() if k in MFMA_KERNELS and v[1] > 0 and v[2] > 0}
                            if prec == pwdft.PW_FP64 else None),
        "kernel_ms_from": ("the warm-up steps, every kernel class timed" if args.warmup > 0
                           else "the timed steps"),
    }
    if not args.no_cpu_baseline and args.mode == "solve":
        line["cpu_baseline"] = cpu_baseline(p, hpsi_per_solve, args.cpu_seconds)
    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 2 * src.numel() * 8
    print(json.dumps(line), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
