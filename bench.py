"""Benchmark of the R-distance engine on MI355X.

Default workload (one step = one full solve through the C ABI):
  ER(8192, 0.02) directed graph, gamma = 0.5 / max out-degree, FP64 blocked
  Gauss-Jordan on the FP64 matrix cores with the int16 readout fused into the
  last update.  Inputs (adjacency and output buffer) are resident in HBM
  before the timed region.

Prints ONE JSON line: graphs/s (whole job), ms per step, effective TFLOP/s
(2 n^3 / t), p50/p99 step latency, the roofline of the dominant kernel (the
trailing-update kernel, timed with HIP events on its launch stream inside
the library), and the CPU oracle timed on a bounded sample of the same solve.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c3|c4|c5|f1|f2|f3|f4]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0

UPDATE_SOURCES = ["paper_2308_07403_amd/csrc/rd_update.hip", "paper_2308_07403_amd/csrc/rd_device.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_sha(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(profile_name: str, sha: str):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE),
    scaled by a copy kernel of known size; None if missing or taken on other sources."""
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_sha:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


def read_mfma_flops(profile_name: str, sha: str):
    """Matrix-core flops per launch from rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_*
    (x 512); None if missing or taken on other sources."""
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_sha:\s*([0-9a-f]+)", text)
    m_f = re.search(r"mfma_flops_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_f or m_sha.group(1) != sha:
        return None
    return float(m_f.group(1))


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def cpu_baseline_c2(A: np.ndarray, gjsteps: int, rows: int, runs: int = 5):
    """The oracle as it stands, on a bounded sample of the same n = 8192 solve:
    gate + M build on the whole graph, `gjsteps` of the n Gauss-Jordan steps,
    the readout of `rows` rows; scaled to one full solve (every GJ step and
    every readout row costs the same).  The Gauss-Jordan sample and the
    readout are timed `runs` times (M rebuilt before each) and the medians
    used.  Beside it, full oracle solves of an n = 2048 graph of the same
    density (the C2 subsample), median of `runs`."""
    import oracle
    import graphgen as gg
    n = A.shape[0]
    t0 = time.perf_counter()
    prep = oracle.prepare(A, -0.5)
    M = oracle.build_m(A, prep.gamma)
    t_build = time.perf_counter() - t0
    t_gj, t_rd = [], []
    for r in range(runs):
        if r:
            M = oracle.build_m(A, prep.gamma)
        t1 = time.perf_counter()
        oracle.gj_steps_inplace(M, 0, gjsteps)
        t2 = time.perf_counter()
        oracle.readout(np.ascontiguousarray(M[:rows, :rows]), prep.gamma)   # rows x rows entries
        t3 = time.perf_counter()
        t_gj.append(t2 - t1)
        t_rd.append(t3 - t2)
    del M
    gj, rd = float(np.median(t_gj)), float(np.median(t_rd))
    t_full = t_build + gj * n / gjsteps + rd * (n * n) / (rows * rows)
    sub = gg.c2_subsample(0, fresh=True)
    t_sub = []
    for _ in range(runs):
        t4 = time.perf_counter()
        oracle.solve(sub, -0.5, keep_y=False)
        t_sub.append(time.perf_counter() - t4)
    m_sub = float(np.median(t_sub))
    return {
        "value": 1.0 / t_full, "unit": "graphs/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": (f"n=8192 C2 graph: gate+M build in full ({t_build:.2f} s), {gjsteps} of {n} Gauss-Jordan "
                   f"steps (median of {runs} runs {gj:.2f} s, range {min(t_gj):.2f}-{max(t_gj):.2f}), readout of "
                   f"{rows}x{rows} entries (median {rd:.3f} s); scaled linearly to one solve ({t_full:.0f} s "
                   f"extrapolated)"),
        "full_n2048": {"median_s": m_sub, "min_s": float(min(t_sub)), "max_s": float(max(t_sub)), "runs": runs,
                       "graphs_per_s": 1.0 / m_sub, "scaled_to_n8192_s": m_sub * 64.0,
                       "graph": "fresh ER(2048, 0.02), the C2 density (c2/sub seed 0)"},
    }


def cpu_floyd_warshall_c2(A: np.ndarray, ksteps: int):
    import oracle
    n = A.shape[0]
    t0 = time.perf_counter()
    oracle.floyd_warshall(A, k_steps=ksteps)
    t = time.perf_counter() - t0
    return {"value": 1.0 / (t * n / ksteps), "unit": "graphs/s", "cores": oracle.num_threads(),
            "sample": f"{ksteps} of {n} Floyd-Warshall relaxation rounds, scaled to all {n}"}


def measure_mixed(ctx, R, torch, A, D_ref, steps, stream):
    """The mixed-precision solve of the same graph: time per solve, its split,
    the fallback fraction and D against the FP64 result."""
    n = A.shape[0]
    D = torch.empty((n, n), dtype=torch.int16, device="cuda")
    info = R.PinnedInfo(1)
    ctx.solve_async(A, -0.5, R.RDIST_MIXED_F32, D, info=info, stream=stream)    # warm-up
    torch.cuda.synchronize()
    # timed region: events only around the FP32 GEMM phases (the dominant kernels)
    ctx.set_timing(True, classes=[R.RDIST_K_MIXED_GEMM])
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.solve_async(A, -0.5, R.RDIST_MIXED_F32, D, info=info, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    gemm = ctx.kernel_stats(R.RDIST_K_MIXED_GEMM)
    # the split from one more solve with every class timed
    ctx.set_timing(True)
    ctx.solve_async(A, -0.5, R.RDIST_MIXED_F32, D, info=info, stream=stream)
    torch.cuda.synchronize()
    split = {name: ctx.kernel_stats(k)["total_ms"] for name, k in
             (("ingest", R.RDIST_K_INGEST), ("panel_fp64", R.RDIST_K_PANEL), ("fp32_rows", R.RDIST_K_ROWCOL),
              ("fp32_gemm", R.RDIST_K_MIXED_GEMM),
              ("certify", R.RDIST_K_CERTIFY), ("refine", R.RDIST_K_REFINE))}
    ctx.set_timing(False)
    st = info.get(0).as_dict()
    mism = int((D != D_ref).sum().item())
    gemm_tf = gemm["flops"] / max(gemm["total_ms"], 1e-9) / 1e9
    return {"ms_per_solve": ms, "graphs_per_s": 1e3 / ms, "eff_tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12,
            "fallback_fraction": st["fallback_fraction"], "n_uncertified": st["n_uncertified"],
            "certification_margin": 0.05, "split_ms": split,
            "fp32_gemm_tflops": gemm_tf, "fp32_gemm_frac_of_peak": gemm_tf / FP32_PEAK_TFLOPS,
            "d_mismatches_vs_fp64": mism}


def bench_c2(args, torch, R, gg):
    n = 8192
    fl = R.RDIST_F64 | {0: 0, 128: R.RDIST_BLOCK_128, 256: R.RDIST_BLOCK_256}[args.block]
    A_np = gg.c2_graph(0)
    A = torch.from_numpy(A_np).cuda()
    D = torch.empty((n, n), dtype=torch.int16, device="cuda")
    ctx = R.Context(0)
    stream = torch.cuda.current_stream()
    info = R.PinnedInfo(1)
    log(f"[bench] c2 n={n}: warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.solve_async(A, -0.5, fl, D, info=info, stream=stream)
    torch.cuda.synchronize()
    st = info.get(0)
    assert st.status == 0, st.as_dict()
    # timed region: events only around the dominant kernel's launches (REST),
    # so that timing disturbs the solve as little as possible
    ctx.set_timing(True, classes=[R.RDIST_K_UPDATE])
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    log(f"[bench] timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        # the REST launches of every fifth solve are timed (a timed launch
        # records two events, which slows the solve by about 0.5%)
        ctx.timing_hold(k % 5 != 0)
        evs[k][0].record(stream)
        ctx.solve_async(A, -0.5, fl, D, info=info, stream=stream)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.timing_hold(False)
    step_ms = [a.elapsed_time(b) for a, b in evs]
    upd = ctx.kernel_stats(R.RDIST_K_UPDATE)
    # per-kernel split from a separate pass with every class timed (not the timed region)
    ctx.set_timing(True)
    nsplit = 3
    for _ in range(nsplit):
        ctx.solve_async(A, -0.5, fl, D, info=info, stream=stream)
    torch.cuda.synchronize()
    edge = ctx.kernel_stats(R.RDIST_K_UPDATE_EDGE)
    panel = ctx.kernel_stats(R.RDIST_K_PANEL)
    rowcol = ctx.kernel_stats(R.RDIST_K_ROWCOL)
    ingest = ctx.kernel_stats(R.RDIST_K_INGEST)
    rest_split = ctx.kernel_stats(R.RDIST_K_UPDATE)
    ctx.set_timing(False)
    # throughput with three independent solves in flight on three streams
    # (each stream has its own workspace); reported beside the value
    conc = None
    streams = [torch.cuda.Stream() for _ in range(3)] if not args.no_concurrent else []
    if streams:
        Dc = [torch.empty((n, n), dtype=torch.int16, device="cuda") for _ in range(3)]
        infc = R.PinnedInfo(3)
        for k in range(3):
            ctx.solve_async(A, -0.5, fl, Dc[k], info=infc, info_index=k, stream=streams[k])
        torch.cuda.synchronize()
        nconc = max(6, 3 * (args.steps // 3))
        t1 = time.perf_counter()
        for k in range(nconc):
            ctx.solve_async(A, -0.5, fl, Dc[k % 3], info=infc, info_index=k % 3, stream=streams[k % 3])
        torch.cuda.synchronize()
        conc_s = (time.perf_counter() - t1) / nconc
        conc = {"streams": 3, "solves": nconc, "graphs_per_s": 1.0 / conc_s,
                "eff_tflops": 2.0 * n ** 3 / conc_s / 1e12,
                "d_equal_single": all(bool(torch.equal(Dc[k], D)) for k in range(3))}
    st = info.get(0).as_dict()
    # next-hop on a kept solve (not part of the step)
    _, g = ctx.solve_async(A, -0.5, fl, D, keep=True, info=info, stream=stream)
    rng = gg.rng_for("bench", 5)
    pairs = torch.from_numpy(rng.integers(0, n, size=(64, 2)).astype(np.int32)).cuda()
    cur, goal = pairs[:, 0].contiguous(), pairs[:, 1].contiguous()
    out_paths = ctx.next_hop(g, cur, goal, max_hops=64, stream=stream)      # warm-up call
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.next_hop(g, cur, goal, max_hops=64, out=out_paths, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    nh_ms = e0.elapsed_time(e1)
    # the readout as its own pass over the kept Y (the unfused epilogue): HBM-bound, 10 B per entry
    import ctypes
    yp, nn, ld = ctypes.c_void_p(), ctypes.c_int32(), ctypes.c_int32()
    R.rdist_graph_y(g.handle, ctypes.byref(yp), ctypes.byref(nn), ctypes.byref(ld))
    D_unf = torch.empty_like(D)
    sp = stream.cuda_stream
    R.rdist_epilogue(ctx.handle, yp, n, ld.value, st["gamma"], D_unf.data_ptr(), info.at(0), sp)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(5):
        R.rdist_epilogue(ctx.handle, yp, n, ld.value, st["gamma"], D_unf.data_ptr(), info.at(0), sp)
    torch.cuda.synchronize()
    ep = ctx.kernel_stats(R.RDIST_K_EPILOGUE)
    ctx.set_timing(False)
    ep_ms = ep["total_ms"] / max(ep["launches"], 1)
    epilogue = {"kernel": "k_epilogue (standalone readout over Y, ld = padded n)", "ms": ep_ms,
                "bytes_per_launch": 10.0 * n * n, "achieved_gbs": 10.0 * n * n / (ep_ms * 1e-3) / 1e9,
                "frac_hbm_peak": 10.0 * n * n / (ep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "d_equals_fused": bool(torch.equal(D_unf, D))}
    g.release()
    mixed = None
    if not args.no_mixed:
        log("[bench] mixed precision on the same graph")
        mixed = measure_mixed(ctx, R, torch, A, D, max(2, args.steps // 3), stream)
        mixed["speed_vs_fp64"] = mixed["graphs_per_s"] / (args.steps / wall)
    ctx.close()

    flops = 2.0 * n ** 3
    ms = wall * 1000.0 / args.steps
    per_launch_flops = upd["flops"] / max(upd["launches"], 1)
    avg_ms = upd["total_ms"] / max(upd["launches"], 1)
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
    sha = source_sha(UPDATE_SOURCES)
    traffic = read_traffic("k_update_c2_n8192_pmc.md", sha)
    mfma_flops = read_mfma_flops("k_update_c2_n8192_pmc.md", sha)
    out = {
        "metric": "APSP graphs/s + eff. TFLOP/s at n=8192 (FP64 vs mixed), p50/p99 latency",
        "value": args.steps / wall,
        "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C2: directed ER(n=8192, p=0.02), gamma=0.5/max_out_degree, FP64 blocked "
                               "Gauss-Jordan on FP64 MFMA + fused int16 D readout",
                   "n": n, "p": 0.02, "gamma": st["gamma"], "delta": st["delta"], "seed": "c2/0",
                   "block": args.block or "auto"},
        "eff_tflops": flops / (ms * 1e-3) / 1e12,
        "frac_fp64_peak_whole_solve": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
        "p50_ms": percentile(step_ms, 50), "p99_ms": percentile(step_ms, 99),
        "roofline": {"bound": "mfma", "kernel": "k_update<kRest> (FP64 MFMA rank-b trailing update, all tiles "
                                                "outside the next block's row and column)",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic, "avg_launch_ms": avg_ms, "launches": upd["launches"],
                     "flops_per_launch": per_launch_flops, "source_sha": sha,
                     "mfma_counter_flops": mfma_flops,
                     "mfma_counter_ratio": mfma_flops / per_launch_flops if mfma_flops else None},
        "kernel_ms_per_step": {k: v["total_ms"] / nsplit for k, v in
                               (("update_rest", rest_split), ("update_edge_and_last", edge), ("panel", panel),
                                ("rowcol", rowcol), ("ingest", ingest))},
        "concurrent": conc,
        "next_hop_64_paths_ms": nh_ms,
        "epilogue_unfused": epilogue,
        "mixed": mixed,
        "solve_info": {k: st[k] for k in ("status", "n_unreachable", "n_subnormal", "n_ambiguous")},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline_c2(A_np, args.cpu_gj_steps, args.cpu_rows)
        out["cpu_floyd_warshall"] = cpu_floyd_warshall_c2(A_np, args.cpu_fw_steps)
    else:
        out["cpu_baseline"] = None
    return out


def bench_c4(args, torch, R, gg):
    """ER(16384, 0.01): the mixed-precision solve (value) against the FP64
    solve of the same graph on the same GPU, D compared entry by entry."""
    import oracle
    n = 16384
    A_np = gg.c4_graph(0)
    A = torch.from_numpy(A_np).cuda()
    D = torch.empty((n, n), dtype=torch.int16, device="cuda")
    ctx = R.Context(0)
    stream = torch.cuda.current_stream()
    info = R.PinnedInfo(1)
    log("[bench] c4 FP64 reference solve")
    ctx.solve_async(A, -0.5, 0, D, info=info, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps64 = max(1, args.steps // 3)
    for _ in range(steps64):
        ctx.solve_async(A, -0.5, 0, D, info=info, stream=stream)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / steps64
    st64 = info.get(0).as_dict()
    log(f"[bench] c4 mixed: {args.steps} steps")
    mixed = measure_mixed(ctx, R, torch, A, D, args.steps, stream)
    ctx.close()
    out = {
        "metric": "mixed-precision APSP graphs/s at n=16384 vs FP64, fallback fraction, D exactness",
        "value": mixed["graphs_per_s"], "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": mixed["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "C4: directed ER(n=16384, p=0.01), gamma=0.5/max_out_degree, FP32 inversion "
                               "(FP64 panels) + certification (margin 0.05, FP32 underflow) + FP64-accurate "
                               "recompute", "n": n, "p": 0.01, "gamma": st64["gamma"], "delta": st64["delta"],
                   "seed": "c4/0"},
        "mixed": mixed,
        "fp64": {"ms_per_solve": ms64, "graphs_per_s": 1e3 / ms64, "eff_tflops": 2.0 * n ** 3 / (ms64 * 1e-3) / 1e12},
        "roofline": {"bound": "mfma", "kernel": "k_gemm32<1> (FP32 MFMA trailing update, rank 256, 128 x 128 tiles)",
                     "achieved": mixed["fp32_gemm_tflops"], "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": mixed["fp32_gemm_frac_of_peak"], "traffic": None},
    }
    if not args.no_cpu:
        sub = gg.c4_subsample(0)
        t0 = time.perf_counter()
        oracle.solve(sub, -0.5, keep_y=False)
        t = time.perf_counter() - t0
        t_full = t * (n / sub.shape[0]) ** 3
        out["cpu_baseline"] = {"value": 1.0 / t_full, "unit": "graphs/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"one n=2048 C4-density solve ({t:.1f} s), scaled by (16384/2048)^3"}
    else:
        out["cpu_baseline"] = None
    return out


def bench_c5(args, torch, R, gg):
    """Serving: Poisson arrivals of full-D and 64-pair path requests on graphs
    with n log-uniform in [64, 4096] (ER or torus lattice, mean degree 6-20),
    through the engine's request loop (continuous batching, HBM-footprint
    admission).  Graphs come from a pool of pre-built graphs resident in HBM
    (request k uses pool entry k mod P); latency runs from the scheduled
    arrival to the poll that reports the result in host memory."""
    pool_n = args.c5_pool
    pool_reqs = gg.c5_requests(pool_n, qps=1.0, stream_index=0)
    log(f"[bench] c5: building a pool of {pool_n} graphs")
    pool = []
    for r in pool_reqs:
        A = r.spec.build()
        n = A.shape[0]
        it = {"A": torch.from_numpy(A).cuda(), "n": n,
              "kind": R.RDIST_QUERY_D if r.query == "D" else R.RDIST_QUERY_PATHS}
        if it["kind"] == R.RDIST_QUERY_D:
            it["D"] = torch.empty((n, n), dtype=torch.int16, pin_memory=True)
        else:
            it["cur"] = torch.from_numpy(r.pairs[:, 0].copy()).pin_memory()
            it["goal"] = torch.from_numpy(r.pairs[:, 1].copy()).pin_memory()
            it["paths"] = torch.empty((len(r.pairs), 65), dtype=torch.int32, pin_memory=True)
        pool.append(it)
    flops_pool = [2.0 * it["n"] ** 3 for it in pool]
    ctx = R.Context(0)
    budget = args.c5_budget_gib << 30

    def run(arrivals):
        """Submits request k at arrivals[k] (seconds from start); returns latencies (s), wall, stats."""
        srv = R.Server(ctx, slots=args.c5_slots, hbm_budget=budget, max_batch=64)
        N = len(arrivals)
        lat = np.zeros(N)
        conc = []
        t0 = time.perf_counter()
        k = 0
        done = 0
        while done < N:
            now = time.perf_counter() - t0
            while k < N and arrivals[k] <= now:
                it = pool[k % pool_n]
                if it["kind"] == R.RDIST_QUERY_D:
                    st = srv.submit(k, it["A"], -0.5, R.RDIST_QUERY_D, D_host=it["D"])
                else:
                    st = srv.submit(k, it["A"], -0.5, R.RDIST_QUERY_PATHS, cur_host=it["cur"], goal_host=it["goal"],
                                    max_hops=64, paths_host=it["paths"])
                assert st == R.RDIST_OK, R.rdist_last_error()
                k += 1
            ids = srv.poll()
            if ids:
                t = time.perf_counter() - t0
                for i in ids:
                    lat[i] = t - arrivals[i]
                done += len(ids)
                conc.append(srv.stats()["in_flight"])
            else:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return lat, wall, st, conc

    # saturated throughput: everything arrives at once
    n_sat = args.c5_sat
    log(f"[bench] c5: saturation run with {n_sat} requests")
    run(np.zeros(min(n_sat, 200)))                    # warm-up (workspaces, kernels)
    lat, wall, st_sat, _ = run(np.zeros(n_sat))
    sat = n_sat / wall
    levels = []
    for frac in [float(x) for x in args.c5_levels.split(",") if x.strip()]:
        qps = frac * sat
        # args.c5_requests per level, fewer at low rates (at most about 10 s of arrivals)
        count = max(1000, min(args.c5_requests, int(qps * 10.0)))
        reqs = gg.c5_requests(count, qps=qps, stream_index=1)
        arrivals = np.array([r.arrival_s for r in reqs])
        log(f"[bench] c5: {count} requests at {qps:.0f} QPS")
        lat, wall, st, conc = run(arrivals)
        fl = sum(flops_pool[k % pool_n] for k in range(len(arrivals)))
        hist = np.bincount(np.asarray(conc, dtype=np.int64), minlength=1).tolist() if conc else []
        levels.append({"qps": qps, "fraction_of_saturated": frac, "requests": len(arrivals),
                       "graphs_per_s": len(arrivals) / wall, "eff_tflops": fl / wall / 1e12,
                       "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                       "mean_ms": float(lat.mean() * 1e3), "batches": st["batches"],
                       "batched_requests": st["batched_requests"], "max_in_flight": st["max_in_flight"],
                       "max_footprint_in_flight_gib": st["max_footprint_in_flight"] / 2 ** 30,
                       "in_flight_histogram": hist})
    ctx.close()
    return {
        "metric": "serving: graphs/s and p50/p99 latency under Poisson arrivals (n in [64, 4096])",
        "value": sat, "unit": "graphs/s", "n_gpus": 1, "steps": n_sat, "warmup": 200,
        "ms_per_step": 1e3 / sat, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "C5: Poisson stream, n log-uniform [64, 4096], ER p=k/(n-1) k~U[6,20] or torus "
                               "lattice (6/8/12/18 neighbours), 50/50 full D or 64 greedy paths, gamma=0.5/Delta; "
                               f"pool of {pool_n} graphs resident in HBM",
                   "slots": args.c5_slots, "hbm_budget_gib": args.c5_budget_gib, "max_batch": 64},
        "saturated": {"graphs_per_s": sat, "requests": n_sat, "batches": st_sat["batches"],
                      "max_in_flight": st_sat["max_in_flight"]},
        "levels": levels,
        "cpu_baseline": None,
    }


def bench_f1(args, torch, R, gg):
    """Positive integer weights (Sec. 3.2): a weighted graph of the C2 shape,
    ER(8192, 0.02) with weights log-uniform in [1, 100] and gamma = 0.5/Delta,
    solved with RDIST_WEIGHTED (value, roofline of the same REST update); and
    the paper's weighted-graph experiment size, n = 1000, p = 0.5, weights
    log-uniform in [1, 100], gamma = 1e-7, beside the oracle on the host."""
    import oracle
    n = 8192
    rng = gg.rng_for("f1", 0)
    W_np = gg.weighted(gg.erdos_renyi(n, 0.02, rng), rng, 1, 100)
    W = torch.from_numpy(W_np).cuda()
    D = torch.empty((n, n), dtype=torch.int16, device="cuda")
    ctx = R.Context(0)
    stream = torch.cuda.current_stream()
    info = R.PinnedInfo(1)
    fl = R.RDIST_WEIGHTED
    for _ in range(args.warmup):
        ctx.solve_async(W, -0.5, fl, D, info=info, stream=stream)
    torch.cuda.synchronize()
    assert info.get(0).status == 0, info.get(0).as_dict()
    ctx.set_timing(True, classes=[R.RDIST_K_UPDATE])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.solve_async(W, -0.5, fl, D, info=info, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd = ctx.kernel_stats(R.RDIST_K_UPDATE)
    ctx.set_timing(False)
    st = info.get(0).as_dict()
    # the paper's weighted experiment size
    n2 = 1000
    rng2 = gg.rng_for("f1", 1)
    W2_np = gg.weighted(gg.erdos_renyi(n2, 0.5, rng2), rng2, 1, 100)
    W2 = torch.from_numpy(W2_np).cuda()
    D2 = torch.empty((n2, n2), dtype=torch.int16, device="cuda")
    for _ in range(3):
        ctx.solve_async(W2, 1e-7, fl, D2, info=info, stream=stream)
    torch.cuda.synchronize()
    reps = 50
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.solve_async(W2, 1e-7, fl, D2, info=info, stream=stream)
    torch.cuda.synchronize()
    ms2 = (time.perf_counter() - t1) * 1e3 / reps
    # accuracy on that graph against Dijkstra (scipy): the correlation of the
    # R-distance log_gamma Y with the weighted distance, D's exact fraction,
    # the fraction of (node, goal) pairs whose greedy successor is the one
    # greedy descent on the true distances picks (Eq. descent: a successor
    # nearest the goal; the paper reports all 1 million correct below 1e-8),
    # and the fraction whose successor also lies on a shortest path (descent
    # ignores the weight of the step itself)
    import scipy.sparse.csgraph as csg
    dist2 = csg.shortest_path(np.ascontiguousarray(W2_np.T, dtype=np.float64), directed=True).T
    reach = np.isfinite(dist2)
    np.fill_diagonal(reach, False)
    pairs = np.argwhere(reach)                            # [goal, cur]
    # the true-distance descent's choice value: min over successors j of cur of dist(j -> goal)
    best_true = np.full((n2, n2), np.inf)
    for c in range(n2):
        succ = np.nonzero(W2_np[:, c])[0]
        if len(succ):
            best_true[:, c] = dist2[:, succ].min(axis=1)
    accuracy = []
    for gam in (1e-5, 1e-7, 1e-9):
        Dg, inf_g, gr = ctx.solve(W2, gam, flags=fl, keep=True)
        Yh = gr.y().cpu().numpy()
        hop = ctx.next_hop(gr, torch.from_numpy(pairs[:, 1].astype(np.int32)),
                           torch.from_numpy(pairs[:, 0].astype(np.int32)), 1).cpu().numpy()
        gr.release()
        R = np.log(Yh[reach]) / np.log(gam)
        r2 = float(np.corrcoef(R, dist2[reach])[0, 1] ** 2)
        exact = float(np.mean(Dg.cpu().numpy()[reach] == dist2[reach].astype(np.int64)))
        g_, c_ = pairs[:, 0], pairs[:, 1]
        j_ = np.maximum(hop, 0)
        ok = (hop >= 0) & (W2_np[j_, c_] > 0) & (dist2[g_, j_] == best_true[g_, c_])
        sp = (hop >= 0) & (W2_np[j_, c_] > 0) & (W2_np[j_, c_] + dist2[g_, j_] == dist2[g_, c_])
        accuracy.append({"gamma": gam, "r2": r2, "d_exact": exact, "local": float(ok.mean()),
                         "local_wrong": int((~ok).sum()), "on_shortest_path": float(sp.mean()),
                         "pairs": int(len(ok))})
    ctx.close()
    ms = wall * 1e3 / args.steps
    per_launch_flops = upd["flops"] / max(upd["launches"], 1)
    avg_ms = upd["total_ms"] / max(upd["launches"], 1)
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
    sha = source_sha(UPDATE_SOURCES)
    out = {
        "metric": "weighted APSP (integer weights) graphs/s at n=8192",
        "value": args.steps / wall, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "f1: directed ER(n=8192, p=0.02), integer weights log-uniform in [1, 100], "
                               "gamma=0.5/Delta, FP64 blocked Gauss-Jordan of I - gamma^W + fused readout",
                   "n": n, "gamma": st["gamma"], "delta": st["delta"]},
        "eff_tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12,
        "roofline": {"bound": "mfma", "kernel": "k_update<kRest> (as C2)", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": read_traffic("k_update_c2_n8192_pmc.md", sha), "avg_launch_ms": avg_ms,
                     "launches": upd["launches"], "flops_per_launch": per_launch_flops, "source_sha": sha},
        "paper_size": {"n": n2, "p": 0.5, "gamma": 1e-7, "ms_per_solve": ms2, "graphs_per_s": 1e3 / ms2,
                       "accuracy": accuracy},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle, n = 1000 weighted solve)")
        t2 = time.perf_counter()
        sol = oracle.solve_weighted(W2_np, 1e-7, keep_y=False)
        tc = time.perf_counter() - t2
        assert np.array_equal(sol.D, D2.cpu().numpy()), "paper-size weighted D differs from the oracle"
        out["cpu_baseline"] = {"value": 1.0 / tc, "unit": "graphs/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"one full n = {n2} weighted solve ({tc:.3f} s)"}
    else:
        out["cpu_baseline"] = None
    return out


DYNAMIC_SOURCES = ["paper_2308_07403_amd/csrc/rd_dynamic.hip", "paper_2308_07403_amd/csrc/rd_device.h"]


def plan_changes(rng, A, delta_cap, count):
    """`count` edge changes applied to A in place, alternating removals of
    existing edges and additions that keep every out-degree <= delta_cap."""
    n = A.shape[0]
    outdeg = (A != 0).sum(axis=0).astype(np.int64)
    out = []
    for k in range(count):
        if k % 2 == 0:
            while True:
                src, dst = map(int, rng.integers(0, n, size=2))
                if src != dst and A[dst, src]:
                    break
            A[dst, src] = 0
            outdeg[src] -= 1
            out.append((src, dst, 0))
        else:
            while True:
                src, dst = map(int, rng.integers(0, n, size=2))
                if src != dst and not A[dst, src] and outdeg[src] < delta_cap:
                    break
            A[dst, src] = 1
            outdeg[src] += 1
            out.append((src, dst, 1))
    return out


def bench_f3(args, torch, R, gg):
    """Edge changes on a kept graph (rank-one update of Y, the dynamic
    re-planning use of the Discussion): the C2 graph, ER(8192, 0.02) at
    gamma = 0.5/Delta, solved once with KEEP_Y; one step = 32 changes
    (alternating removals and additions), each rewriting Y, its error bounds
    and D in one pass.  Re-inversions the bounds call for are inside the
    timed region and counted."""
    n, per_step = 8192, 32
    rng = gg.rng_for("f3", 0)
    A_np = gg.erdos_renyi(n, 0.02, rng)
    A = torch.from_numpy(A_np).cuda()
    D = torch.empty((n, n), dtype=torch.int16, device="cuda")
    ctx = R.Context(0)
    stream = torch.cuda.current_stream()
    D0, info, g = ctx.solve(A, -0.5, keep=True)
    assert info["status"] == 0
    gamma, delta = info["gamma"], info["delta"]
    # a full re-solve of the same graph on the GPU, for comparison
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.solve_async(A, -0.5, 0, D, stream=stream)
    torch.cuda.synchronize()
    resolve_ms = (time.perf_counter() - t0) * 1e3 / reps
    A_host = A_np.copy()
    warm = plan_changes(rng, A_host, delta, args.warmup * per_step)
    timed = plan_changes(rng, A_host, delta, args.steps * per_step)
    for src, dst, w in warm:
        g.update_edge(src, dst, w, D=D)
    torch.cuda.synchronize()
    ctx.set_timing(True, classes=[R.RDIST_K_EDGE_UPDATE])
    lost = refreshed = 0
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (src, dst, w) in enumerate(timed):
        ctx.timing_hold(k % 5 != 0)          # every fifth change's apply pass is timed
        t1 = time.perf_counter()
        inf = g.update_edge(src, dst, w, D=D)
        lat.append((time.perf_counter() - t1) * 1e3)
        lost += inf["n_uncertified"]
        refreshed += inf["fallback_fraction"] == 1.0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.kernel_stats(R.RDIST_K_EDGE_UPDATE)
    ctx.timing_hold(False)
    ctx.set_timing(False)
    assert inf["status"] == 0, inf
    # the same kind of changes in batches: one call per step of 32 (4 passes of 8)
    batches = [plan_changes(rng, A_host, delta, per_step) for _ in range(args.steps + 1)]
    g.update_edges(batches[0], D=D)
    torch.cuda.synchronize()
    ctx.set_timing(True, classes=[R.RDIST_K_EDGE_UPDATE])
    t0 = time.perf_counter()
    for b in batches[1:]:
        binf = g.update_edges(b, D=D)
        lost += binf["n_uncertified"]
        refreshed += binf["fallback_fraction"] == 1.0
    torch.cuda.synchronize()
    bwall = time.perf_counter() - t0
    bst = ctx.kernel_stats(R.RDIST_K_EDGE_UPDATE)
    ctx.set_timing(False)
    assert binf["status"] == 0, binf
    g.release()
    ctx.close()
    nch = len(timed)
    per_launch_bytes = 22.0 * n * n
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    sha = source_sha(DYNAMIC_SOURCES)
    out = {
        "metric": "edge changes/s on a kept n=8192 graph (Y and D rewritten per change)",
        "value": nch / wall, "unit": "changes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "f3: directed ER(n=8192, p=0.02), gamma=0.5/Delta, kept Y; one step = 32 edge "
                               "changes (alternating removals and additions), each a rank-one update of Y with "
                               "its error bounds and the int16 D readout in the same pass",
                   "n": n, "gamma": gamma, "delta": delta, "changes_per_step": per_step},
        "ms_per_change": wall * 1e3 / nch, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
        "resolve_ms": resolve_ms, "speedup_vs_resolve": resolve_ms / (wall * 1e3 / nch),
        "lost_entries": int(lost), "reinversions": int(refreshed),
        "batched": {"changes_per_s": per_step * args.steps / bwall, "ms_per_step": bwall * 1e3 / args.steps,
                    "passes_per_step": (per_step + 7) // 8,
                    "apply_ms": bst["total_ms"] / max(bst["launches"], 1),
                    "apply_gbs": 22.0 * n * n / (bst["total_ms"] / max(bst["launches"], 1) * 1e-3) / 1e9},
        "roofline": {"bound": "hbm", "kernel": "k_sm_apply<4>", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic("k_sm_apply_f3_n8192_pmc.md", sha), "avg_launch_ms": avg_ms,
                     "launches": st["launches"], "bytes_per_launch": per_launch_bytes, "source_sha": sha},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle re-solve of the changed graph, sampled)")
        cb = cpu_baseline_c2(A_host, args.cpu_gj_steps, args.cpu_rows)
        cb["unit"] = "changes/s"
        cb["sample"] = "one oracle re-solve per change; " + cb["sample"]
        out["cpu_baseline"] = cb
    else:
        out["cpu_baseline"] = None
    return out


ROWS_SOURCES = ["paper_2308_07403_amd/csrc/rd_rows.hip", "paper_2308_07403_amd/csrc/rd_device.h"]


def bench_f4(args, torch, R, gg):
    """Goal rows without an inversion (the network's fixed point, Sec. 2): a
    1024 x 1024 lattice with 10% of its directed edges deleted (n = 1048576,
    successor lists), gamma = 0.5/Delta; one step = the rows (and D rows) of
    64 random goals.  Beside it: 64 goal rows of the C2 graph against one
    full C2 solve."""
    import oracle
    n = 1024 * 1024
    rng = gg.rng_for("f4", 0)
    ptr_np, idx_np = gg.grid_lattice_csr(n, rng)
    ptr, idx = torch.from_numpy(ptr_np).cuda(), torch.from_numpy(idx_np).cuda()
    goal_sets = [torch.from_numpy(rng.integers(0, n, size=64).astype(np.int32)) for _ in range(args.warmup + args.steps)]
    ctx = R.Context(0)
    for k in range(args.warmup):
        ctx.goal_rows(ptr, idx, goal_sets[k], -0.5)
    torch.cuda.synchronize()
    ctx.set_timing(True, classes=[R.RDIST_K_ROWS_STEP])
    steps_run = []
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        # the first timed call's steps are timed (eager launches with events);
        # the others replay the captured chunk, as an untimed caller's would
        ctx.timing_hold(k != args.warmup)
        Y, D, info, steps = ctx.goal_rows(ptr, idx, goal_sets[k], -0.5)
        steps_run.append(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.kernel_stats(R.RDIST_K_ROWS_STEP)
    ctx.timing_hold(False)
    ctx.set_timing(False)
    assert info["status"] == 0, info
    gamma, delta = info["gamma"], info["delta"]
    del Y, D
    # one goal at a time on the same lattice (latency of a single row)
    one = []
    for k in range(3):
        t1 = time.perf_counter()
        _, _, inf1, steps1 = ctx.goal_rows(ptr, idx, goal_sets[k % len(goal_sets)][:1], -0.5)
        one.append((time.perf_counter() - t1) * 1e3)
    # the C2 graph: 64 goal rows against the full solve
    A_np = gg.erdos_renyi(8192, 0.02, gg.rng_for("f4", 1))
    p2, i2, _ = gg.csr_from_dense(A_np)
    p2t, i2t = torch.from_numpy(p2).cuda(), torch.from_numpy(i2).cuda()
    g2 = torch.from_numpy(np.arange(0, 8192, 128, dtype=np.int32))
    ctx.goal_rows(p2t, i2t, g2, -0.5)
    reps = 5
    t1 = time.perf_counter()
    for _ in range(reps):
        _, _, inf2, steps2 = ctx.goal_rows(p2t, i2t, g2, -0.5)
    torch.cuda.synchronize()
    c2_rows_ms = (time.perf_counter() - t1) * 1e3 / reps
    A2 = torch.from_numpy(A_np).cuda()
    D2 = torch.empty((8192, 8192), dtype=torch.int16, device="cuda")
    ctx.solve_async(A2, -0.5, 0, D2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.solve_async(A2, -0.5, 0, D2)
    torch.cuda.synchronize()
    c2_solve_ms = (time.perf_counter() - t1) * 1e3 / reps
    ctx.close()
    q = 64
    nnz = int(idx_np.shape[0])
    per_launch_bytes = 2.0 * n * q * 8 + 8.0 * (n + 1) + 4.0 * nnz
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    sha = source_sha(ROWS_SOURCES)
    out = {
        "metric": "goal rows/s on a 1M-node lattice (no inversion)", "value": q * args.steps / wall,
        "unit": "rows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "f4: 1024x1024 4-neighbour lattice, 10% of directed edges deleted (n=1048576), "
                               "gamma=0.5/Delta, successor lists; one step = Y and D rows of 64 random goals by "
                               "the fixed-point iteration",
                   "n": n, "nnz": nnz, "gamma": gamma, "delta": delta, "goals_per_step": q},
        "iterations_per_step": float(np.mean(steps_run)),
        "roofline": {"bound": "hbm", "kernel": "k_rows_step64<16>", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic("k_rows_step_f4_lattice1m_pmc.md", sha), "avg_launch_ms": avg_ms,
                     "launches": st["launches"], "bytes_per_launch": per_launch_bytes, "source_sha": sha},
        "c2_graph": {"rows": 64, "ms": c2_rows_ms, "iterations": steps2, "full_solve_ms": c2_solve_ms},
        "single_goal": {"ms": float(np.median(one)), "iterations": steps1},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle series row on the lattice)")
        t2 = time.perf_counter()
        oracle.y_row_csr(ptr_np, idx_np, gamma, int(goal_sets[-1][0]))
        tc = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": 1.0 / tc, "unit": "rows/s", "cores": 1, "kind": "oracle",
                               "sample": f"one goal row of the same lattice by the oracle's series ({tc:.1f} s)"}
    else:
        out["cpu_baseline"] = None
    return out


def bfs_distances(A: np.ndarray) -> np.ndarray:
    """Graph distances by scipy's breadth-first search: [i, j] = hops from j to i
    (A[i, j] = 1 for an edge j -> i), -1 where unreachable; the sweep's ground truth."""
    import scipy.sparse.csgraph as csg
    d = csg.shortest_path(np.ascontiguousarray(A.T, dtype=np.float64), unweighted=True, directed=True).T
    return np.where(np.isinf(d), -1, d).astype(np.int64)


GAMMA_SOURCES = ["paper_2308_07403_amd/csrc/rd_gamma.hip", "paper_2308_07403_amd/csrc/rd_device.h"]


def bench_f2(args, torch, R, gg):
    """Gain selection and the per-entry certificate (Sec. 4.1, 4.2, 5.1):
    the certificate pass and the spectral-radius bracket on the C2 graph
    (value: certified-entry checks per second), and the accuracy sweep of the
    paper's Fig. 2 families (Towers of Hanoi, square grid, binary tree, dense
    random p = 0.5, preferential attachment): global, local and certified
    fractions against BFS over gains up to the gate gamma Delta < 1."""
    import oracle
    n = 8192
    A_np = gg.erdos_renyi(n, 0.02, gg.rng_for("f2", 0))
    A = torch.from_numpy(A_np).cuda()
    ctx = R.Context(0)
    D, info, g = ctx.solve(A, -0.5, keep=True)
    t0 = time.perf_counter()
    gb = ctx.gain_bounds(A)
    gain_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(args.warmup):
        ctx.certify(g)
    ctx.set_timing(True, classes=[R.RDIST_K_CERTIFY])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnt, _ = ctx.certify(g)
    wall = time.perf_counter() - t0
    st = ctx.kernel_stats(R.RDIST_K_CERTIFY)
    ctx.set_timing(False)
    g.release()
    # the accuracy sweep
    rng = gg.rng_for("f2", 1)
    fams = [("hanoi", 5, gg.hanoi(5)), ("hanoi", 6, gg.hanoi(6)), ("grid", 10, gg.square_grid(10)),
            ("grid", 20, gg.square_grid(20)), ("binary_tree", 7, gg.binary_tree(7)),
            ("binary_tree", 9, gg.binary_tree(9)), ("dense_p0.5", 100, gg.erdos_renyi(100, 0.5, rng)),
            ("dense_p0.5", 400, gg.erdos_renyi(400, 0.5, rng)),
            ("power_law", 200, gg.barabasi_albert(200, 2, rng)), ("power_law", 800, gg.barabasi_albert(800, 2, rng))]
    fracs = [1e-6, 1e-5, 1e-4, 1e-3, 0.01, 0.03, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99]
    sweep = []
    for fam, size, G_np in fams:
        m = G_np.shape[0]
        dist = bfs_distances(G_np)
        G = torch.from_numpy(G_np).cuda()
        r = ctx.gain_bounds(G, diameter=int(dist.max()))
        delta = r["delta"]
        pairs = np.argwhere(dist > 0)                     # [goal, cur] with the goal reachable from cur
        goal_t = torch.from_numpy(pairs[:, 0].astype(np.int32))
        cur_t = torch.from_numpy(pairs[:, 1].astype(np.int32))
        pts = []
        for f in fracs:
            gamma = f / delta
            Dg, inf, gr = ctx.solve(G, gamma, keep=True)
            c, _ = ctx.certify(gr)
            hop = ctx.next_hop(gr, cur_t, goal_t, 1).cpu().numpy()
            gr.release()
            Dh = Dg.cpu().numpy()
            ok = np.where(dist >= 0, Dh == dist, Dh == R.RDIST_UNREACHABLE)
            np.fill_diagonal(ok, False)
            good = (hop >= 0) & (dist[pairs[:, 0], np.maximum(hop, 0)] == dist[pairs[:, 0], pairs[:, 1]] - 1)
            pts.append({"gamma": gamma, "gamma_delta": f, "global": float(ok.sum()) / (m * (m - 1)),
                        "local": float(good.mean()) if len(good) else 1.0, "certified": c / (m * m)})
        sweep.append({"family": fam, "size": size, "n": m, "delta": delta, "diameter": int(dist.max()),
                      "rho": [r["rho_lo"], r["rho_hi"]], "gamma_c_lo": r["gamma_c_lo"],
                      "gamma_global": r["gamma_global"], "gamma_precision": r["gamma_precision"], "points": pts})
        log(f"[bench] sweep {fam} n={m}: global {[round(p['global'], 3) for p in pts]}")
    ctx.close()
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    per_launch_bytes = 8.0 * n * n
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    sha = source_sha(GAMMA_SOURCES)
    out = {
        "metric": "certified-entry checks/s on a kept n=8192 graph", "value": args.steps * n * n / wall,
        "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "f2: per-entry certificate of D on the kept C2 graph (ER(8192, 0.02), "
                               "gamma = 0.5/Delta) and the spectral-radius bracket; plus the Fig. 2 accuracy sweep",
                   "n": n, "gamma": info["gamma"], "delta": info["delta"]},
        "certified_fraction": cnt / (n * n),
        "gain_bounds": {"ms": gain_ms, "rho": [gb["rho_lo"], gb["rho_hi"]], "steps": gb["steps"],
                        "gamma_c_lo": gb["gamma_c_lo"], "gamma_gate": gb["gamma_gate"]},
        "roofline": {"bound": "hbm", "kernel": "k_certify", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic("k_certify_f2_n8192_pmc.md", sha), "avg_launch_ms": avg_ms,
                     "launches": st["launches"], "bytes_per_launch": per_launch_bytes, "source_sha": sha},
        "sweep": sweep,
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle certificate on a 2048 x 2048 sample)")
        m = 2048
        rs = np.random.default_rng(7)
        Ys = np.exp(rs.uniform(-40.0, 0.0, size=(m, m)))
        Ds = oracle.readout(Ys, info["gamma"]).D
        t2 = time.perf_counter()
        oracle.certify(Ys, Ds, info["gamma"], info["delta"])
        tc = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": m * m / tc, "unit": "entries/s", "cores": 1, "kind": "oracle",
                               "sample": f"oracle.certify on a synthetic {m}x{m} Y ({tc:.2f} s)"}
    else:
        out["cpu_baseline"] = None
    return out


def bench_c1(args, torch, R, gg):
    import oracle
    As = [torch.from_numpy(gg.c1_graph(s)).cuda() for s in range(100)]
    D = torch.empty((64, 64), dtype=torch.int16, device="cuda")
    ctx = R.Context(0)
    stream = torch.cuda.current_stream()
    info = R.PinnedInfo(1)
    for A in As[: args.warmup * 10 + 1]:
        ctx.solve_async(A, gg.C1_GAMMA, 0, D, info=info, stream=stream)
    torch.cuda.synchronize()
    lat = []
    for k in range(args.steps * 10):
        t0 = time.perf_counter()
        ctx.solve_async(As[k % 100], gg.C1_GAMMA, 0, D, info=info, stream=stream)
        stream.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    # the floor of that round trip: one minimal kernel launch and the same synchronisation
    z = torch.zeros(1, device="cuda")
    for _ in range(20):
        z.add_(1.0)
    stream.synchronize()
    lat0 = []
    for k in range(args.steps * 10):
        t0 = time.perf_counter()
        z.add_(1.0)
        stream.synchronize()
        lat0.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = args.steps * 100
    for k in range(reps):
        ctx.solve_async(As[k % 100], gg.C1_GAMMA, 0, D, info=info, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    A0 = gg.c1_graph(0)
    t0 = time.perf_counter()
    for _ in range(200):
        oracle.solve(A0, gg.C1_GAMMA, keep_y=False)
    tc = (time.perf_counter() - t0) / 200
    return {"metric": "C1 single-solve latency and back-to-back graphs/s (n=64)", "value": reps / wall,
            "unit": "graphs/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / reps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "C1: ER(64, 0.1), gamma=0.05, 100 seeds"},
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "empty_kernel_round_trip": {"p50_ms": percentile(lat0, 50), "p99_ms": percentile(lat0, 99),
                                        "what": "one one-element torch add kernel + stream synchronise"},
            "cpu_baseline": {"value": 1.0 / tc, "unit": "graphs/s", "cores": oracle.num_threads(),
                             "kind": "oracle", "sample": "200 solves of the seed-0 graph"}}


def bench_c3(args, torch, R, gg):
    """1024 small graphs (n log-uniform in [32, 512], ER / lattice / RGG) per
    step, solved by one persistent batched launch."""
    import oracle
    specs = gg.c3_specs(1024, batch_index=0)
    A_np = [s.build() for s in specs]
    As = [torch.from_numpy(A).cuda() for A in A_np]
    Ds = [torch.empty((a.shape[0],) * 2, dtype=torch.int16, device="cuda") for a in As]
    ns = np.array([a.shape[0] for a in A_np], dtype=np.float64)
    flops = float(np.sum(2.0 * ns ** 3))
    import tempfile
    tile_cache = os.path.join(tempfile.mkdtemp(prefix="rdist_"), "tiles.json")
    ctx = R.Context(0, tile_cache=tile_cache)
    stream = torch.cuda.current_stream()
    info = R.PinnedInfo(len(As))
    batch = R.Batch(As, -0.5, Ds)
    log(f"[bench] c3 {len(As)} graphs: autotune + warmup {args.warmup}")
    t0 = time.perf_counter()
    ctx.solve_batched(batch, info=info, stream=stream)        # tunes, then builds and captures the plan
    tune_s = time.perf_counter() - t0
    tuned = json.load(open(tile_cache))["batched"]
    for _ in range(args.warmup):
        ctx.solve_batched(batch, info=info, stream=stream, sync=False)
    torch.cuda.synchronize()
    bad = [k for k in range(len(As)) if info.get(k).status != 0]
    assert not bad, f"graphs {bad[:5]} refused"
    ctx.set_timing(True, classes=[R.RDIST_K_BATCHED])
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    log(f"[bench] timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        ctx.solve_batched(batch, info=info, stream=stream, sync=False)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in evs]
    bk = ctx.kernel_stats(R.RDIST_K_BATCHED)
    ctx.set_timing(False)
    # eager launches of the same plan (no HIP graph), for comparison
    for _ in range(2):
        ctx.solve_batched(batch, flags=R.RDIST_NO_GRAPH, info=info, stream=stream, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.solve_batched(batch, flags=R.RDIST_NO_GRAPH, info=info, stream=stream, sync=False)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    # the dominant kernel, k_lv_update: every launch of it in eager runs of
    # the plan timed with HIP events on its stream (a captured graph cannot
    # hold per-launch events); flops per launch = its product tiles x
    # 2 * 128^2 * inner dimension
    ctx.set_timing(True, classes=[R.RDIST_K_UPDATE, R.RDIST_K_UPDATE_EDGE])
    for _ in range(args.steps):
        ctx.solve_batched(batch, flags=R.RDIST_NO_GRAPH, info=info, stream=stream, sync=False)
    torch.cuda.synchronize()
    ku, ke = ctx.kernel_stats(R.RDIST_K_UPDATE), ctx.kernel_stats(R.RDIST_K_UPDATE_EDGE)
    ctx.set_timing(False)
    ctx.close()
    ms = wall * 1000.0 / args.steps
    avg_ms = bk["total_ms"] / max(bk["launches"], 1)
    upd_launches = ku["launches"] + ke["launches"]
    upd_ms = ku["total_ms"] + ke["total_ms"]
    upd_flops = ku["flops"] + ke["flops"]
    achieved = upd_flops / (upd_ms * 1e-3) / 1e12 if upd_ms > 0 else None
    out = {
        "metric": "batched small-graph APSP graphs/s (1024 graphs, n in [32, 512])",
        "value": len(As) * args.steps / wall, "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "C3: 1024 graphs per step, n log-uniform in [32, 512], ER(p~U[0.05,0.2]) / "
                               "2-D grid lattice with 10% of directed edges deleted / RGG (mean degree 8), "
                               "gamma=0.5/max_out_degree, one captured plan",
                   "graphs": len(As), "sum_n3": float(np.sum(ns ** 3)), "tuning": tuned[0],
                   "autotune_s": tune_s},
        "eager_ms_per_step": eager_ms,
        "eff_tflops": flops / (ms * 1e-3) / 1e12,
        "p50_ms": percentile(step_ms, 50), "p99_ms": percentile(step_ms, 99),
        "plan_ms_events": avg_ms,
        "roofline": {"bound": "mfma",
                     "kernel": "k_lv_update (level plan: diagonal, edge and rest tiles; eager runs of the plan)",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS if achieved else None, "traffic": None,
                     "avg_launch_ms": upd_ms / max(upd_launches, 1), "launches": upd_launches,
                     "flops_per_launch": upd_flops / max(upd_launches, 1)},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle sample)")
        idx = list(range(0, len(A_np), 16))
        t0 = time.perf_counter()
        for k in idx:
            oracle.solve(A_np[k], -0.5, keep_y=False)
        t = time.perf_counter() - t0
        frac = float(np.sum(ns[idx] ** 3) / np.sum(ns ** 3))
        out["cpu_baseline"] = {"value": len(A_np) / (t / frac), "unit": "graphs/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{len(idx)} of the 1024 graphs (every 16th), scaled by their share "
                                         f"of sum n^3 ({frac:.3f}); {t:.1f} s sampled"}
    else:
        out["cpu_baseline"] = None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c2", "c1", "c3", "c4", "c5", "f1", "f2", "f3", "f4"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baselines")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="C2: skip the three-stream throughput (profiling runs, one solve at a time)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--block", type=int, default=0, choices=[0, 128, 256],
                    help="force the blocked plan's block width (0: the engine's choice)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--c5-pool", type=int, default=96, help="C5: distinct graphs in the pool")
    ap.add_argument("--c5-requests", type=int, default=20000, help="C5: requests per QPS level")
    ap.add_argument("--c5-sat", type=int, default=3000, help="C5: requests of the saturation run")
    ap.add_argument("--c5-slots", type=int, default=2)
    ap.add_argument("--c5-budget-gib", type=int, default=16)
    ap.add_argument("--c5-levels", default="0.1,0.5,0.8",
                    help="C5: Poisson rates as fractions of the saturated rate (comma list; empty for none)")
    ap.add_argument("--cpu-gj-steps", type=int, default=256)
    ap.add_argument("--cpu-rows", type=int, default=2048)
    ap.add_argument("--cpu-fw-steps", type=int, default=128)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this engine runs on one GPU; multi-GPU runs are not supported "
              "(independent graphs would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    import graphgen as gg
    from paper_2308_07403_amd import rdist as R
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        # reference for the HBM byte counters: a plain device copy of a known size
        # whose source was pushed out of the caches by a larger scrub write first
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        scrub = torch.empty(nb // 16, dtype=torch.float64, device="cuda")
        scrub.fill_(2.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calibrate_copy} MiB done")
        del src, dst, scrub
    out = {"c2": bench_c2, "c1": bench_c1, "c3": bench_c3, "c4": bench_c4, "c5": bench_c5,
           "f1": bench_f1, "f2": bench_f2, "f3": bench_f3, "f4": bench_f4}[args.workload](args, torch, R, gg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
