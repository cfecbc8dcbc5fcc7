#!/usr/bin/env python3
"""Benchmark of the MI355X Cartesian form-factor engine.

One step = the whole hot path for one molecule and its transitions, from
inputs resident in HBM to f and |f|^2 in HBM:
  load the molecule (geometry + basis: a few KB of host arrays), take the
  transition density matrices from device memory, run the device pair
  precompute / screening / packing, build the 1D V-tables and run the fused
  generator + MFMA contraction over the whole q-grid.

Prints one JSON line.  `value` is q-points x transitions per second of the
whole step on one GPU.  `roofline` describes the fused grid kernel (timed with
HIP events on its stream inside the timed region); `cpu_baseline` times the
FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12   # MI355X FP32 vector (published; counts packed FP32)
PEAK_FP32_MFMA = 157.3e12     # MI355X FP32 matrix
PEAK_BF16_MFMA = 2.5166e15    # MI355X BF16 matrix, dense
PEAK_HBM = 8.0e12


def kernel_source_hash() -> str:
    """Hash of the kernel source with comments and blank lines dropped (a
    comment edit does not invalidate measured counters; a code edit does)."""
    import re
    h = hashlib.sha256()
    for name in ("kernels.hip", "engine.h"):
        with open(os.path.join(ROOT, "paper_2512_18010_amd", "csrc", name)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update("\n".join(l.rstrip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "grid_kernel_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload_key}/{precision}")
    if not e or e.get("kernel_sha") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(W, seconds: float, threads: int):
    import oracle
    pts_all = W.grid.points()
    rng = np.random.Generator(np.random.PCG64(77))
    # calibrate on a small batch, then time a sample of about `seconds`
    probe = pts_all[rng.choice(len(pts_all), size=max(threads, 8), replace=False)]
    t0 = time.perf_counter()
    oracle.eval_points(W.mol, W.T, probe, n_threads=threads)
    per_pt = (time.perf_counter() - t0) / len(probe)
    n = int(max(threads, min(len(pts_all), seconds / max(per_pt, 1e-9))))
    n = (n // threads) * threads or threads
    sample = pts_all[rng.choice(len(pts_all), size=n, replace=False)]
    t0 = time.perf_counter()
    oracle.eval_points(W.mol, W.T, sample, n_threads=threads)
    dt = time.perf_counter() - t0
    ns = W.T.shape[0]
    return {"value": n * ns / dt, "unit": "q-points*transitions/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} seeded grid points of the benchmark workload x {ns} transitions, "
                      f"FP64 direct sum, {dt:.1f} s"}


def serving_benchmark(precision: str, n_pool: int, n_sat: int, n_per_rate: int, n_warm: int,
                      max_inflight: int, budget_gb: float, screen_eps: float, log=None):
    """Request serving: a seeded pool of mixed requests (2-30 heavy atoms,
    1-24 transitions, N^3 grids with N in 32..96, q_max in [5, 8]).
    1. saturated rate mu: closed loop, 2 * max_inflight requests outstanding;
    2. open-loop Poisson arrivals at 0.5, 0.8 and 0.95 mu.
    Latency = result in host memory - submission (the server's steady clock);
    each arrival draws a request from the pool.  The device time of each pool
    request evaluated alone (precompute + 1D tables + grid kernel, HIP events)
    gives the rate the device could sustain without overlap, 1 / mean."""
    import threading
    import torch
    import workload as wl
    from paper_2512_18010_amd import binding

    rng = np.random.Generator(np.random.PCG64(5000))
    pool = [wl.make_serving_request(rng) for _ in range(n_pool)]
    qt = [w.T.shape[0] * w.grid.n_points for w in pool]

    def device_ms_alone(w):
        with binding.Context(0) as ctx:
            ctx.set_timing(True)
            ctx.load_molecule(w.mol)
            ctx.set_options(screen_eps, 1.0)
            shape = (w.T.shape[0],) + tuple(w.grid.n)
            f = torch.empty(shape + (2,), dtype=torch.float32, device="cuda")
            f2 = torch.empty(shape, dtype=torch.float32, device="cuda")
            ms = 0.0
            for _ in range(2):   # the first call allocates; the second is timed
                ctx.load_transitions(w.T)   # the precompute runs again
                ctx.eval_grid_device(w.grid, f, f2, precision=precision)
                torch.cuda.synchronize()
                ms = sum(ctx.last_timing())
            return ms

    alone = [device_ms_alone(w) for w in pool]
    srv = binding.Server(0, int(budget_gb * (1 << 30)), max_inflight)

    def submit(i):
        w = pool[i]
        return srv.submit(w.mol, w.T, w.grid, precision=precision, screen_eps=screen_eps)

    def run_closed(n, seed):
        pick = np.random.Generator(np.random.PCG64(seed)).integers(0, n_pool, size=n)
        out, lat, pending = [], [], []
        t0 = time.perf_counter()
        k = 0
        while k < n or pending:
            while k < n and len(pending) < 2 * max_inflight:
                pending.append((submit(pick[k]), pick[k]))
                k += 1
            t, i = pending.pop(0)
            st, ns, _, _ = srv.wait(t)
            if st != 0:
                raise RuntimeError(f"serving request failed with status {st}")
            lat.append(ns * 1e-6)
            out.append(i)
        dt = time.perf_counter() - t0
        return dt, lat, out

    names = ("wait_prep", "prep", "wait_run", "run", "copy")

    def stage_means(a, b):
        """mean time per request in each server stage between two stats snapshots (ms)"""
        n = max(b["completed"] - a["completed"], 1)
        return {k: (b["ns_stage"][i] - a["ns_stage"][i]) * 1e-6 / n for i, k in enumerate(names)}

    run_closed(n_warm, 4999)
    st_sat = srv.stats()
    dt, lat, done = run_closed(n_sat, 5100)
    mu = n_sat / dt
    res = {"precision": precision, "screen_eps": screen_eps, "pool": n_pool, "max_inflight": max_inflight,
           "budget_gb": budget_gb,
           "device_ms_alone": {"mean": float(np.mean(alone)), "min": float(np.min(alone)),
                               "max": float(np.max(alone)), "bound_req_per_s": 1000.0 / float(np.mean(alone))},
           "saturated": {"requests": n_sat, "req_per_s": mu, "q_t_per_s": sum(qt[i] for i in done) / dt,
                         "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                         "stage_ms_mean": stage_means(st_sat, srv.stats())},
           "rates": []}
    if log:
        log(f"serving {precision}: saturated {mu:.2f} req/s (device time alone {np.mean(alone):.2f} ms "
            f"per request on average -> {1000.0 / np.mean(alone):.1f} req/s without overlap)")
    for ri, frac in enumerate((0.5, 0.8, 0.95)):
        st0 = srv.stats()
        lam = frac * mu
        g = np.random.Generator(np.random.PCG64(5000 + ri + 1))
        arrivals = np.cumsum(g.exponential(1.0 / lam, size=n_per_rate))
        pick = g.integers(0, n_pool, size=n_per_rate)
        tickets = [None] * n_per_rate
        ready = threading.Semaphore(0)
        late = [0.0]

        def producer():
            t0 = time.perf_counter()
            for j in range(n_per_rate):
                d = arrivals[j] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                else:
                    late[0] = max(late[0], -d)
                tickets[j] = submit(pick[j])
                ready.release()

        th = threading.Thread(target=producer)
        t0 = time.perf_counter()
        th.start()
        lat = []
        for j in range(n_per_rate):
            ready.acquire()
            st, ns, _, _ = srv.wait(tickets[j])
            if st != 0:
                raise RuntimeError(f"serving request failed with status {st}")
            lat.append(ns * 1e-6)
        dt = time.perf_counter() - t0
        th.join()
        res["rates"].append({"lambda_frac": frac, "lambda_req_per_s": lam, "requests": n_per_rate,
                             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "throughput_req_per_s": n_per_rate / dt,
                             "q_t_per_s": sum(qt[i] for i in pick) / dt,
                             "max_submit_lag_ms": float(late[0] * 1e3),
                             "stage_ms_mean": stage_means(st0, srv.stats())})
        if log:
            r = res["rates"][-1]
            log(f"serving {precision}: lambda {frac:.2f} mu -> p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms, "
                f"{r['throughput_req_per_s']:.2f} req/s")
    st = srv.stats()
    res["server_stats"] = {k: v for k, v in st.items()
                           if k.startswith("peak") or k in ("completed", "failed", "mol_cache_hits")}
    srv.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1, help="workload: 1 (64^3), 2 (128^3), 3 (96^3, 570 bf)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--screen-eps", type=float, default=1e-9)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-points", type=int, default=48, help="oracle-checked grid points (0 = skip)")
    ap.add_argument("--no-bf16", action="store_true", help="skip the split-BF16 comparison run")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving latency leg")
    ap.add_argument("--no-symmetric", action="store_true",
                    help="skip the symmetric-grid measurement (f(-q) = f(q)*, half the planes evaluated)")
    ap.add_argument("--serve-pool", type=int, default=24, help="distinct requests in the serving pool")
    ap.add_argument("--serve-sat", type=int, default=48, help="requests of the closed-loop saturation run")
    ap.add_argument("--serve-requests", type=int, default=96, help="requests per Poisson arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=8)
    ap.add_argument("--serve-inflight", type=int, default=4)
    ap.add_argument("--serve-precisions", default="fp32,bf16x3")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the measurement, run one plain device copy of this many MiB (a known-size "
                         "kernel for calibrating hardware byte counters in the same profiled run)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build runs on one GPU "
              "(the q-grid shards into independent slabs; multi-GPU runs are out of scope here)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workload as wl
    from paper_2512_18010_amd import binding

    W = wl.make_config(args.config)
    ns = W.T.shape[0]
    n = tuple(W.grid.n)
    nq = n[0] * n[1] * n[2]
    ctx = binding.Context(0)
    ctx.set_timing(True)
    T_dev = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
    f = torch.empty((ns,) + n + (2,), dtype=torch.float32, device="cuda")
    f2 = torch.empty((ns,) + n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(precision, steps, warmup):
        """Whole-path steps with inputs resident in HBM; HIP events per stage."""
        def step():
            ctx.load_molecule(W.mol)
            ctx.load_transitions_device(T_dev, stream)
            ctx.set_options(args.screen_eps, 1.0)
            ctx.eval_grid_device(W.grid, f, f2, precision=precision, stream=stream)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        stages = []
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
            stages.append(ctx.last_timing())   # HIP events of this step's kernels, on `stream`
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = np.array(stages)
        prep_ms, vt_ms, grid_ms = (float(np.mean(st[:, i])) for i in range(3))
        return {"ms_per_step": wall / steps * 1e3, "precompute_ms": prep_ms, "vtables_ms": vt_ms,
                "grid_kernel_ms": grid_ms}

    def check_errors():
        """Accuracy of the last step on a seeded sample against the FP64 oracle."""
        if args.check_points <= 0:
            return None
        import oracle
        from tests.metrics import errors as err_fn
        idx = wl.sample_grid_indices(W.grid, args.check_points, seed=4242)
        f2h = f2.reshape(ns, -1).cpu().numpy()
        idx = np.unique(np.concatenate([idx, f2h.argmax(axis=1)]))
        fh = f.reshape(ns, -1, 2).cpu().numpy()
        fs = fh[:, idx, 0] + 1j * fh[:, idx, 1]
        ref = oracle.eval_points(W.mol, W.T, W.grid.points()[idx], n_threads=min(16, os.cpu_count() or 1))
        e = err_fn(fs, ref)
        return {"points": int(len(idx)), "max_f2_peak_normalised": float(e["f2_peak_norm"].max()),
                "max_complex": float(e["complex"].max())}

    main_run = timed(args.precision, args.steps, args.warmup)
    ms_per_step, grid_ms = main_run["ms_per_step"], main_run["grid_kernel_ms"]
    prep_ms, vt_ms = main_run["precompute_ms"], main_run["vtables_ms"]
    errors = check_errors()
    info = ctx.query()
    K, R = info["pairs_kept"], info["prim_comp_pairs_kept"]

    # roofline of the fused grid kernel
    gen_flops = 8.0 * R * nq                    # one complex MAC per (pair, prim pair, q)
    con_flops = 4.0 * K * ns * nq               # real Tp x complex G per (pair, q, transition)
    t_valu = gen_flops / PEAK_FP32_VECTOR

    def t_mfma(precision):
        return con_flops * (3 if precision == "bf16x3" else 1) / (
            PEAK_BF16_MFMA if precision == "bf16x3" else PEAK_FP32_MFMA)

    grid_s = grid_ms * 1e-3
    achieved = gen_flops / grid_s
    wkey = f"cfg{args.config}/eps{args.screen_eps:g}"
    traffic = measured_traffic(wkey, args.precision)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
            "kernel": "grid_kernel", "kernel_ms": grid_ms,
            "algorithmic": {"generator_flops": gen_flops, "contraction_flops": con_flops,
                            "t_valu_ms": t_valu * 1e3, "t_mfma_ms": t_mfma(args.precision) * 1e3,
                            "t_star_ms": max(t_valu, t_mfma(args.precision)) * 1e3,
                            "frac_of_t_star": max(t_valu, t_mfma(args.precision)) / grid_s,
                            # a SIMD does not execute VALU and MFMA work at the same time, so
                            # the attainable time is the sum of the two pipes' times
                            "t_additive_ms": (t_valu + t_mfma(args.precision)) * 1e3,
                            "frac_of_additive": (t_valu + t_mfma(args.precision)) / grid_s,
                            "mfma_achieved_tflops": con_flops / grid_s / 1e12}}

    # the other contraction precision on the same workload (FP32 vs split-BF16)
    other = None
    if not args.no_bf16:
        oprec = "bf16x3" if args.precision == "fp32" else "fp32"
        o = timed(oprec, max(3, args.steps // 2), 1)
        o["errors_vs_oracle"] = check_errors()
        o["precision"] = oprec
        o["value"] = ns * nq / (o["ms_per_step"] * 1e-3)
        o["kernel_only_value"] = ns * nq / (o["grid_kernel_ms"] * 1e-3)
        o["t_star_ms"] = max(t_valu, t_mfma(oprec)) * 1e3
        o["t_additive_ms"] = (t_valu + t_mfma(oprec)) * 1e3
        other = o

    # the same workload in the symmetric-grid mode: the grid is symmetric about
    # q = 0 and T is real, so the planes ix >= ceil(nx/2) are written as
    # f(-q) = f(q)* of evaluated ones (not part of the headline value)
    symmetric = None
    sym_grid = all(W.grid.qmin[a] == -W.grid.qmax[a] for a in range(3))
    if not args.no_symmetric and sym_grid:
        ctx.set_symmetry(True)
        o = timed(args.precision, max(3, args.steps // 2), 1)
        o["errors_vs_oracle"] = check_errors()
        ctx.set_symmetry(False)
        o["precision"] = args.precision
        o["value"] = ns * nq / (o["ms_per_step"] * 1e-3)
        o["kernel_only_value"] = ns * nq / (o["grid_kernel_ms"] * 1e-3)
        o["planes_evaluated"] = (n[0] + 1) // 2
        symmetric = o

    serving = None
    if not args.no_serving:
        serving = []
        for prec in [p for p in args.serve_precisions.split(",") if p]:
            serving.append(serving_benchmark(prec, args.serve_pool, args.serve_sat, args.serve_requests,
                                             args.serve_warmup, args.serve_inflight, 64.0, args.screen_eps,
                                             log=lambda m: print(m, file=sys.stderr, flush=True)))

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")   # fill: writes N MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)                                                  # reads and writes N MiB
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(W, args.cpu_seconds, threads)

    out = {
        "metric": "q-points x transitions / s (Cartesian form factor, full grid)",
        "value": ns * nq / (ms_per_step * 1e-3),
        "unit": "q-points*transitions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": W.name, "config_id": args.config, "nbf": W.mol.nbf, "n_states": ns,
                   "grid": list(n), "qmax": W.grid.qmax[0], "precision": args.precision,
                   "screen_eps": args.screen_eps, "pairs_kept_K": K, "terms_kept_R": R,
                   "pairs_total": info["pairs_total"], "terms_total": info["prim_pairs_total"]},
        "stages_ms": {"precompute": prep_ms, "vtables": vt_ms, "grid_kernel": grid_ms},
        "kernel_only_value": ns * nq / grid_s,
        "roofline": roof,
        "cpu_baseline": cpu,
        "errors_vs_oracle": errors,
        "other_precision": other,
        "symmetric_grid": symmetric,
        "serving": serving,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
