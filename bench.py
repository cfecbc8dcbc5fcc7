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
    h = hashlib.sha256()
    for name in ("kernels.hip",):
        with open(os.path.join(ROOT, "paper_2512_18010_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
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

    def step():
        ctx.load_molecule(W.mol)
        ctx.load_transitions_device(T_dev, stream)
        ctx.set_options(args.screen_eps, 1.0)
        ctx.eval_grid_device(W.grid, f, f2, precision=args.precision, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        stages.append(ctx.last_timing())   # HIP events of this step's kernels, on `stream`
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    info = ctx.query()
    K, R = info["pairs_kept"], info["prim_comp_pairs_kept"]
    st = np.array(stages)
    prep_ms, vt_ms, grid_ms = (float(np.mean(st[:, i])) for i in range(3))

    # roofline of the fused grid kernel
    gen_flops = 8.0 * R * nq                    # one complex MAC per (pair, prim pair, q)
    con_flops = 4.0 * K * ns * nq               # real Tp x complex G per (pair, q, transition)
    t_valu = gen_flops / PEAK_FP32_VECTOR
    t_mfma = con_flops * (3 if args.precision == "bf16x3" else 1) / (
        PEAK_BF16_MFMA if args.precision == "bf16x3" else PEAK_FP32_MFMA)
    grid_s = grid_ms * 1e-3
    achieved = gen_flops / grid_s
    wkey = f"cfg{args.config}/eps{args.screen_eps:g}"
    traffic = measured_traffic(wkey, args.precision)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic,
            "kernel": "grid_kernel", "kernel_ms": grid_ms,
            "algorithmic": {"generator_flops": gen_flops, "contraction_flops": con_flops,
                            "t_valu_ms": t_valu * 1e3, "t_mfma_ms": t_mfma * 1e3,
                            "t_star_ms": max(t_valu, t_mfma) * 1e3,
                            "frac_of_t_star": max(t_valu, t_mfma) / grid_s,
                            "mfma_achieved_tflops": con_flops / grid_s / 1e12}}

    # accuracy on a seeded sample against the FP64 oracle (outside the timed region)
    errors = None
    if args.check_points > 0:
        import oracle
        from tests.metrics import errors as err_fn
        idx = wl.sample_grid_indices(W.grid, args.check_points, seed=4242)
        f2h = f2.reshape(ns, -1).cpu().numpy()
        idx = np.unique(np.concatenate([idx, f2h.argmax(axis=1)]))
        fh = f.reshape(ns, -1, 2).cpu().numpy()
        fs = fh[:, idx, 0] + 1j * fh[:, idx, 1]
        ref = oracle.eval_points(W.mol, W.T, W.grid.points()[idx], n_threads=min(16, os.cpu_count() or 1))
        e = err_fn(fs, ref)
        errors = {"points": int(len(idx)), "max_f2_peak_normalised": float(e["f2_peak_norm"].max()),
                  "max_complex": float(e["complex"].max())}

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
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
