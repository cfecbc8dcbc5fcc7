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
    """Hash of the grid kernel's source: kernels.hip and the part of engine.h
    that defines its layout constants and descriptor (from the namespace to
    the first runtime declaration), with comments and blank lines dropped (a
    comment edit or a change elsewhere does not invalidate measured counters;
    a change of the kernel's code does)."""
    import re
    h = hashlib.sha256()
    for name in ("kernels.hip", "engine.h"):
        with open(os.path.join(ROOT, "paper_2512_18010_amd", "csrc", name)) as fh:
            text = fh.read()
        if name == "engine.h":
            text = text[text.index("namespace scff {"):text.index("struct DeviceBuffer")]
        text = re.sub(r"//[^\n]*", "", text)
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
                raise RuntimeError(f"serving request failed with status {st}: {srv.last_failure()}")
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
                raise RuntimeError(f"serving request failed with status {st}: {srv.last_failure()}")
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
                           if k.startswith("peak") or k in ("completed", "failed", "mol_cache_hits", "batches",
                                                            "batched_requests", "graphs_instantiated",
                                                            "graphs_updated", "eager_batches")}
    srv.close()
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def grid_roofline(K, R, ns, nq, precision, grid_ms):
    """Algorithmic bounds of the fused grid kernel on one launch: generator
    flops (8 R per q-point) on the FP32 vector units, contraction flops
    (4 K per q-point and transition; three products for split-BF16) on the
    matrix cores.  The binding pipe is the one with the larger time bound."""
    gen_flops = 8.0 * R * nq
    con_flops = 4.0 * K * ns * nq
    bf = precision == "bf16x3"
    con_issued = con_flops * (3 if bf else 1)
    mfma_peak = PEAK_BF16_MFMA if bf else PEAK_FP32_MFMA
    t_valu = gen_flops / PEAK_FP32_VECTOR
    t_mfma = con_issued / mfma_peak
    grid_s = grid_ms * 1e-3
    if t_mfma > t_valu:
        bound, achieved, peak = "mfma", con_issued / grid_s, mfma_peak
    else:
        bound, achieved, peak = "alu", gen_flops / grid_s, PEAK_FP32_VECTOR
    return {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "algorithmic": {"generator_flops": gen_flops, "contraction_flops": con_flops,
                            "contraction_flops_issued": con_issued,
                            "t_valu_ms": t_valu * 1e3, "t_mfma_ms": t_mfma * 1e3,
                            "t_star_ms": max(t_valu, t_mfma) * 1e3,
                            "frac_of_t_star": max(t_valu, t_mfma) / grid_s,
                            "t_additive_ms": (t_valu + t_mfma) * 1e3,
                            "frac_of_additive": (t_valu + t_mfma) / grid_s,
                            "valu_achieved_tflops": gen_flops / grid_s / 1e12,
                            "mfma_achieved_tflops": con_issued / grid_s / 1e12}}


def fft_benchmark(ctx, stream, n_axis, steps, warmup, log, precision="fp32"):
    """FFT method on the config-1 molecule and its 12 transitions in the
    paper's doubled box (bounding box + 5 bohr, times 2) sampled at n_axis^3
    points: one step = molecule load + T from HBM + weight packing + density +
    transforms + finishing, f and |f|^2 left in HBM.  precision: the density
    contraction's arithmetic ("fp32" or split "bf16x3")."""
    import torch
    import workload as wl
    W = wl.make_config(1)
    n, xmin, L = wl.fft_box(W.mol, (n_axis,) * 3)
    ns, nbf = W.T.shape[0], W.mol.nbf
    npts = n[0] * n[1] * n[2]
    T_dev = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
    f = torch.empty((ns,) + n + (2,), dtype=torch.float32, device="cuda")
    f2 = torch.empty((ns,) + n, dtype=torch.float32, device="cuda")

    def step():
        ctx.load_molecule(W.mol)
        ctx.load_transitions_device(T_dev, stream)
        ctx.set_options(0.0, 1.0)
        ctx.eval_fft_device(n, xmin, L, f, f2, None, stream=stream, precision=precision)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        st.append(ctx.last_fft_timing())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    st = np.array(st)
    pack_ms, dens_ms, tr_ms = (float(np.mean(st[:, i])) for i in range(3))
    # checks: the density on seeded points against the oracle, Parseval's identity
    import oracle
    _, _, phi, ps = ctx.eval_fft_host(n, xmin, L, want_f=False, want_f2=False, want_phi=True, parseval=True,
                                      precision=precision)
    rng = np.random.Generator(np.random.PCG64(99))
    idx = np.concatenate([rng.integers(0, npts, 200), np.abs(phi.reshape(ns, -1)).argmax(axis=1)])
    ax = oracle.real_space_axes(n, xmin, L)
    ii = np.unravel_index(idx, n)
    pts = np.stack([ax[0][ii[0]], ax[1][ii[1]], ax[2][ii[2]]], axis=1)
    ref = oracle.density(W.mol, W.T, pts, n_threads=min(16, os.cpu_count() or 1))
    e_phi = np.abs(phi.reshape(ns, -1)[:, idx] - ref).max(axis=1) / np.abs(phi.reshape(ns, -1)).max(axis=1)
    e_par = np.abs(ps[:, 0] / ps[:, 1] - 1.0)
    del T_dev, f, f2
    pairs = nbf * (nbf + 1) // 2
    flops = 2.0 * pairs * ns * npts
    nb = (ns + 1) // 2
    passes = sum(1 for a in range(3) if n[a] > 1)
    tr_bytes = passes * 2 * nb * npts * 8 + 2 * nb * npts * 8 + ns * npts * 12
    bf = precision == "bf16x3"
    peak = PEAK_BF16_MFMA if bf else PEAK_FP32_MFMA
    # matrix-core instructions as issued: per 16-point tile, state and row block rb
    # of 16 functions, the k-steps from the block's diagonal to the end
    nbf_pad = (nbf + 15) // 16 * 16
    RB, kstep = nbf_pad // 16, (8 if bf else 4)
    n_mfma = ns * ((npts + 15) // 16) * sum(nbf_pad // kstep - 16 * rb // kstep for rb in range(RB))
    issued = n_mfma * 2.0 * 16 * 16 * (32 if bf else 4)
    log(f"fft method {n} {precision}: {ms:.2f} ms/step, density {dens_ms:.2f} ms ({flops / dens_ms / 1e9:.1f} TFLOP/s), "
        f"transforms {tr_ms:.2f} ms, density error {e_phi.max():.2e}, Parseval {e_par.max():.2e}")
    return {
        "workload": f"{W.name}; FFT box {n[0]}x{n[1]}x{n[2]} = bounding box + 5 bohr, doubled",
        "precision": precision,
        "box": {"n": list(n), "xmin": list(xmin), "L": list(L)},
        "steps": steps, "ms_per_step": ms,
        "value": ns * npts / (ms * 1e-3), "unit": "q-points*transitions/s",
        "stages_ms": {"pack": pack_ms, "density": dens_ms, "transforms": tr_ms},
        "roofline": {"bound": "mfma", "kernel": "fft_density_kernel",
                     "achieved": flops / (dens_ms * 1e-3) / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": flops / (dens_ms * 1e-3) / peak,
                     "per_unit": "2 flops per (unordered AO pair, real-space point, transition) on the matrix cores",
                     "issued_tflops": issued / (dens_ms * 1e-3) / 1e12,
                     "issued_frac": issued / (dens_ms * 1e-3) / peak,
                     "units": {"pairs": pairs, "points": npts, "n_states": ns}},
        "transforms_roofline": {"bound": "hbm", "achieved": tr_bytes / (tr_ms * 1e-3) / 1e9,
                                "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                "frac": tr_bytes / (tr_ms * 1e-3) / PEAK_HBM,
                                "per_unit": "per pass 16 B per complex point of each state pair; finishing "
                                            "16 B read per pair and 12 B written per state per point"},
        "errors_vs_oracle": {"density_sampled_max": float(e_phi.max()),
                             "density_per_transition": [float(x) for x in e_phi],
                             "parseval_max": float(e_par.max())},
    }


def lowq_benchmark(ctx, case, log, calls=20):
    """Separable integrals (Sec. 5.3) and the low-momentum limit (Sec. 6) on
    the benchmark workload, whose FP32 grid f is resident in HBM: one
    separable integral I_s = sum_q wx wy wz f_s(q) per call (seeded complex
    weights; cost linear in the axis sizes), checked against the FP64
    weighted sum of the GPU's own grid; the transition dipoles and oscillator
    strengths.  Both calls return host results and wait for the device."""
    import torch
    W = case.W
    ns, nq = case.ns, case.nq
    rng = np.random.Generator(np.random.PCG64(123))
    ws = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in case.n]
    ctx.eval_separable(W.grid, *ws)
    t0 = time.perf_counter()
    for _ in range(calls):
        I = ctx.eval_separable(W.grid, *ws)
    sep_ms = (time.perf_counter() - t0) / calls * 1e3
    fc = torch.view_as_complex(case.f.double().contiguous())
    wt = [torch.from_numpy(w).to(device=fc.device) for w in ws]
    ref = (fc * wt[0][None, :, None, None] * wt[1][None, None, :, None] * wt[2][None, None, None, :]).sum(dim=(1, 2, 3))
    ref = ref.cpu().numpy()
    e_sep = float(np.abs(I - ref).max() / np.abs(ref).max())
    dE = np.full(ns, 0.2)
    ctx.dipole(dE)
    t0 = time.perf_counter()
    for _ in range(calls):
        mu, f0 = ctx.dipole(dE)
    dip_ms = (time.perf_counter() - t0) / calls * 1e3
    log(f"separable integral: {sep_ms:.3f} ms per call ({ns * nq / (sep_ms * 1e-3):.3g} equivalent q-points*transitions/s), "
        f"vs the FP32 grid {e_sep:.1e}; dipoles: {dip_ms:.3f} ms per call")
    return {
        "workload": W.name,
        "separable_integral": {
            "ms_per_call": sep_ms, "calls": calls,
            "value": ns * nq / (sep_ms * 1e-3), "unit": "equivalent q-points*transitions/s",
            "note": "host-timed synchronous calls (weights in, I_s out): three small FP64 kernels "
                    "(row sums, triple products per term, transition-weighted reduction), latency-bound",
            "relative_difference_vs_fp32_grid": e_sep},
        "dipole": {"ms_per_call": dip_ms, "calls": calls,
                   "mu_norm": [float(x) for x in np.linalg.norm(mu, axis=1)],
                   "f0": [float(x) for x in f0]},
    }


def sph_benchmark(ctx, stream, lmax, n, steps, warmup, log):
    """Spherical method on the config-1 molecule and its 12 transitions: R_lm
    up to lmax on n radii in (0, 6] a.u. and f on n x n angles per radius
    (n^3 q-points).  One step = molecule load + T from HBM + pair precompute +
    geometry kernel + contraction + coupling + angular grid, outputs in HBM."""
    import torch
    import workload as wl
    W = wl.make_config(1)
    ns = W.T.shape[0]
    qs = 6.0 * np.arange(1, n + 1) / n
    nl = (lmax + 1) ** 2
    T_dev = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
    f = torch.empty((ns, n, n, n, 2), dtype=torch.float32, device="cuda")
    f2 = torch.empty((ns, n, n, n), dtype=torch.float32, device="cuda")
    R = torch.empty((ns, n, nl, 2), dtype=torch.float64, device="cuda")
    avg = torch.empty((ns, n), dtype=torch.float64, device="cuda")

    def step():
        ctx.load_molecule(W.mol)
        ctx.load_transitions_device(T_dev, stream)
        ctx.set_options(0.0, 1.0)
        ctx.eval_spherical_device(lmax, qs, n, n, f, f2, R, avg, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        st.append(ctx.last_sph_timing())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    st = np.array(st)
    geom_ms, con_ms, rest_ms = (float(np.mean(st[:, i])) for i in range(3))
    # check: R on one radius against the oracle's projection (the GPU tests cover the rest)
    import oracle
    k = max(0, n // 8 - 1)
    rmax = float(np.linalg.norm(W.mol.xyz, axis=1).max()) + 3.0
    nt = int((lmax + np.e * qs[k] * rmax / 2 + 24) / 2) + 2
    Rref = oracle.spherical_R(W.mol, W.T, [qs[k]], lmax, nt, n_threads=min(16, os.cpu_count() or 1))[:, 0, :]
    Rg = R[:, k].cpu().numpy()
    Rg = Rg[..., 0] + 1j * Rg[..., 1]
    e_R = np.abs(Rg - Rref).max(axis=1) / np.abs(Rref).max(axis=1)
    n_geo = int(sum(int(W.mol.shell_nprim[a]) * int(W.mol.shell_nprim[b])
                    for a in range(W.mol.n_shells) for b in range(a, W.mol.n_shells)))
    ncols = (lmax + 5) ** 2
    flops = 8.0 * ns * 25 * ncols * n_geo * n
    del T_dev, f, f2, R, avg
    log(f"spherical method lmax {lmax}, {n}^3: {ms:.2f} ms/step, contraction {con_ms:.2f} ms "
        f"({flops / con_ms / 1e9:.1f} TFLOP/s FP64), geometry {geom_ms:.2f} ms, rest {rest_ms:.2f} ms, "
        f"R error {e_R.max():.1e}")
    return {
        "workload": f"{W.name}; lmax {lmax}, {n} radii in (0, 6] x {n} polar x {n} azimuthal angles",
        "lmax": lmax, "n_radii": n, "n_theta": n, "n_phi": n, "geometries": n_geo,
        "steps": steps, "ms_per_step": ms,
        "value": ns * n ** 3 / (ms * 1e-3), "unit": "q-points*transitions/s",
        "stages_ms": {"geometry": geom_ms, "contraction": con_ms, "coupling_and_grid": rest_ms},
        "roofline": {"bound": "fp64", "kernel": "sph_q_kernel", "achieved": flops / (con_ms * 1e-3) / 1e12,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": flops / (con_ms * 1e-3) / 78.6e12,
                     "per_unit": "8 flops per (transition, harmonic lam mu <= 4, harmonic L M <= lmax + 4, "
                                 "geometry, radius): one complex multiply-add of the contraction over geometries"},
        "errors_vs_oracle": {"R_relative_max": float(e_R.max()), "R_per_transition": [float(x) for x in e_R],
                             "radius": float(qs[k])},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3,
                    help="headline workload: 3 (570 bf, 24 transitions, 96^3; default), 1 (190 bf, 64^3), "
                         "2 (190 bf, 128^3)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--screen-eps", type=float, default=1e-9)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-seconds-1core", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-points", type=int, default=48, help="oracle-checked grid points (0 = skip)")
    ap.add_argument("--no-bf16", action="store_true", help="skip the other-precision run of the headline workload")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the 128^3 leg (190 bf, 12 transitions: split-BF16 vs FP32, error per transition)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving latency leg")
    ap.add_argument("--no-fft", action="store_true",
                    help="skip the FFT-method leg (190 bf, 12 transitions, 128^3 real-space box)")
    ap.add_argument("--fft-n", type=int, default=128, help="real-space points per axis of the FFT-method leg")
    ap.add_argument("--no-lowq", action="store_true",
                    help="skip the separable-integral and dipole leg")
    ap.add_argument("--no-sph", action="store_true",
                    help="skip the spherical-method leg (190 bf, 12 transitions, lmax 24, 64 radii x 64 x 64 angles)")
    ap.add_argument("--sph-lmax", type=int, default=24)
    ap.add_argument("--sph-n", type=int, default=64, help="radii, polar and azimuthal points of the spherical leg")
    ap.add_argument("--no-symmetric", action="store_true",
                    help="skip the symmetric-grid measurement (f(-q) = f(q)*, half the planes evaluated)")
    ap.add_argument("--serve-pool", type=int, default=24, help="distinct requests in the serving pool")
    ap.add_argument("--serve-sat", type=int, default=120, help="requests of the closed-loop saturation run")
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

    def log(m):
        print(m, file=sys.stderr, flush=True)

    ctx = binding.Context(0)
    ctx.set_timing(True)
    stream = torch.cuda.current_stream()

    class Case:
        """One workload resident in HBM: T on the device, output tensors."""

        def __init__(self, cfg):
            self.cfg = cfg
            self.W = wl.make_config(cfg)
            self.ns = self.W.T.shape[0]
            self.n = tuple(self.W.grid.n)
            self.nq = self.n[0] * self.n[1] * self.n[2]
            self.T_dev = torch.from_numpy(np.ascontiguousarray(self.W.T)).cuda()
            self.f = torch.empty((self.ns,) + self.n + (2,), dtype=torch.float32, device="cuda")
            self.f2 = torch.empty((self.ns,) + self.n, dtype=torch.float32, device="cuda")

        def release(self):
            del self.T_dev, self.f, self.f2

        def step(self, precision):
            ctx.load_molecule(self.W.mol)
            ctx.load_transitions_device(self.T_dev, stream)
            ctx.set_options(args.screen_eps, 1.0)
            ctx.eval_grid_device(self.W.grid, self.f, self.f2, precision=precision, stream=stream)

        def timed(self, precision, steps, warmup):
            """Whole-path steps with inputs resident in HBM; HIP events per stage."""
            for _ in range(warmup):
                self.step(precision)
            torch.cuda.synchronize()
            stages = []
            t0 = time.perf_counter()
            for _ in range(steps):
                self.step(precision)
                stages.append(ctx.last_timing())   # HIP events of this step's kernels, on `stream`
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = np.array(stages)
            prep_ms, vt_ms, grid_ms = (float(np.mean(st[:, i])) for i in range(3))
            info = ctx.query()
            K, R = info["pairs_kept"], info["prim_comp_pairs_kept"]
            ms = wall / steps * 1e3
            return {"precision": precision, "steps": steps, "ms_per_step": ms,
                    "value": self.ns * self.nq / (ms * 1e-3),
                    "kernel_only_value": self.ns * self.nq / (grid_ms * 1e-3),
                    "stages_ms": {"precompute": prep_ms, "vtables": vt_ms, "grid_kernel": grid_ms},
                    "pairs_kept_K": K, "terms_kept_R": R,
                    "roofline": grid_roofline(K, R, self.ns, self.nq, precision, grid_ms)}

        def errors(self, n_points, seed=4242):
            """Accuracy of the last step on a seeded sample plus every
            transition's |f|^2 maximum, against the FP64 oracle, per transition."""
            if n_points <= 0:
                return None
            import oracle
            from tests.metrics import errors as err_fn
            idx = wl.sample_grid_indices(self.W.grid, n_points, seed=seed)
            f2h = self.f2.reshape(self.ns, -1).cpu().numpy()
            idx = np.unique(np.concatenate([idx, f2h.argmax(axis=1)]))
            fh = self.f.reshape(self.ns, -1, 2).cpu().numpy()
            fs = fh[:, idx, 0] + 1j * fh[:, idx, 1]
            ref = oracle.eval_points(self.W.mol, self.W.T, self.W.grid.points()[idx],
                                     n_threads=min(16, os.cpu_count() or 1))
            e = err_fn(fs, ref)
            return {"points": int(len(idx)), "max_f2_peak_normalised": float(e["f2_peak_norm"].max()),
                    "max_complex": float(e["complex"].max()),
                    "f2_peak_normalised_per_transition": [float(x) for x in e["f2_peak_norm"]]}

    def run_both(case, first, steps, warmup, check_points, other=True):
        res = case.timed(first, steps, warmup)
        res["errors_vs_oracle"] = case.errors(check_points)
        out = {first: res}
        if other:
            op = "bf16x3" if first == "fp32" else "fp32"
            o = case.timed(op, max(3, steps // 2), 1)
            o["errors_vs_oracle"] = case.errors(check_points)
            out[op] = o
        for p, r in out.items():
            e = r["errors_vs_oracle"]
            log(f"config {case.cfg} {p}: {r['ms_per_step']:.2f} ms/step, grid kernel "
                f"{r['stages_ms']['grid_kernel']:.2f} ms, {r['roofline']['algorithmic']['frac_of_t_star']:.3f} "
                f"of t*" + (f", max |f|^2 error {e['max_f2_peak_normalised']:.2e}" if e else ""))
        return out

    # ---- headline workload: the requested precision, then the other one
    main_case = Case(args.config)
    W = main_case.W
    ns, n, nq = main_case.ns, main_case.n, main_case.nq
    legs = run_both(main_case, args.precision, args.steps, args.warmup, args.check_points, not args.no_bf16)
    head = legs[args.precision]
    other = legs.get("bf16x3" if args.precision == "fp32" else "fp32")
    ms_per_step = head["ms_per_step"]
    grid_ms = head["stages_ms"]["grid_kernel"]
    K, R = head["pairs_kept_K"], head["terms_kept_R"]
    info = ctx.query()

    roof = dict(head["roofline"])
    wkey = f"cfg{args.config}/eps{args.screen_eps:g}"
    roof["traffic"] = measured_traffic(wkey, args.precision)
    roof["kernel"] = "grid_kernel"
    roof["kernel_ms"] = grid_ms
    roof["units"] = {"K": K, "R": R, "n_states": ns, "q_points": nq,
                     "per_unit": "8 flops per (term, q-point) on the vector units; 4 flops per "
                                 "(pair, q-point, transition) on the matrix cores (x3 for split-BF16)"}

    # the same workload in the symmetric-grid mode: the grid is symmetric about
    # q = 0 and T is real, so the planes ix >= ceil(nx/2) are written as
    # f(-q) = f(q)* of evaluated ones (not part of the headline value)
    symmetric = None
    sym_grid = all(W.grid.qmin[a] == -W.grid.qmax[a] for a in range(3))
    if not args.no_symmetric and sym_grid:
        ctx.set_symmetry(True)
        o = main_case.timed(args.precision, max(3, args.steps // 2), 1)
        o["errors_vs_oracle"] = main_case.errors(args.check_points)
        ctx.set_symmetry(False)
        o["planes_evaluated"] = (n[0] + 1) // 2
        del o["roofline"]
        symmetric = o
    # ---- separable integrals and the low-momentum limit on the same workload
    lowq = None
    if not args.no_lowq:
        main_case.step("fp32")
        torch.cuda.synchronize()
        lowq = lowq_benchmark(ctx, main_case, log)
    main_case.release()

    # ---- 128^3 leg: split-BF16 against plain FP32, error per transition
    config2 = None
    if not args.no_config2 and args.config != 2:
        c2 = Case(2)
        legs2 = run_both(c2, "fp32", max(5, args.steps // 2), 2, max(args.check_points, 64))
        c2.release()
        config2 = {"workload": c2.W.name, "grid": list(c2.n), "n_states": c2.ns, "legs": legs2}

    # ---- FFT method (Sec. 3, Sec. 5.2): config-1 molecule and transitions
    fft_leg = None
    if not args.no_fft:
        fft_leg = fft_benchmark(ctx, stream, args.fft_n, max(10, args.steps // 2), 2, log)
        fft_leg["other_precision"] = fft_benchmark(ctx, stream, args.fft_n, max(10, args.steps // 2), 2, log,
                                                   precision="bf16x3")

    # ---- spherical method (Sec. 4, Sec. 5.4): config-1 molecule and transitions
    sph_leg = None
    if not args.no_sph:
        sph_leg = sph_benchmark(ctx, stream, args.sph_lmax, args.sph_n, max(3, args.steps // 4), 1, log)

    serving = None
    if not args.no_serving:
        serving = []
        for prec in [p for p in args.serve_precisions.split(",") if p]:
            serving.append(serving_benchmark(prec, args.serve_pool, args.serve_sat, args.serve_requests,
                                             args.serve_warmup, args.serve_inflight, 64.0, args.screen_eps,
                                             log=log))

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
        one = cpu_baseline(W, args.cpu_seconds_1core, 1)
        cpu["cpu_model"] = cpu_model()
        cpu["host_threads_available"] = os.cpu_count()
        cpu["value_1core"] = one["value"]
        cpu["sample_1core"] = one["sample"]

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
        "stages_ms": head["stages_ms"],
        "kernel_only_value": head["kernel_only_value"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "errors_vs_oracle": head["errors_vs_oracle"],
        "other_precision": other,
        "config2": config2,
        "symmetric_grid": symmetric,
        "serving": serving,
        "low_momentum_and_separable": lowq,
        "fft_method": fft_leg,
        "spherical_method": sph_leg,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
