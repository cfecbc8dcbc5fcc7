"""Serving on the GPU: requests admitted while others run, overlapping on the
device; every result is the same alone and in the mix, and matches the oracle."""
import os
import sys

import numpy as np
import pytest

import workload as wl
from tests.metrics import TOL_F2, errors, report

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def requests(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        n_heavy = int(rng.integers(2, 9))
        mol = wl.make_molecule(rng, n_heavy, int(round(0.8 * n_heavy)), layout="box",
                               box_A=12.0 * (n_heavy / 30.0) ** (1 / 3) + 1.0)
        ns = int(rng.integers(1, 25))
        N = int(rng.integers(16, 41))
        qm = float(rng.uniform(5.0, 8.0))
        T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), ns)
        out.append((mol, T, wl.Grid(n=(N, N + 1, N - 1), qmin=(-qm,) * 3, qmax=(qm,) * 3)))
    return out


def big_request(seed):
    """A request at the large end of the serving mix: 24 heavy atoms with
    proportional hydrogens (s/p/d basis, 456 functions), 20 transitions, a
    64 x 66 x 65 grid with |q_i| <= 7."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_heavy = 24
    mol = wl.make_molecule(rng, n_heavy, int(round(0.8 * n_heavy)), layout="box",
                           box_A=12.0 * (n_heavy / 30.0) ** (1 / 3))
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 20)
    return mol, T, wl.Grid(n=(64, 66, 65), qmin=(-7.0,) * 3, qmax=(7.0,) * 3)


def oracle_sample_check(oracle_mod, name, mol, T, g, f, f2, precision, n=40, seed=0):
    """Seeded grid points plus every transition's |f|^2 maximum against the
    oracle; logs the error of each transition."""
    idx = wl.sample_grid_indices(g, n, seed=seed)
    idx = np.unique(np.concatenate([idx, f2.reshape(T.shape[0], -1).argmax(axis=1)]))
    ref = oracle_mod.eval_points(mol, T, g.points()[idx], n_threads=min(16, os.cpu_count() or 1))
    e = errors(f.reshape(T.shape[0], -1)[:, idx], ref)
    report(f"[serving {name}] {precision}: " + " ".join(f"{x:.2e}" for x in e["f2_peak_norm"]))
    assert e["f2_peak_norm"].max() <= TOL_F2[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_alone_vs_mix_identical_and_correct(oracle_mod, precision):
    """Eight small requests and one at the large end of the serving mix
    (24 heavy atoms, 456 functions, 20 transitions, 64 x 66 x 65), each run
    alone and then all submitted at once: every result is bit-identical alone
    and in the mix, and the large request and two small ones match the
    oracle on sampled points."""
    import torch  # noqa: F401
    from paper_2512_18010_amd import binding
    reqs = requests(2024, 8)
    reqs.insert(2, big_request(2025))
    alone = []
    with binding.Server(0, 0, max_inflight=4) as srv:
        for k, (mol, T, g) in enumerate(reqs):
            log(f"alone {k} {precision}: nbf={mol.nbf} states={T.shape[0]} grid={g.n}")
            t = srv.submit(mol, T, g, precision=precision, screen_eps=1e-9)
            status, lat, f, f2 = srv.wait(t)
            assert status == binding.SCFF_OK
            alone.append((f.copy(), f2.copy()))
        log("mix: submitting all")
        tickets = [srv.submit(mol, T, g, precision=precision, screen_eps=1e-9) for (mol, T, g) in reqs]
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
    log("stats", st)
    assert st["peak_inflight"] >= 2, "requests should overlap on the device"
    for k, ((fa, f2a), (status, lat, fm, f2m)) in enumerate(zip(alone, mixed)):
        assert status == binding.SCFF_OK
        assert np.array_equal(fa, fm) and np.array_equal(f2a, f2m), f"request {k} differs alone vs mix"
    for k in (0, 2, 4):
        mol, T, g = reqs[k]
        oracle_sample_check(oracle_mod, f"request {k}", mol, T, g, alone[k][0], alone[k][1], precision, seed=k)


def test_molecule_cache_reuses_loaded_molecule():
    """A request on a molecule that an idle context already holds is given
    that context and skips the molecule load; with new transitions and a new
    grid its result equals a fresh context's bit for bit."""
    import torch  # noqa: F401
    from paper_2512_18010_amd import binding
    (mol, T1, g1), (_, _, g2) = requests(77, 2)
    rng = np.random.Generator(np.random.PCG64(78))
    T2 = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 3)
    with binding.Server(0, 0, max_inflight=2) as srv:
        status, _, _, _ = srv.wait(srv.submit(mol, T1, g1, screen_eps=1e-9))
        assert status == binding.SCFF_OK
        hits0 = srv.stats()["mol_cache_hits"]
        status, _, f, f2 = srv.wait(srv.submit(mol, T2, g2, screen_eps=1e-9))
        assert status == binding.SCFF_OK
        st = srv.stats()
    log("stats", st)
    assert hits0 == 0 and st["mol_cache_hits"] == 1
    with binding.Context(0) as ctx:
        ctx.load_molecule(mol)
        ctx.load_transitions(T2)
        ctx.set_options(1e-9, 1.0)
        fr, f2r = ctx.eval_grid_host(g2, "fp32")
    assert np.array_equal(f, fr) and np.array_equal(f2, f2r)


def test_failing_requests_fail_alone_on_the_device():
    """On a real device the molecule is validated by its load in prep: a
    request with a negative exponent and one with an unknown precision fail
    with SCFF_EINVAL, the requests around them complete and match a fresh
    context, and a context whose load failed is not reused as if it held
    the bad molecule."""
    import dataclasses
    import torch  # noqa: F401
    from paper_2512_18010_amd import binding
    (mol, T, g), (mol2, T2, g2) = requests(99, 2)
    bad_exps = mol.exps.copy()
    bad_exps[0] = -1.0
    bad = dataclasses.replace(mol, exps=bad_exps)
    with binding.Server(0, 0, max_inflight=2) as srv:
        t_ok1 = srv.submit(mol, T, g, screen_eps=1e-9)
        t_bad = srv.submit(bad, T, g, screen_eps=1e-9)
        t_prec = srv.submit(mol2, T2, g2, precision_code=7)
        t_ok2 = srv.submit(mol2, T2, g2, screen_eps=1e-9)
        r1, rb, rp, r2 = (srv.wait(t) for t in (t_ok1, t_bad, t_prec, t_ok2))
        st = srv.stats()
    assert rb[0] == binding.SCFF_EINVAL and rp[0] == binding.SCFF_EINVAL
    assert r1[0] == binding.SCFF_OK and r2[0] == binding.SCFF_OK
    assert st["failed"] == 2 and st["completed"] == 2
    for (m, TT, gg), res in (((mol, T, g), r1), ((mol2, T2, g2), r2)):
        with binding.Context(0) as ctx:
            ctx.load_molecule(m)
            ctx.load_transitions(TT)
            ctx.set_options(1e-9, 1.0)
            f, f2 = ctx.eval_grid_host(gg, "fp32")
        assert np.array_equal(res[2], f) and np.array_equal(res[3], f2)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_graph_replays_match_eager(precision):
    """Requests of one shape submitted one after another each run as a batch
    of the same launch topology, so the runner replays one executable graph
    with updated parameters; every replay (new transitions each time, eager
    work of the caller's own in between) is bit-identical to a plain context
    evaluation of the same request."""
    import torch
    from paper_2512_18010_amd import binding
    (mol, T0, g), = requests(31, 1)
    rng = np.random.Generator(np.random.PCG64(32))
    Ts = [wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 5) for _ in range(5)]
    results = []
    with binding.Server(0, 0, max_inflight=2) as srv:
        for T in Ts:
            status, _, f, f2 = srv.wait(srv.submit(mol, T, g, precision=precision, screen_eps=1e-9))
            assert status == binding.SCFF_OK
            results.append((f.copy(), f2.copy()))
            x = torch.ones(1 << 20, device="cuda")
            torch.cuda.synchronize()
            assert float(x.sum()) == float(1 << 20)   # eager device work between the replays
        st = srv.stats()
    log("stats", st)
    assert st["graphs_updated"] >= 1, st
    with binding.Context(0) as ctx:
        ctx.load_molecule(mol)
        ctx.set_options(1e-9, 1.0)
        for T, (f, f2) in zip(Ts, results):
            ctx.load_transitions(T)
            fe, f2e = ctx.eval_grid_host(g, precision)
            assert np.array_equal(f, fe) and np.array_equal(f2, f2e)


def test_batches_share_launches_and_budget_caps_admission():
    """Sixteen requests submitted at once under a budget that holds only a
    few of them: they run in batches of several requests (fewer batch
    launches than requests), the admitted bytes never exceed the budget, and
    every result equals its run alone."""
    import torch  # noqa: F401
    from paper_2512_18010_amd import binding
    reqs = requests(404, 16)
    alone = []
    with binding.Server(0, 0, max_inflight=8) as srv:
        for (mol, T, g) in reqs:
            status, _, f, f2 = srv.wait(srv.submit(mol, T, g, screen_eps=1e-9))
            assert status == binding.SCFF_OK
            alone.append((f.copy(), f2.copy()))
        fp = srv.stats()["peak_admitted_bytes"]
    budget = int(3 * fp)
    with binding.Server(0, budget, max_inflight=8) as srv:
        tickets = [srv.submit(mol, T, g, screen_eps=1e-9) for (mol, T, g) in reqs]
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
    log("stats", st)
    assert st["peak_admitted_bytes"] <= budget
    assert st["batches"] < st["batched_requests"] == 16, st
    for k, ((fa, f2a), (status, _, fm, f2m)) in enumerate(zip(alone, mixed)):
        assert status == binding.SCFF_OK
        assert np.array_equal(fa, fm) and np.array_equal(f2a, f2m), f"request {k} differs alone vs batched"
