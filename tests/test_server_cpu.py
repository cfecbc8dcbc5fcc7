"""Scheduler of the request server, exercised in its no-GPU test mode
(device = -1): admission by footprint, FIFO order, cancellation, error
isolation, refusal of requests larger than the budget."""
import numpy as np
import pytest

import workload as wl
from paper_2512_18010_amd import binding


def small_request(rng, n_heavy=2, N=10, ns=2):
    mol = wl.make_molecule(rng, n_heavy, 1, layout="box", box_A=3.0, with_d=False, h_p=False)
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), ns)
    g = wl.Grid(n=(N, N, N), qmin=(-4.0,) * 3, qmax=(4.0,) * 3)
    return mol, T, g


def footprint(ns, N):
    return N * N * N * ns * 12    # test-mode footprint: outputs only


def test_admission_respects_budget_and_slots():
    rng = np.random.Generator(np.random.PCG64(1))
    budget = int(2.5 * footprint(2, 10))
    with binding.Server(-1, budget, max_inflight=4) as srv:
        tickets = [srv.submit(*small_request(rng)) for _ in range(12)]
        for t in tickets:
            status, lat, _, _ = srv.wait(t)
            assert status == binding.SCFF_OK
            assert lat > 0
        st = srv.stats()
    assert st["completed"] == 12 and st["failed"] == 0
    assert st["peak_admitted_bytes"] <= budget
    assert st["peak_inflight"] <= 2        # only two requests fit the budget at once
    assert st["admitted_bytes"] == 0 and st["inflight"] == 0


def test_inflight_limit():
    rng = np.random.Generator(np.random.PCG64(2))
    with binding.Server(-1, 0, max_inflight=3) as srv:
        ts = [srv.submit(*small_request(rng)) for _ in range(10)]
        for t in ts:
            assert srv.wait(t)[0] == binding.SCFF_OK
        assert srv.stats()["peak_inflight"] <= 3


def test_error_isolation():
    rng = np.random.Generator(np.random.PCG64(3))
    with binding.Server(-1, 0, max_inflight=2) as srv:
        good1 = srv.submit(*small_request(rng))
        bad = srv.submit(*small_request(rng), precision_code=7)
        mol, T, g = small_request(rng)
        mol.shell_atom[0] = 99                    # shell on a missing atom
        bad2 = srv.submit(mol, T, g)
        good2 = srv.submit(*small_request(rng))
        assert srv.wait(good1)[0] == binding.SCFF_OK
        assert srv.wait(bad)[0] == binding.SCFF_EINVAL
        assert srv.wait(bad2)[0] == binding.SCFF_EINVAL
        assert srv.wait(good2)[0] == binding.SCFF_OK
        st = srv.stats()
        assert st["failed"] == 2 and st["completed"] == 2


def test_request_larger_than_budget_is_refused():
    rng = np.random.Generator(np.random.PCG64(4))
    with binding.Server(-1, footprint(2, 10) // 2, max_inflight=2) as srv:
        t = srv.submit(*small_request(rng))
        assert srv.wait(t)[0] == binding.SCFF_ENOMEM


def test_cancel_and_timeout():
    rng = np.random.Generator(np.random.PCG64(5))
    with binding.Server(-1, footprint(2, 10), max_inflight=1) as srv:
        ts = [srv.submit(*small_request(rng)) for _ in range(20)]
        last = ts[-1]
        with pytest.raises(binding.ScffError) as ei:
            srv.wait(last, timeout_ns=0)
        assert ei.value.code == binding.SCFF_EBUSY
        srv.cancel(last)
        assert srv.wait(last)[0] == binding.SCFF_ECANCELLED
        for t in ts[:-1]:
            assert srv.wait(t)[0] == binding.SCFF_OK
        with pytest.raises(binding.ScffError):
            srv.wait(ts[0])                      # a ticket is waited for once


def test_submit_validation():
    rng = np.random.Generator(np.random.PCG64(6))
    mol, T, g = small_request(rng)
    with binding.Server(-1, 0, max_inflight=1) as srv:
        with pytest.raises(binding.ScffError):
            srv.submit(mol, T, g, want_f=False, want_f2=False)
        bad = np.zeros((33,) + T.shape[1:])
        with pytest.raises(binding.ScffError):
            srv.submit(mol, bad, g)


def test_stage_times_add_up_to_latency():
    """The per-stage times the server reports (waiting for prep, prep,
    waiting for a run slot, run, host copy) are non-negative, include the
    test mode's 2 ms of run per request, and sum to the requests' latencies."""
    rng = np.random.Generator(np.random.PCG64(9))
    with binding.Server(-1, 0, max_inflight=2) as srv:
        tickets = [srv.submit(*small_request(rng)) for _ in range(10)]
        lat_ns = 0
        for t in tickets:
            status, lat, _, _ = srv.wait(t)
            assert status == binding.SCFF_OK
            lat_ns += lat
        st = srv.stats()
    ns = st["ns_stage"]
    assert all(v >= 0 for v in ns)
    assert ns[3] >= 10 * 2_000_000
    assert abs(sum(ns) - lat_ns) <= 1000 * 10   # rounding to whole nanoseconds per stage
