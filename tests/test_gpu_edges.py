"""GPU edge cases of the grid path, through the C ABI, against the FP64
oracle: the largest state count (32 transitions, two MFMA row blocks),
degenerate grids (one point along an axis, lines through q = 0), a single
atom (same-centre pairs only), a molecule of s shells only, and an all-zero
transition density (f must be exactly zero).  Tolerances as in the parity
tests: peak-normalised |f|^2 within 1e-6 (FP32) and 1e-4 (split-BF16).
"""
import os
import sys

import numpy as np
import pytest

import workload as wl
from tests.metrics import TOL_F2, errors

pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    import torch  # noqa: F401  (initialises HIP the same way the benchmark does)
    from paper_2512_18010_amd import binding
    ctx = binding.Context(0)
    yield ctx
    ctx.close()


def run(eng, mol, T, grid, precision, eps=0.0):
    eng.load_molecule(mol)
    eng.load_transitions(T)
    eng.set_options(eps, 1.0)
    return eng.eval_grid_host(grid, precision)


def check(name, f, f2, ref, precision):
    e = errors(f, ref)
    np.testing.assert_allclose(f2, np.abs(f) ** 2, rtol=2e-6, atol=1e-12 * np.abs(f).max() ** 2)
    log(f"[{name}] {precision}: max peak-normalised |f|^2 err {e['f2_peak_norm'].max():.3e}")
    assert e["f2_peak_norm"].max() <= TOL_F2[precision], e["f2_peak_norm"]


def h2_s_only():
    """Two H atoms with two contracted s shells each (no p, no d)."""
    return wl.Molecule(Z=np.array([1, 1]), xyz=np.array([[0.0, 0.0, -0.7], [0.1, 0.2, 0.7]]),
                       shell_atom=np.array([0, 0, 1, 1], np.int32), shell_l=np.zeros(4, np.int32),
                       shell_nprim=np.array([3, 1, 3, 1], np.int32),
                       exps=np.array([13.0, 1.96, 0.44, 0.12, 13.0, 1.96, 0.44, 0.12]),
                       coefs=np.array([0.02, 0.14, 0.48, 1.0, 0.02, 0.14, 0.48, 1.0]))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_32_states_full_grid(eng, oracle_mod, precision):
    """The maximum state count: both 16-row MFMA blocks full."""
    rng = np.random.Generator(np.random.PCG64(321))
    mol = wl.make_molecule(rng, 3, 2, layout="box", box_A=3.0)
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 32)
    grid = wl.Grid(n=(5, 9, 19), qmin=(-5.0, -4.5, -6.0), qmax=(4.0, 5.0, 6.0))
    log("case 32 states", grid.n, mol.nbf)
    f, f2 = run(eng, mol, T, grid, precision)
    assert f.shape == (32,) + grid.n
    check("32 states 5x9x19", f, f2, oracle_mod.eval_grid(mol, T, grid, n_threads=NTH), precision)


@pytest.mark.parametrize("n,qmin,qmax", [
    ((1, 1, 7), (0.0, 0.0, -3.0), (0.0, 0.0, 3.0)),      # the q_z axis through q = 0
    ((1, 13, 1), (0.5, -6.0, -0.25), (0.5, 6.0, -0.25)),  # one q_y line
    ((9, 1, 1), (-4.0, 0.0, 0.0), (4.0, 0.0, 0.0)),       # the q_x axis through q = 0
    ((1, 1, 1), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),        # the single point q = 0
])
def test_degenerate_grids(eng, oracle_mod, n, qmin, qmax):
    """Axes with one point (grid spacing zero) and the point q = 0.  The
    error of |f|^2 is normalised by the peak of |f|^2 over these points and
    the q_z line through q = 0: on the single point q = 0 alone, f(0) =
    Tr(T S) is a cancelling sum much smaller than the transition's scale, and
    normalising by it would measure the error relative to that cancellation."""
    W = wl.make_config(0)
    grid = wl.Grid(n=n, qmin=qmin, qmax=qmax)
    line = wl.Grid(n=(1, 1, 7), qmin=(0.0, 0.0, -3.0), qmax=(0.0, 0.0, 3.0))
    log("case degenerate grid", n)
    f, f2 = run(eng, W.mol, W.T, grid, "fp32")
    ref = oracle_mod.eval_grid(W.mol, W.T, grid, n_threads=NTH)
    ref_line = oracle_mod.eval_grid(W.mol, W.T, line, n_threads=NTH)
    np.testing.assert_allclose(f2, np.abs(f) ** 2, rtol=2e-6, atol=1e-12 * np.abs(f).max() ** 2)
    ns = ref.shape[0]
    peak2 = np.maximum(np.abs(ref.reshape(ns, -1)).max(axis=1), np.abs(ref_line.reshape(ns, -1)).max(axis=1)) ** 2
    err = np.abs(np.abs(f.reshape(ns, -1)) ** 2 - np.abs(ref.reshape(ns, -1)) ** 2).max(axis=1) / peak2
    log(f"[grid {n}] fp32: |f|^2 error / line peak {err.max():.3e}")
    assert err.max() <= TOL_F2["fp32"], err


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_single_atom(eng, oracle_mod, precision):
    """One heavy atom (s, p, d shells): every pair is a same-centre pair."""
    rng = np.random.Generator(np.random.PCG64(17))
    mol = wl.make_molecule(rng, 1, 0, layout="box", box_A=1.0)
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 5)
    grid = wl.Grid(n=(11, 6, 23), qmin=(-5.0, -5.0, -5.0), qmax=(5.0, 4.0, 5.0))
    log("case single atom", mol.nbf)
    f, f2 = run(eng, mol, T, grid, precision)
    check("single atom", f, f2, oracle_mod.eval_grid(mol, T, grid, n_threads=NTH), precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_s_shells_only(eng, oracle_mod, precision):
    """A molecule with s shells only (all power pairs (0, 0))."""
    rng = np.random.Generator(np.random.PCG64(23))
    mol = h2_s_only()
    T = wl.make_transitions(rng, mol.nbf, 1, 3)
    grid = wl.Grid(n=(7, 8, 17), qmin=(-4.0, -4.0, -4.0), qmax=(4.0, 4.0, 4.0))
    log("case s only")
    f, f2 = run(eng, mol, T, grid, precision)
    check("H2 s only", f, f2, oracle_mod.eval_grid(mol, T, grid, n_threads=NTH), precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("eps", [0.0, 1e-9])
def test_zero_transition_density(eng, precision, eps):
    """T = 0 gives exactly f = 0 and |f|^2 = 0: with eps = 0 every term is
    kept with zero weight, with eps > 0 every term is screened out (no pair
    left; the evaluation runs on one padded unit of zero rows)."""
    W = wl.make_config(0)
    T = np.zeros((2,) + W.T.shape[1:])
    grid = wl.Grid(n=(6, 7, 18), qmin=(-5.0,) * 3, qmax=(5.0,) * 3)
    f, f2 = run(eng, W.mol, T, grid, precision, eps=eps)
    info = eng.query()
    if eps > 0:
        assert info["pairs_kept"] == 0 and info["prim_comp_pairs_kept"] == 0
    assert np.all(f == 0) and np.all(f2 == 0)


@pytest.mark.parametrize("case", range(8))
def test_random_cases(eng, oracle_mod, case):
    """Seeded random problems: 1-4 heavy atoms (+ H), 1-32 transitions, grid
    sizes 1-21 per axis with asymmetric bounds, screening off or on, both
    precisions; every grid point against the oracle (screened cases keep the
    oracle unscreened: the screening bound is part of the error budget)."""
    rng = np.random.Generator(np.random.PCG64(7000 + case))
    n_heavy = int(rng.integers(1, 5))
    mol = wl.make_molecule(rng, n_heavy, int(rng.integers(0, n_heavy + 1)), layout="box", box_A=3.0,
                           with_d=bool(rng.integers(0, 2)))
    ns = int(rng.integers(1, 33))
    T = wl.make_transitions(rng, mol.nbf, min(wl.n_occupied(mol.Z), mol.nbf - 1), ns)
    n = tuple(int(v) for v in rng.integers(1, 22, size=3))
    lo = rng.uniform(-7.0, -1.0, size=3)
    hi = rng.uniform(1.0, 7.0, size=3)
    grid = wl.Grid(n=n, qmin=tuple(lo), qmax=tuple(hi))
    precision = "bf16x3" if case % 2 else "fp32"
    eps = 0.0 if case % 3 == 0 else 1e-10
    log(f"case random {case}: heavy {n_heavy}, nbf {mol.nbf}, states {ns}, grid {n}, {precision}, eps {eps:g}")
    f, f2 = run(eng, mol, T, grid, precision, eps=eps)
    assert f.shape == (ns,) + n
    check(f"random {case}", f, f2, oracle_mod.eval_grid(mol, T, grid, n_threads=NTH), precision)
