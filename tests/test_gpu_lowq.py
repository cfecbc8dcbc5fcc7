"""GPU tests of the FP64 V-tensor paths through the C ABI: separable
integrals (paper Sec. 5.3) against the oracle's full grid weighted and
summed in FP64, and the low-momentum limit (Sec. 6): transition dipoles
against the oracle's Richardson derivative of Im f at q = 0, oscillator
strengths, and the angular-average fit A + B q^2 + C q^4."""
import os
import sys

import numpy as np
import pytest

import workload as wl
from tests.metrics import report

pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    import torch  # noqa: F401
    from paper_2512_18010_amd import binding
    ctx = binding.Context(0)
    yield ctx
    ctx.close()


def weights(rng, n):
    return rng.normal(size=n) + 1j * rng.normal(size=n)


@pytest.mark.parametrize("cfg,n,eps,tol", [(0, (13, 11, 17), 0.0, 1e-10), (1, (16, 15, 17), 0.0, 1e-10),
                                          (1, (16, 15, 17), 1e-9, 1e-7)])
def test_separable_matches_oracle_grid_sum(eng, oracle_mod, cfg, n, eps, tol):
    """sum wx wy wz f over a ragged grid, per transition: the engine's FP64
    separable evaluation against the oracle's FP64 grid summed with the same
    weights, relative to sum |w| |f|."""
    W = wl.make_config(cfg)
    g = wl.Grid(n=n, qmin=(-5.0, -4.5, -5.5), qmax=(5.0, 4.0, 5.5))
    rng = np.random.Generator(np.random.PCG64(700 + cfg))
    wx, wy, wz = (weights(rng, n[a]) for a in range(3))
    eng.load_molecule(W.mol)
    eng.load_transitions(W.T)
    eng.set_options(eps, 1.0)
    out = eng.eval_separable(g, wx, wy, wz)
    f = oracle_mod.eval_grid(W.mol, W.T, g, n_threads=NTH)
    wq = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
    ref = np.einsum("xyz,sxyz->s", wq, f)
    scale = np.einsum("xyz,sxyz->s", np.abs(wq), np.abs(f))
    err = np.abs(out - ref) / scale
    report(f"[separable cfg{cfg} {n} eps={eps:g}] relative to sum|w||f|: " + " ".join(f"{x:.1e}" for x in err))
    assert err.max() <= tol, err


def test_separable_rejects_bad_weights(eng):
    from paper_2512_18010_amd import binding
    W = wl.make_config(0)
    g = wl.Grid(n=(4, 5, 6), qmin=(-1.0,) * 3, qmax=(1.0,) * 3)
    eng.load_molecule(W.mol)
    eng.load_transitions(W.T)
    eng.set_options(0.0, 1.0)
    wx = np.ones(4, complex)
    wx[2] = np.nan
    with pytest.raises(binding.ScffError) as ei:
        eng.eval_separable(g, wx, np.ones(5), np.ones(6))
    assert ei.value.code == binding.SCFF_EINVAL


def richardson_dipole(oracle_mod, mol, T):
    """grad_q Im f at q = 0 from central differences of the oracle (h, h/2)."""
    ns = T.shape[0]
    mu = np.zeros((ns, 3))
    for ax in range(3):
        def d(h):
            e = np.zeros((2, 3))
            e[0, ax], e[1, ax] = h, -h
            f = oracle_mod.eval_points(mol, T, e, n_threads=NTH)
            return (f[:, 0].imag - f[:, 1].imag) / (2 * h)
        h = 2e-3
        mu[:, ax] = (4 * d(h / 2) - d(h)) / 3.0
    return mu


@pytest.mark.parametrize("cfg", [0, 1])
def test_dipole_matches_oracle(eng, oracle_mod, cfg):
    W = wl.make_config(cfg)
    eng.load_molecule(W.mol)
    eng.load_transitions(W.T)
    eng.set_options(0.0, 1.0)
    dE = 0.1 + 0.02 * np.arange(W.T.shape[0])
    mu, f0 = eng.dipole(dE)
    ref = richardson_dipole(oracle_mod, W.mol, W.T)
    err = np.abs(mu - ref).max(axis=1) / np.abs(ref).max(axis=1)
    report(f"[dipole cfg{cfg}] relative to max|mu_s|: " + " ".join(f"{x:.1e}" for x in err))
    assert err.max() <= 1e-7, err
    np.testing.assert_allclose(f0, 2.0 / 3.0 * dE * np.sum(ref ** 2, axis=1), rtol=1e-6)
    # spin factor scales mu linearly
    eng.set_options(0.0, np.sqrt(2.0))
    mu2, _ = eng.dipole()
    np.testing.assert_allclose(mu2, np.sqrt(2.0) * mu, rtol=1e-12, atol=1e-14 * np.abs(mu).max())


def test_dipole_fit_reconstructs_oscillator_strength(eng, oracle_mod):
    """With S-orthonormal orbitals (C = S^{-1/2} Q) every transition has
    f(0) = 0, so the fit's B is |mu|^2 / 3 and its f0 = 2 dE B matches the
    analytic (2/3) dE |mu|^2 (to the fit's truncation at q^4 over
    |q| <= 0.05 a.u.); A vanishes to the same order."""
    W = wl.make_config(0)
    mol = W.mol
    S = oracle_mod.pair_matrix(mol, np.zeros(3)).real
    ev, U = np.linalg.eigh(S)
    Sm12 = U @ np.diag(ev ** -0.5) @ U.T
    rng = np.random.Generator(np.random.PCG64(808))
    Q, R = np.linalg.qr(rng.normal(size=(mol.nbf, mol.nbf)))
    C = Sm12 @ (Q * np.sign(np.diag(R))[None, :])
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 3, C=C)
    eng.load_molecule(mol)
    eng.load_transitions(T)
    eng.set_options(0.0, 1.0)
    dE = np.array([0.15, 0.2, 0.3])
    mu, f0 = eng.dipole(dE)
    f_zero = oracle_mod.eval_points(mol, T, np.zeros((1, 3)), n_threads=NTH)[:, 0]
    assert np.abs(f_zero).max() <= 1e-10 * np.abs(mu).max()
    coef, f0_fit = eng.dipole_fit(0.05, dE)
    rel = np.abs(f0_fit / f0 - 1.0)
    report("[dipole fit q_fit=0.05] |f0_fit/f0 - 1|: " + " ".join(f"{x:.1e}" for x in rel))
    assert rel.max() <= 1e-3, (f0_fit, f0)
    # A is the fit's constant: zero up to the truncation of the q^6 terms
    assert np.abs(coef[:, 0]).max() <= 1e-5 * np.abs(coef[:, 1]).max() * 0.05 ** 2
