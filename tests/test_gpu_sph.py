"""GPU parity of the spherical method (Sec. 4 eqs. SphericalMethod, RTensor;
Sec. 5.4; App. B) through the C ABI.

The engine's R_lm(q) (FP64, exact up to rounding) is compared with the
oracle's projection of the Cartesian f onto the harmonics (a quadrature of
high enough order that its error is below 1e-12), the angular grid (FP32
output) with the oracle's truncated sum of its own R, the angular average
with sum |R|^2 / 4 pi, and at a large lmax the grid with the Cartesian f
itself.  Sizes: the config-0 molecule in full; the config-1 molecule with
its 12 transitions at lmax = 24 on one radius.
"""
import os
import sys

import numpy as np
import pytest

import workload as wl
from tests.metrics import errors, report

pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)
TOL_R = 1e-9      # FP64 path, relative to max |R|
TOL_GRID = 1e-6   # FP32 grid output, peak-normalised |f|^2


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


def load(eng, mol, T, spin=1.0):
    eng.load_molecule(mol)
    eng.load_transitions(T)
    eng.set_options(0.0, spin)


def n_theta_for(mol, q, lmax):
    """Gauss-Legendre order of the oracle's projection: the rule is exact for
    harmonics of total degree < 2 n, and f on the sphere of radius q has no
    weight above degree ~ e q r_max / 2 + 20 (its coefficients fall like
    j_l(q r) < 1e-15 there), so n >= (lmax + that) / 2 + 2 leaves the
    projections onto l <= lmax unaliased."""
    rmax = float(np.linalg.norm(mol.xyz, axis=1).max()) + 3.0
    return int((lmax + np.e * q * rmax / 2 + 24) / 2) + 2


def oracle_R(oracle_mod, mol, T, qs, lmax, spin=1.0):
    out = []
    for q in qs:
        out.append(oracle_mod.spherical_R(mol, T, [q], lmax, n_theta_for(mol, q, lmax), spin_factor=spin,
                                          n_threads=NTH))
    return np.concatenate(out, axis=1)


def r_error(R, Rref):
    ns = Rref.shape[0]
    return np.abs(R - Rref).reshape(ns, -1).max(axis=1) / np.abs(Rref).reshape(ns, -1).max(axis=1)


@pytest.mark.parametrize("n_states", [1, 3])
def test_R_grid_and_average_match_oracle(eng, oracle_mod, n_states):
    W = wl.make_config(0)
    T = W.T
    if n_states > 1:
        rng = np.random.Generator(np.random.PCG64(31))
        T = wl.make_transitions(rng, W.mol.nbf, wl.n_occupied(W.mol.Z), n_states)
    load(eng, W.mol, T, spin=np.sqrt(2.0))
    lmax = 12
    qs = np.array([0.0, 0.7, 2.0, 4.5])
    nt, npf = 9, 14
    R, f, f2, avg = eng.eval_spherical_host(lmax, qs, nt, npf, want_R=True, want_f=True, want_f2=True,
                                            want_avg=True)
    Rref = oracle_R(oracle_mod, W.mol, T, qs, lmax, spin=np.sqrt(2.0))
    eR = r_error(R, Rref)
    th = np.pi * np.arange(nt) / (nt - 1)
    ph = 2 * np.pi * np.arange(npf) / npf
    fref = oracle_mod.spherical_grid(Rref, lmax, th, ph)
    ns = T.shape[0]
    eg = errors(f.reshape(ns, -1), fref.reshape(ns, -1))
    aref = oracle_mod.angular_average_from_R(Rref)
    ea = np.abs(avg - aref).max() / aref.max()
    log(f"[sph cfg0 {ns} states] R {eR.max():.2e} grid |f|^2 {eg['f2_peak_norm'].max():.2e} avg {ea:.2e}")
    report(f"[sph cfg0 {ns} states lmax 12] R relative per transition: " + " ".join(f"{x:.1e}" for x in eR))
    assert eR.max() <= TOL_R, eR
    assert eg["f2_peak_norm"].max() <= TOL_GRID, eg["f2_peak_norm"]
    np.testing.assert_allclose(f2, np.abs(f) ** 2, rtol=2e-6, atol=1e-12 * np.abs(f).max() ** 2)
    assert ea <= TOL_R
    # q = 0: only R_00 = sqrt(4 pi) f(0)
    f0 = oracle_mod.eval_points(W.mol, T, np.zeros((1, 3)), spin_factor=np.sqrt(2.0))[:, 0]
    np.testing.assert_allclose(R[:, 0, 0], np.sqrt(4 * np.pi) * f0, rtol=1e-9, atol=1e-12 * np.abs(R).max())


def test_large_lmax_grid_approaches_cartesian_f(eng, oracle_mod):
    """With lmax = 40 the spherical grid reproduces the Cartesian form factor
    at the same points (config 0, |q| <= 2)."""
    W = wl.make_config(0)
    load(eng, W.mol, W.T)
    qs = np.array([0.8, 2.0])
    nt, npf = 7, 10
    _, f, _, _ = eng.eval_spherical_host(40, qs, nt, npf, want_R=False, want_f=True, want_avg=False)
    th = np.pi * np.arange(nt) / (nt - 1)
    ph = 2 * np.pi * np.arange(npf) / npf
    Q, TH, PH = np.meshgrid(qs, th, ph, indexing="ij")
    pts = np.stack([Q * np.sin(TH) * np.cos(PH), Q * np.sin(TH) * np.sin(PH), Q * np.cos(TH)], axis=-1).reshape(-1, 3)
    ref = oracle_mod.eval_points(W.mol, W.T, pts)
    e = errors(f.reshape(1, -1), ref)
    log(f"[sph lmax 40 vs Cartesian] |f|^2 {e['f2_peak_norm'].max():.2e}")
    assert e["f2_peak_norm"].max() <= TOL_GRID


def test_benchmark_molecule_R(eng, oracle_mod):
    """Config-1 molecule and its 12 transitions at lmax = 24 (the benchmark's
    angular order) on one radius: every R_lm against the oracle's quadrature."""
    W = wl.make_config(1)
    load(eng, W.mol, W.T)
    qs = np.array([1.5])
    R, _, _, avg = eng.eval_spherical_host(24, qs)
    Rref = oracle_R(oracle_mod, W.mol, W.T, qs, 24)
    eR = r_error(R, Rref)
    log(f"[sph cfg1 lmax 24] R {eR.max():.2e}")
    report("[sph cfg1 lmax 24, q = 1.5] R relative per transition: " + " ".join(f"{x:.1e}" for x in eR))
    assert eR.max() <= TOL_R, eR
    np.testing.assert_allclose(avg, oracle_mod.angular_average_from_R(Rref), rtol=1e-9)


def test_device_outputs_match_host(eng):
    import torch
    W = wl.make_config(0)
    load(eng, W.mol, W.T)
    qs = np.array([0.5, 1.5, 3.0])
    lmax, nt, npf = 8, 5, 8
    R, f, f2, avg = eng.eval_spherical_host(lmax, qs, nt, npf, want_R=True, want_f=True, want_f2=True)
    df = torch.empty((1, 3, nt, npf, 2), dtype=torch.float32, device="cuda")
    df2 = torch.empty((1, 3, nt, npf), dtype=torch.float32, device="cuda")
    dR = torch.empty((1, 3, (lmax + 1) ** 2, 2), dtype=torch.float64, device="cuda")
    davg = torch.empty((1, 3), dtype=torch.float64, device="cuda")
    eng.eval_spherical_device(lmax, qs, nt, npf, df, df2, dR, davg)
    torch.cuda.synchronize()
    Rd = dR.cpu().numpy()
    assert np.array_equal(Rd[..., 0] + 1j * Rd[..., 1], R)
    fd = df.cpu().numpy()
    assert np.array_equal(fd[..., 0] + 1j * fd[..., 1], f.astype(np.complex64))
    assert np.array_equal(df2.cpu().numpy(), f2)
    assert np.array_equal(davg.cpu().numpy(), avg)


def test_argument_errors(eng):
    from paper_2512_18010_amd import binding
    W = wl.make_config(0)
    load(eng, W.mol, W.T)
    for args in [dict(lmax=-1, qs=[1.0]), dict(lmax=49, qs=[1.0]), dict(lmax=4, qs=[-1.0]),
                 dict(lmax=4, qs=[np.nan]), dict(lmax=4, qs=[1.0], n_theta=1, n_phi=4, want_f=True)]:
        with pytest.raises(binding.ScffError) as ei:
            eng.eval_spherical_host(**args)
        assert ei.value.code == binding.SCFF_EINVAL
    with pytest.raises(binding.ScffError) as ei:
        eng.eval_spherical_host(4, [1.0], want_R=False, want_avg=False)
    assert ei.value.code == binding.SCFF_EINVAL
    fresh = binding.Context(0)
    try:
        with pytest.raises(binding.ScffError) as ei:
            fresh.eval_spherical_host(4, [1.0])
        assert ei.value.code == binding.SCFF_ESTATE
    finally:
        fresh.close()
