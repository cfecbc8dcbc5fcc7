"""GPU parity of the FFT method (Sec. 3, Sec. 5.2) through the C ABI.

Small boxes are compared element by element with the oracle's FFT method
(FP64 density on the same periodic grid, library FFT, the same frequency
order, pixel volume and corner phase): the transition density, f, |f|^2 and
both sides of Parseval's identity.  At the benchmark size (the config-1
molecule and transitions on 128^3) the density is checked on a seeded sample
of grid points against the oracle's density, and the transform against the
oracle's transform steps applied to the GPU's own density; the two stages
then cover the whole path.
"""
import ctypes
import dataclasses
import os
import sys

import numpy as np
import pytest

import workload as wl
from tests.metrics import TOL_FFT, TOL_FFT_BF16, errors, report

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


def load(eng, mol, T, spin=1.0):
    eng.load_molecule(mol)
    eng.load_transitions(T)
    eng.set_options(0.0, spin)


def compare(name, oracle_mod, mol, T, n, xmin, L, f, f2, phi, ps, spin=1.0, tol=TOL_FFT):
    f_ref, phi_ref = oracle_mod.fft_form_factor(mol, T, n, xmin, L, spin_factor=spin, n_threads=NTH)
    ns = T.shape[0]
    e = errors(f, f_ref)
    ephi = np.abs(phi.reshape(ns, -1) - phi_ref.reshape(ns, -1)).max(axis=1) / \
        np.abs(phi_ref.reshape(ns, -1)).max(axis=1)
    a, b = oracle_mod.parseval_sums(phi_ref, f_ref, n, L)
    eps_p = np.maximum(np.abs(ps[:, 0] / a - 1), np.abs(ps[:, 1] / b - 1))
    log(f"[{name}] |f|^2 {e['f2_peak_norm'].max():.2e} complex {e['complex'].max():.2e} "
        f"phi {ephi.max():.2e} parseval {eps_p.max():.2e}")
    report(f"[fft {name}] |f|^2 per transition: " + " ".join(f"{x:.2e}" for x in e["f2_peak_norm"]))
    np.testing.assert_allclose(f2, np.abs(f) ** 2, rtol=2e-6, atol=1e-12 * np.abs(f).max() ** 2)
    assert e["f2_peak_norm"].max() <= tol, e["f2_peak_norm"]
    assert ephi.max() <= tol, ephi
    assert eps_p.max() <= tol, (ps, a, b)
    # the GPU's own two Parseval sums agree (identity of the discrete transform)
    assert np.abs(ps[:, 0] / ps[:, 1] - 1).max() <= TOL_FFT


@pytest.mark.parametrize("n", [(16, 32, 8), (1, 16, 32), (32, 2, 16)])
def test_fft_small_boxes_match_oracle(eng, oracle_mod, n):
    """Config-0 molecule, 1 transition, on non-cubic boxes (including a
    one-point and a two-point axis): every element of phi, f, |f|^2."""
    W = wl.make_config(0)
    n, xmin, L = wl.fft_box(W.mol, n, margin_bohr=5.0, scale=1.5)
    load(eng, W.mol, W.T)
    f, f2, phi, ps = eng.eval_fft_host(n, xmin, L, want_phi=True)
    compare(f"cfg0 {n}", oracle_mod, W.mol, W.T, n, xmin, L, f, f2, phi, ps)


def test_fft_odd_state_count_and_spin(eng, oracle_mod):
    """Three transitions (two share a complex transform, the third is alone)
    with the paper's spin factor sqrt(2)."""
    W = wl.make_config(0)
    rng = np.random.Generator(np.random.PCG64(901))
    T = wl.make_transitions(rng, W.mol.nbf, wl.n_occupied(W.mol.Z), 3)
    n, xmin, L = wl.fft_box(W.mol, (16, 16, 16), margin_bohr=4.0, scale=2.0)
    load(eng, W.mol, T, spin=np.sqrt(2.0))
    f, f2, phi, ps = eng.eval_fft_host(n, xmin, L, want_phi=True)
    compare("cfg0 3 states", oracle_mod, W.mol, T, n, xmin, L, f, f2, phi, ps, spin=np.sqrt(2.0))


@pytest.mark.parametrize("n_heavy,n_states", [(20, 2), (30, 3), (36, 2)])
def test_fft_large_basis_tiles(eng, oracle_mod, n_heavy, n_states):
    """Bases of 380, 570 and 685 functions: 32-point tiles for the first,
    16-point tiles for the others (24, 36 and 43 row blocks of 16, so the four
    waves of a tile take different numbers of them)."""
    rng = np.random.Generator(np.random.PCG64(950 + n_heavy))
    mol = wl.make_molecule(rng, n_heavy, int(round(0.8 * n_heavy)), layout="box",
                           box_A=12.0 * (n_heavy / 30.0) ** (1 / 3))
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), n_states)
    n, xmin, L = wl.fft_box(mol, (8, 16, 16), margin_bohr=3.0, scale=1.0)
    load(eng, mol, T)
    f, f2, phi, ps = eng.eval_fft_host(n, xmin, L, want_phi=True)
    compare(f"{mol.nbf} bf", oracle_mod, mol, T, n, xmin, L, f, f2, phi, ps)


@pytest.mark.parametrize("n_heavy,n_states", [(4, 1), (20, 2), (36, 3)])
def test_fft_bf16x3_matches_oracle(eng, oracle_mod, n_heavy, n_states):
    """Split-BF16 density contraction: config-0-sized, 380- and 685-function
    bases (64-, 32- and 16-point tiles) against the oracle, element by
    element, at the split-BF16 tolerance."""
    rng = np.random.Generator(np.random.PCG64(970 + n_heavy))
    if n_heavy == 4:
        W = wl.make_config(0)
        mol, T, box = W.mol, W.T, (16, 32, 8)
    else:
        mol = wl.make_molecule(rng, n_heavy, int(round(0.8 * n_heavy)), layout="box",
                               box_A=12.0 * (n_heavy / 30.0) ** (1 / 3))
        T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), n_states)
        box = (8, 16, 16)
    n, xmin, L = wl.fft_box(mol, box, margin_bohr=3.0, scale=1.0)
    load(eng, mol, T, spin=np.sqrt(2.0))
    f, f2, phi, ps = eng.eval_fft_host(n, xmin, L, want_phi=True, precision="bf16x3")
    compare(f"bf16x3 {mol.nbf} bf", oracle_mod, mol, T, n, xmin, L, f, f2, phi, ps, spin=np.sqrt(2.0),
            tol=TOL_FFT_BF16)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_fft_benchmark_size_sampled(eng, oracle_mod, precision):
    """Config-1 molecule and its 12 transitions on the benchmark's 128^3 box:
    the density on 400 seeded grid points against the oracle's FP64 density,
    and f against the oracle's transform of the GPU's own density."""
    tol = TOL_FFT if precision == "fp32" else TOL_FFT_BF16
    W = wl.make_config(1)
    n, xmin, L = wl.fft_box(W.mol, (128, 128, 128))
    load(eng, W.mol, W.T)
    f, f2, phi, ps = eng.eval_fft_host(n, xmin, L, want_phi=True, precision=precision)
    ns = W.T.shape[0]
    rng = np.random.Generator(np.random.PCG64(77))
    idx = rng.integers(0, np.prod(n), size=400)
    # plus the points of largest |Phi| of each transition
    idx = np.concatenate([idx, np.abs(phi.reshape(ns, -1)).argmax(axis=1)])
    ax = oracle_mod.real_space_axes(n, xmin, L)
    ii = np.unravel_index(idx, n)
    pts = np.stack([ax[0][ii[0]], ax[1][ii[1]], ax[2][ii[2]]], axis=1)
    ref = oracle_mod.density(W.mol, W.T, pts, n_threads=NTH)
    got = phi.reshape(ns, -1)[:, idx]
    peak = np.abs(phi.reshape(ns, -1)).max(axis=1)
    ephi = np.abs(got - ref).max(axis=1) / peak
    f_ref, _ = oracle_mod.fft_form_factor(W.mol, W.T, n, xmin, L, phi=phi.astype(np.float64))
    e = errors(f, f_ref)
    log(f"[fft cfg1 128^3 {precision}] phi sampled {ephi.max():.2e}, transform |f|^2 {e['f2_peak_norm'].max():.2e}")
    report(f"[fft cfg1 128^3 {precision}] density, per transition: " + " ".join(f"{x:.2e}" for x in ephi))
    report(f"[fft cfg1 128^3 {precision}] transform |f|^2, per transition: " +
           " ".join(f"{x:.2e}" for x in e["f2_peak_norm"]))
    assert ephi.max() <= tol, ephi
    assert e["f2_peak_norm"].max() <= TOL_FFT, e["f2_peak_norm"]
    assert np.abs(ps[:, 0] / ps[:, 1] - 1).max() <= TOL_FFT


def test_fft_device_outputs_match_host(eng):
    """Device outputs on a torch stream equal the host outputs bit for bit."""
    import torch
    W = wl.make_config(0)
    n, xmin, L = wl.fft_box(W.mol, (16, 8, 32))
    load(eng, W.mol, W.T)
    f, f2, phi, _ = eng.eval_fft_host(n, xmin, L, want_phi=True, parseval=False)
    shape = (1,) + n
    df = torch.empty(shape + (2,), dtype=torch.float32, device="cuda")
    df2 = torch.empty(shape, dtype=torch.float32, device="cuda")
    dphi = torch.empty(shape, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    eng.eval_fft_device(n, xmin, L, df, df2, dphi, stream=s)
    s.synchronize()
    fd = df.cpu().numpy()
    assert np.array_equal(fd[..., 0] + 1j * fd[..., 1], f.astype(np.complex64))
    assert np.array_equal(df2.cpu().numpy(), f2)
    assert np.array_equal(dphi.cpu().numpy(), phi)


def test_fft_argument_errors(eng):
    from paper_2512_18010_amd import binding
    W = wl.make_config(0)
    load(eng, W.mol, W.T)
    n, xmin, L = wl.fft_box(W.mol, (16, 16, 16))
    for bad in [((12, 16, 16), xmin, L), ((16, 16, 2048), xmin, L), (n, xmin, (L[0], 0.0, L[2])),
                (n, (np.nan, 0.0, 0.0), L)]:
        with pytest.raises(binding.ScffError) as ei:
            eng.eval_fft_host(*bad)
        assert ei.value.code == binding.SCFF_EINVAL
    with pytest.raises(binding.ScffError) as ei:
        eng.eval_fft_host(n, xmin, L, want_f=False, want_f2=False, want_phi=False, parseval=False)
    assert ei.value.code == binding.SCFF_EINVAL
    g = binding.make_fft_grid(n, xmin, L)
    ps = np.empty((1, 2), np.float64)
    rc = binding.scff_eval_fft(eng._h, ctypes.byref(g), 7, None, None, None,
                               ps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, None)
    assert rc == binding.SCFF_EINVAL
    fresh = binding.Context(0)
    try:
        with pytest.raises(binding.ScffError) as ei:
            fresh.eval_fft_host(n, xmin, L)
        assert ei.value.code == binding.SCFF_ESTATE
    finally:
        fresh.close()
