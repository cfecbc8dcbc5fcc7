"""Pins for the oracle's FFT method (Sec. 3, eqs. PhiTDM, Falbega, continuFFT,
fftABC, qabc; Sec. 5.2; the Parseval check of Sec. 7).

They tie the transition density and the transform steps to closed forms, to
the analytic form factor (an independent route), to a direct DFT sum and to
Parseval's identity, so that a wrong normalisation, a dropped component, a
wrong sign of the corner phase, a mis-ordered frequency axis or a missing
pixel volume fails at least one of them.
"""
import dataclasses
import math

import numpy as np

import workload as wl
from tests.test_oracle_pins import mol_of


def small_smooth_molecule(seed, n_heavy=3, lo=0.3, hi=3.0):
    """A config-0-like molecule whose exponents lie in [lo, hi] bohr^-2, so a
    real-space grid of spacing ~0.2 bohr resolves every product of two
    primitives (exponent <= 2 hi) and a box with ~8 bohr of margin holds them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mol = wl.make_molecule(rng, n_heavy, n_heavy, layout="box", box_A=3.0)
    ex = np.exp(rng.uniform(np.log(lo), np.log(hi), size=mol.exps.shape[0]))
    mol = dataclasses.replace(mol, exps=ex)
    T = wl.make_transitions(rng, mol.nbf, wl.n_occupied(mol.Z), 2)
    return mol, T


def box_around(mol, margin, n):
    lo = mol.xyz.min(axis=0) - margin
    hi = mol.xyz.max(axis=0) + margin
    L = hi - lo
    return tuple(int(x) for x in n), tuple(lo), tuple(L)


def test_density_single_s_primitive_closed_form(oracle_mod):
    """One normalised s primitive: phi = (2a/pi)^{3/4} e^{-a r^2}, so
    Phi = s_f t (2a/pi)^{3/2} e^{-2a |r-A|^2}."""
    A = (0.3, -0.7, 1.1)
    a = 0.8
    mol = mol_of([A], [(0, 0, [a], [0.6])])
    T = np.array([[[1.7]]])
    rng = np.random.Generator(np.random.PCG64(1))
    r = rng.normal(size=(40, 3)) + np.array(A)
    phi = oracle_mod.density(mol, T, r, spin_factor=math.sqrt(2.0))[0]
    d2 = ((r - np.array(A)) ** 2).sum(axis=1)
    ref = math.sqrt(2.0) * 1.7 * (2 * a / math.pi) ** 1.5 * np.exp(-2 * a * d2)
    np.testing.assert_allclose(phi, ref, rtol=1e-13, atol=0)


def test_ao_values_p_and_d_normalisation(oracle_mod):
    """Single-primitive p and d shells: the normalised Cartesian components
    are N x^a y^b z^c e^{-a r^2} with N^2 = (2a/pi)^{3/2} (4a)^l / ((2a-1)!!(2b-1)!!(2c-1)!!):
    p: (4a)^{1/2}; d_xx: 4a/sqrt(3); d_xy: 4a (App. A with sigma^2 = 1/2a)."""
    A = np.array([0.2, 0.1, -0.4])
    a = 1.3
    mol = mol_of([A], [(0, 1, [a], [1.0]), (0, 2, [a], [0.4])])
    rng = np.random.Generator(np.random.PCG64(2))
    r = rng.normal(size=(25, 3)) * 0.8 + A
    phi = oracle_mod.ao_values(mol, r)
    d = r - A
    g = (2 * a / math.pi) ** 0.75 * np.exp(-a * (d ** 2).sum(axis=1))
    npz = math.sqrt(4 * a)
    ref = np.stack([npz * d[:, 0] * g, npz * d[:, 1] * g, npz * d[:, 2] * g,
                    4 * a / math.sqrt(3) * d[:, 0] ** 2 * g, 4 * a * d[:, 0] * d[:, 1] * g,
                    4 * a * d[:, 0] * d[:, 2] * g, 4 * a / math.sqrt(3) * d[:, 1] ** 2 * g,
                    4 * a * d[:, 1] * d[:, 2] * g, 4 * a / math.sqrt(3) * d[:, 2] ** 2 * g], axis=1)
    np.testing.assert_allclose(phi, ref, rtol=1e-13, atol=1e-15)


def test_density_integrates_to_f_at_zero(oracle_mod):
    """int Phi_s d^3r = f_s(0) = s_f Tr(T S): the trapezoid sum of the
    tabulated density (exponentially accurate for Gaussians on a fine, wide
    grid) against the analytic form factor at q = 0."""
    mol, T = small_smooth_molecule(11)
    n, xmin, L = box_around(mol, 8.0, (0, 0, 0))
    h = 0.2
    n = tuple(int(math.ceil(L[a] / h)) for a in range(3))
    L = tuple(n[a] * h for a in range(3))
    phi = oracle_mod.density_grid(mol, T, n, xmin, L)
    integral = phi.reshape(T.shape[0], -1).sum(axis=1) * h ** 3
    f0 = oracle_mod.eval_points(mol, T, np.zeros((1, 3)))[:, 0]
    assert np.abs(f0.imag).max() < 1e-14
    scale = (np.abs(phi).reshape(T.shape[0], -1).sum(axis=1) * h ** 3)
    err = np.abs(integral - f0.real) / scale
    assert err.max() < 1e-10, (integral, f0.real, err)


def test_fft_equals_direct_dft_sum(oracle_mod):
    """On tiny grids (odd and even sizes) the FFT route equals the defining
    sum f(q) = V_pix sum_abc Phi(x_abc) e^{+i q.x_abc} at q = 2 pi alpha / L."""
    mol, T = small_smooth_molecule(12, n_heavy=2)
    for n in [(6, 5, 4), (3, 8, 7)]:
        xmin = (-4.1, -3.7, -5.2)
        L = (9.0, 8.3, 10.1)
        f, phi = oracle_mod.fft_form_factor(mol, T, n, xmin, L)
        ax = oracle_mod.real_space_axes(n, xmin, L)
        X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
        x = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        q = oracle_mod.fft_q_axes(n, L)
        QX, QY, QZ = np.meshgrid(q[0], q[1], q[2], indexing="ij")
        qq = np.stack([QX.ravel(), QY.ravel(), QZ.ravel()], axis=1)
        vpix = np.prod(np.array(L) / np.array(n))
        ph = np.exp(1j * qq @ x.T)
        ref = vpix * (ph @ phi.reshape(T.shape[0], -1).T).T
        np.testing.assert_allclose(f.reshape(T.shape[0], -1), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_fft_converges_to_analytic_form_factor(oracle_mod):
    """On a grid of spacing h = 0.2 bohr in a box with 8 bohr of margin, the
    FFT method's f equals the analytic form factor at every q with
    |q_i| <= pi / (2h): the aliased copies sit >= 3 pi / (2h) away, where the
    Gaussian factor e^{-q^2/(4p)} (p <= 6) is ~1e-10, and the box truncation
    is e^{-0.6 * 64}.  Checked on a sample of such q plus the lowest ones."""
    mol, T = small_smooth_molecule(13)
    h = 0.2
    lo = mol.xyz.min(axis=0) - 8.0
    hi = mol.xyz.max(axis=0) + 8.0
    n = tuple(int(2 * math.ceil((hi[a] - lo[a]) / (2 * h))) for a in range(3))
    L = tuple(n[a] * h for a in range(3))
    f, phi = oracle_mod.fft_form_factor(mol, T, n, tuple(lo), L)
    q = oracle_mod.fft_q_axes(n, L)
    rng = np.random.Generator(np.random.PCG64(3))
    qlim = math.pi / (2 * h)
    idx = []
    for a in range(3):
        ok = np.nonzero(np.abs(q[a]) <= qlim)[0]
        idx.append(rng.choice(ok, size=40))
    idx = np.stack(idx, axis=1)
    idx = np.concatenate([idx, np.array([[n[0] // 2, n[1] // 2, n[2] // 2],
                                         [n[0] // 2 + 1, n[1] // 2, n[2] // 2 - 1]])], axis=0)
    qs = np.stack([q[0][idx[:, 0]], q[1][idx[:, 1]], q[2][idx[:, 2]]], axis=1)
    ref = oracle_mod.eval_points(mol, T, qs)
    got = f[:, idx[:, 0], idx[:, 1], idx[:, 2]]
    peak = np.abs(ref).max(axis=1, keepdims=True)
    err = np.abs(got - ref) / peak
    assert err.max() < 1e-9, err.max()


def test_parseval_identity_holds_on_the_grid(oracle_mod):
    """int |Phi|^2 d^3r = int |f|^2 d^3q / (2 pi)^3 (Sec. 7) holds exactly for
    the grid sums with V_pix and dq = 2 pi / L; a missing pixel volume or a
    wrong q spacing breaks it."""
    mol, T = small_smooth_molecule(14, n_heavy=2)
    n = (16, 12, 10)
    xmin = (-6.0, -5.5, -5.0)
    L = (13.0, 11.0, 10.5)
    f, phi = oracle_mod.fft_form_factor(mol, T, n, xmin, L)
    a, b = oracle_mod.parseval_sums(phi, f, n, L)
    np.testing.assert_allclose(a, b, rtol=1e-12)
