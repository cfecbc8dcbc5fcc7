"""Pins for the FP64 oracle: closed forms, quadrature, the paper's Hermite form, invariants.

Each test ties the oracle to something other than itself, chosen so that a
plausible mistake (a dropped term, a wrong sign of the phase, a transposed
operand, a wrong normalisation, a mis-ordered component) fails at least one.
"""
import math

import numpy as np
import pytest

import workload as wl
from tests import paper_forms, quadrature

pytestmark = []


def mol_of(atoms, shells, Z=None):
    """atoms: [(x,y,z)], shells: [(atom, l, [exps], [coefs])]."""
    xyz = np.array(atoms, dtype=float).reshape(-1, 3)
    sa, sl, sn, ex, co = [], [], [], [], []
    for a, l, e, c in shells:
        sa.append(a)
        sl.append(l)
        sn.append(len(e))
        ex += list(e)
        co += list(c)
    if Z is None:
        Z = np.full(len(xyz), 6)
    return wl.Molecule(Z=np.asarray(Z), xyz=xyz, shell_atom=np.array(sa, np.int32),
                       shell_l=np.array(sl, np.int32), shell_nprim=np.array(sn, np.int32),
                       exps=np.array(ex, float), coefs=np.array(co, float))


def unit_T(nbf, m, n):
    T = np.zeros((1, nbf, nbf))
    T[0, m, n] = 1.0
    return T


RNG = np.random.Generator(np.random.PCG64(7))
QS = np.concatenate([np.zeros((1, 3)), RNG.uniform(-6, 6, size=(12, 3))])


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("alpha", [0.13, 1.7, 42.0])
def test_ss_same_centre_closed_form(oracle_mod, alpha):
    C = np.array([0.4, -1.1, 2.3])
    mol = mol_of([C], [(0, 0, [alpha], [1.0])])
    f = oracle_mod.eval_points(mol, unit_T(1, 0, 0), QS, normalise=False)[0]
    ref = np.exp(-np.sum(QS ** 2, 1) / (8 * alpha)) * np.exp(1j * QS @ C)
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-15)


def test_ss_two_centre_gaussian_product(oracle_mod):
    A, B = np.array([0.1, 0.2, -0.5]), np.array([1.3, -0.7, 0.9])
    a, b = 0.8, 2.9
    mol = mol_of([A, B], [(0, 0, [a], [1.0]), (1, 0, [b], [1.0])])
    f = oracle_mod.eval_points(mol, unit_T(2, 0, 1), QS, normalise=False)[0]
    p = a + b
    P = (a * A + b * B) / p
    ref = (4 * a * b / np.pi ** 2) ** 0.75 * (np.pi / p) ** 1.5 * np.exp(-a * b / p * np.sum((A - B) ** 2)) \
        * np.exp(-np.sum(QS ** 2, 1) / (4 * p)) * np.exp(1j * QS @ P)
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("alpha", [0.3, 5.0])
def test_pp_dd_same_centre_closed_forms(oracle_mod, alpha):
    """Textbook FTs of x^2 e^{-2 alpha x^2}-type densities (Gaussian moments)."""
    mol = mol_of([[0.0, 0.0, 0.0]], [(0, 1, [alpha], [1.0]), (0, 2, [alpha], [1.0])])
    # order: px py pz | xx xy xz yy yz zz
    qx, qy, qz = QS[:, 0], QS[:, 1], QS[:, 2]
    g = np.exp(-np.sum(QS ** 2, 1) / (8 * alpha))
    cases = {
        (2, 2): (1 - qz ** 2 / (4 * alpha)) * g,                        # pz pz
        (0, 1): -qx * qy / (4 * alpha) * g,                             # px py
        (4, 4): (1 - qx ** 2 / (4 * alpha)) * (1 - qy ** 2 / (4 * alpha)) * g,   # dxy dxy
        (3, 3): (1 - qx ** 2 / (2 * alpha) + qx ** 4 / (48 * alpha ** 2)) * g,   # dxx dxx
    }
    for (m, n), ref in cases.items():
        f = oracle_mod.eval_points(mol, unit_T(9, m, n), QS, normalise=False)[0]
        np.testing.assert_allclose(f, ref, rtol=1e-12, atol=1e-14, err_msg=str((m, n)))


def test_pz_normalisation_matches_appendix_a(oracle_mod):
    """App. A prints N^{p_z} = (pi^{3/2} sigma^5 / 2)^{-1/2}; a d=1 primitive must then have unit self-overlap."""
    for alpha in (0.2, 3.0, 70.0):
        sigma = 1.0 / math.sqrt(2 * alpha)
        n_paper = (0.5 * math.pi ** 1.5 * sigma ** 5) ** -0.5
        assert abs(n_paper - paper_forms.norm_app_a(sigma, (0, 0, 1))) < 1e-12 * n_paper
        mol = mol_of([[0.0, 0.0, 0.0]], [(0, 1, [alpha], [1.0])])
        f0 = oracle_mod.eval_points(mol, unit_T(3, 2, 2), np.zeros((1, 3)), normalise=False)[0, 0]
        assert abs(f0 - 1.0) < 1e-13


# -------------------------------------------------------- quadrature pins

def _two_centre_mol():
    return mol_of([[0.2, -0.4, 0.1], [1.1, 0.9, -1.3]],
                  [(0, 2, [3.1, 0.45], [0.7, 0.4]), (1, 1, [1.3], [1.0]), (1, 2, [0.6], [1.0]),
                   (0, 0, [5.0, 0.8], [0.3, 0.9])])


def test_pair_values_vs_1d_quadrature(oracle_mod):
    """Every component pair (s,p,d on two centres, contracted, normalised) vs products of 1D trapezoid integrals."""
    mol = _two_centre_mol()
    nbf = mol.nbf
    q = np.array([0.7, -2.2, 1.5])
    om = oracle_mod.pair_matrix(mol, q, normalise=True)
    rng = np.random.Generator(np.random.PCG64(3))
    pairs = [(m, n) for m in range(nbf) for n in range(nbf)]
    for k in rng.choice(len(pairs), size=60, replace=False):
        m, n = pairs[k]
        ref = quadrature.omega(mol, m, n, q, normalise=True)
        assert abs(om[m, n] - ref) <= 1e-10 * max(1.0, abs(ref)), (m, n, om[m, n], ref)


def test_normalisation_by_quadrature(oracle_mod):
    """normalise=1 makes every contracted Cartesian component unit-normalised (S_mumu = 1)."""
    mol = _two_centre_mol()
    c = oracle_mod.norms(mol)
    comps = quadrature.components(mol)
    for mu in range(mol.nbf):
        assert abs(c[mu] - quadrature.contracted_norm(mol, comps[mu])) < 1e-10 * c[mu]
    om0 = oracle_mod.pair_matrix(mol, np.zeros(3), normalise=True)
    np.testing.assert_allclose(np.diag(om0).real, 1.0, atol=1e-12)


@pytest.mark.slow
def test_3d_real_space_quadrature(oracle_mod):
    """Brute-force 3D trapezoid of Phi(r) e^{iq.r} over a small molecule (narrowed exponents)."""
    rng = np.random.Generator(np.random.PCG64(11))
    atoms = [[0.0, 0.0, 0.0], [1.4, 0.8, -0.5], [-1.0, 1.2, 0.9]]
    shells = [(0, 0, [2.5, 0.5], [0.6, 0.5]), (0, 1, [1.5], [1.0]), (0, 2, [1.0], [1.0]),
              (1, 0, [1.8], [1.0]), (1, 1, [0.9, 2.2], [0.8, 0.3]), (2, 0, [0.7], [1.0])]
    mol = mol_of(atoms, shells)
    nbf = mol.nbf
    T = rng.normal(size=(2, nbf, nbf))
    h, lo, hi = 0.14, -8.0, 8.0
    ax = np.arange(lo, hi + h / 2, h)
    qs = rng.uniform(-3, 3, size=(6, 3))
    acc = np.zeros((2, len(qs)), dtype=complex)
    X, Y = np.meshgrid(ax, ax, indexing="ij")
    for z in ax:
        pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1)
        phi = quadrature.basis_values(mol, pts)
        dens = np.einsum("pm,smn,pn->sp", phi, T, phi)
        acc += dens @ np.exp(1j * pts @ qs.T) * h ** 3
    f = oracle_mod.eval_points(mol, T, qs)
    scale = np.abs(f).max()
    assert np.abs(f - acc).max() < 1e-9 * scale, np.abs(f - acc).max() / scale


# ------------------------------------------------- the paper's Hermite form

def test_paper_hermite_form_per_primitive_pair(oracle_mod):
    """Sec. 4 eqs. sigmaTidbits..CartesianMethod for single primitives vs the oracle's route."""
    A, B = np.array([0.3, -1.2, 0.8]), np.array([-0.9, 0.5, 2.0])
    for (la, lb, a, b) in [(0, 0, 0.7, 2.0), (1, 1, 1.3, 0.4), (2, 1, 0.9, 3.3), (2, 2, 0.25, 0.6),
                           (0, 2, 12.0, 0.3)]:
        mol = mol_of([A, B], [(0, la, [a], [1.0]), (1, lb, [b], [1.0])])
        na = wl.n_cart(la)
        for m, pa in enumerate(wl.CART_ORDER[la]):
            for n, pb in enumerate(wl.CART_ORDER[lb]):
                ref = paper_forms.pair_form_factor(A, B, a, b, pa, pb, 1.0, 1.0, QS)
                f = oracle_mod.eval_points(mol, unit_T(mol.nbf, m, na + n), QS, normalise=False)[0]
                scale = max(np.abs(ref).max(), 1e-300)
                assert np.abs(f - ref).max() <= 1e-12 * scale, (la, lb, pa, pb)


def test_paper_monomial_form_equals_hermite_form():
    """eq. Ccoefficients: the monomial rewrite of the V polynomial equals the Hermite form."""
    q = np.linspace(-7, 7, 31)
    for ai, aj, xi, xj, ai_, aj_ in [(2, 2, 0.3, -1.1, 0.8, 2.0), (1, 2, -0.4, 0.9, 0.2, 5.0),
                                     (2, 0, 1.0, 1.0, 3.0, 0.1)]:
        si, sj = paper_forms.sigma_of(ai_), paper_forms.sigma_of(aj_)
        v = paper_forms.v_tensor(ai, aj, xi, xj, si, sj, q)
        C, sij, X = paper_forms.c_coefficients(ai, aj, xi, xj, si, sj)
        mono = np.exp(1j * q * X - q ** 2 * sij ** 2 / 2) * sum(C[u] * q ** u for u in range(len(C)))
        np.testing.assert_allclose(mono, v, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def cfg0():
    return wl.make_config(0)


def test_conjugate_symmetry(oracle_mod, cfg0):
    q = RNG.uniform(-5, 5, size=(20, 3))
    f = oracle_mod.eval_points(cfg0.mol, cfg0.T, np.concatenate([q, -q]))
    np.testing.assert_allclose(f[:, 20:], np.conj(f[:, :20]), rtol=1e-12, atol=1e-15)


def test_translation_phase(oracle_mod, cfg0):
    q = RNG.uniform(-5, 5, size=(16, 3))
    d = np.array([37.0, -61.0, 80.5])
    f = oracle_mod.eval_points(cfg0.mol, cfg0.T, q)
    g = oracle_mod.eval_points(cfg0.mol.translated(d), cfg0.T, q)
    np.testing.assert_allclose(g, f * np.exp(1j * q @ d)[None, :], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(np.abs(g) ** 2, np.abs(f) ** 2, rtol=1e-9, atol=1e-14)


def _signed_permutation_basis(mol, R):
    """Rotate the molecule by a signed permutation R; return (new mol, P) with T' = P T P^T."""
    Rinv = R.T
    comps = quadrature.components(mol)
    # new molecule: same shells, rotated centres
    new = wl.Molecule(Z=mol.Z, xyz=mol.xyz @ R.T, shell_atom=mol.shell_atom, shell_l=mol.shell_l,
                      shell_nprim=mol.shell_nprim, exps=mol.exps, coefs=mol.coefs)
    # index of each component of shell s in the new basis
    start, off = [], 0
    for s in range(mol.n_shells):
        start.append(off)
        off += wl.n_cart(int(mol.shell_l[s]))
    P = np.zeros((mol.nbf, mol.nbf))
    mu = 0
    for s in range(mol.n_shells):
        l = int(mol.shell_l[s])
        for pw in wl.CART_ORDER[l]:
            # phi'(r) = phi(R^{-1} (r - RA)); (R^{-1} v)_i = sum_j Rinv[i,j] v_j = sign_i v_{perm_i}
            new_pw = [0, 0, 0]
            sign = 1.0
            for i in range(3):
                j = int(np.argmax(np.abs(Rinv[i])))
                new_pw[j] += pw[i]
                sign *= np.sign(Rinv[i, j]) ** pw[i]
            nu = start[s] + wl.CART_ORDER[l].index(tuple(new_pw))
            P[nu, mu] = sign
            mu += 1
    return new, P


@pytest.mark.parametrize("Rrows", [((0, 1, 0), (-1, 0, 0), (0, 0, 1)),
                                   ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
                                   ((-1, 0, 0), (0, -1, 0), (0, 0, -1))])
def test_rotation_signed_permutations(oracle_mod, Rrows):
    W = wl.make_config(1)
    mol, T = W.mol, W.T[:2]
    R = np.array(Rrows, dtype=float)
    new, P = _signed_permutation_basis(mol, R)
    Tn = np.einsum("ab,sbc,dc->sad", P, T, P)
    q = RNG.uniform(-4, 4, size=(4, 3))
    f_new = oracle_mod.eval_points(new, Tn, q)
    f_old = oracle_mod.eval_points(mol, T, q @ R)     # R^T q for each row q
    np.testing.assert_allclose(f_new, f_old, rtol=1e-10, atol=1e-13)


def test_linearity_and_transpose(oracle_mod, cfg0):
    q = RNG.uniform(-5, 5, size=(10, 3))
    T1 = cfg0.T[0]
    T2 = RNG.normal(size=T1.shape)
    f1 = oracle_mod.eval_points(cfg0.mol, T1, q)
    f2 = oracle_mod.eval_points(cfg0.mol, T2, q)
    f12 = oracle_mod.eval_points(cfg0.mol, 2.0 * T1 - 0.5 * T2, q)
    np.testing.assert_allclose(f12, 2.0 * f1 - 0.5 * f2, rtol=1e-11, atol=1e-13)
    ft = oracle_mod.eval_points(cfg0.mol, T2.T, q)
    np.testing.assert_allclose(ft, f2, rtol=1e-11, atol=1e-13)
    fs = oracle_mod.eval_points(cfg0.mol, T1, q, spin_factor=math.sqrt(2))
    np.testing.assert_allclose(fs, math.sqrt(2) * f1, rtol=1e-14)


def test_centrosymmetric_odd_T_is_imaginary(oracle_mod):
    """Inversion-symmetric molecule with a T odd under inversion gives f = i Im f (Sec. 3.2 remark)."""
    base = mol_of([[0.7, -0.3, 1.1], [1.9, 0.4, -0.6]],
                  [(0, 0, [1.1, 0.3], [0.5, 0.6]), (0, 1, [0.8], [1.0]), (1, 2, [0.5], [1.0]),
                   (1, 1, [2.0], [1.0])])
    # mirrored copy at -r
    xyz = np.concatenate([base.xyz, -base.xyz])
    sa = np.concatenate([base.shell_atom, base.shell_atom + 2]).astype(np.int32)
    mol = wl.Molecule(Z=np.array([6, 6, 6, 6]), xyz=xyz, shell_atom=sa,
                      shell_l=np.concatenate([base.shell_l] * 2).astype(np.int32),
                      shell_nprim=np.concatenate([base.shell_nprim] * 2).astype(np.int32),
                      exps=np.concatenate([base.exps] * 2), coefs=np.concatenate([base.coefs] * 2))
    nb = base.nbf
    P = np.zeros((2 * nb, 2 * nb))
    ls = [l for s in range(base.n_shells) for l in [int(base.shell_l[s])] * wl.n_cart(int(base.shell_l[s]))]
    for mu in range(nb):
        sgn = (-1.0) ** ls[mu]
        P[nb + mu, mu] = sgn
        P[mu, nb + mu] = sgn
    T0 = RNG.normal(size=(2 * nb, 2 * nb))
    T = 0.5 * (T0 - P @ T0 @ P.T)
    q = RNG.uniform(-4, 4, size=(12, 3))
    f = oracle_mod.eval_points(mol, T, q)[0]
    assert np.abs(f.real).max() < 1e-12 * np.abs(f).max()
    assert np.abs(f.imag).max() > 1e-3


def test_f0_equals_trace_TS_by_quadrature(oracle_mod):
    mol = _two_centre_mol()
    nbf = mol.nbf
    S = np.zeros((nbf, nbf))
    for m in range(nbf):
        for n in range(nbf):
            S[m, n] = quadrature.omega(mol, m, n, np.zeros(3)).real
    T = RNG.normal(size=(3, nbf, nbf))
    f0 = oracle_mod.eval_points(mol, T, np.zeros((1, 3)), spin_factor=1.5)[:, 0]
    ref = 1.5 * np.einsum("smn,mn->s", T, S)
    np.testing.assert_allclose(f0, ref, rtol=1e-10, atol=1e-12)


def test_low_q_dipole_limit(oracle_mod):
    """grad_q Im f at q = 0 equals sum T <mu| r |nu> (Sec. 6 oscillator-strength relation)."""
    mol = _two_centre_mol()
    nbf = mol.nbf
    T = RNG.normal(size=(1, nbf, nbf))
    mu = np.zeros(3)
    for ax in range(3):
        D = np.zeros((nbf, nbf))
        for m in range(nbf):
            for n in range(nbf):
                D[m, n] = quadrature.omega(mol, m, n, np.zeros(3), dipole_axis=ax).real
        mu[ax] = np.sum(T[0] * D)
    grad = np.zeros(3)
    for ax in range(3):
        def d(h):
            e = np.zeros((2, 3))
            e[0, ax], e[1, ax] = h, -h
            f = oracle_mod.eval_points(mol, T, e)[0]
            return (f[0].imag - f[1].imag) / (2 * h)
        h = 2e-3
        grad[ax] = (4 * d(h / 2) - d(h)) / 3.0        # Richardson
    np.testing.assert_allclose(grad, mu, rtol=1e-7, atol=1e-9)


def test_bad_shell_rejected(oracle_mod):
    mol = mol_of([[0, 0, 0]], [(0, 3, [1.0], [1.0])])
    with pytest.raises(ValueError):
        oracle_mod.eval_points(mol, np.zeros((1, 10, 10)), np.zeros((1, 3)))
