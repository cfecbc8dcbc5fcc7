"""Pins for the oracle's spherical-method functions (Sec. 4 eqs. SphericalMethod,
RTensor and the angular average; Sec. 5.4).

R_lm(q) is pinned against closed forms: a normalised s primitive at the
origin is isotropic, and one shifted to C has the plane-wave expansion
R_lm = 4 pi i^l j_l(q|C|) Y_l^m*(C^) e^{-q^2/(8 alpha)} (library spherical
Bessel functions); the harmonics against their closed forms for l <= 2 and
a library implementation; the truncated sum against the Cartesian f; the
angular average against its quadrature.  A wrong phase convention, a
missing conjugate, a wrong normalisation or an off-by-one in l fails one.
"""
import math

import numpy as np
import scipy.special as sp

import workload as wl
from tests.test_oracle_pins import mol_of


def test_harmonics_closed_forms_and_library(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(5))
    th = rng.uniform(0, np.pi, 30)
    ph = rng.uniform(0, 2 * np.pi, 30)
    Y = oracle_mod.sph_harm_table(8, th, ph)
    c, s = np.cos(th), np.sin(th)
    closed = {
        (0, 0): np.full_like(th, 0.5 / math.sqrt(math.pi)) + 0j,
        (1, 0): math.sqrt(3 / (4 * math.pi)) * c + 0j,
        (1, 1): -math.sqrt(3 / (8 * math.pi)) * s * np.exp(1j * ph),
        (1, -1): math.sqrt(3 / (8 * math.pi)) * s * np.exp(-1j * ph),
        (2, 0): math.sqrt(5 / (16 * math.pi)) * (3 * c * c - 1) + 0j,
        (2, 1): -math.sqrt(15 / (8 * math.pi)) * s * c * np.exp(1j * ph),
        (2, 2): math.sqrt(15 / (32 * math.pi)) * s * s * np.exp(2j * ph),
    }
    for (l, m), ref in closed.items():
        np.testing.assert_allclose(Y[oracle_mod.ylm_index(l, m)], ref, rtol=0, atol=1e-14)
    for l in range(9):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[oracle_mod.ylm_index(l, m)], sp.sph_harm_y(l, m, th, ph),
                                       rtol=0, atol=1e-13)
    # orthonormal under the product rule
    t, p, w = oracle_mod.sphere_rule(12)
    Yq = oracle_mod.sph_harm_table(8, t, p)
    G = (Yq * w[None, :]) @ np.conj(Yq).T
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-13)


def test_R_of_s_primitive_at_origin_is_isotropic(oracle_mod):
    a = 0.9
    mol = mol_of([(0.0, 0.0, 0.0)], [(0, 0, [a], [1.0])])
    qs = np.array([0.5, 1.7, 3.0])
    R = oracle_mod.spherical_R(mol, np.ones((1, 1, 1)), qs, 6, n_theta=12)[0]
    ref = np.zeros_like(R)
    ref[:, 0] = math.sqrt(4 * math.pi) * np.exp(-qs ** 2 / (8 * a))
    np.testing.assert_allclose(R, ref, rtol=0, atol=1e-13)


def test_R_of_shifted_s_primitive_is_the_plane_wave_expansion(oracle_mod):
    a = 1.3
    C = np.array([0.7, -1.1, 0.9])
    mol = mol_of([tuple(C)], [(0, 0, [a], [1.0])])
    qs = np.array([0.8, 2.4, 4.5])
    lmax = 10
    R = oracle_mod.spherical_R(mol, np.ones((1, 1, 1)), qs, lmax, n_theta=40)[0]
    d = np.linalg.norm(C)
    thc, phc = math.acos(C[2] / d), math.atan2(C[1], C[0])
    Yc = oracle_mod.sph_harm_table(lmax, [thc], [phc])[:, 0]
    for k, q in enumerate(qs):
        for l in range(lmax + 1):
            for m in range(-l, l + 1):
                i = oracle_mod.ylm_index(l, m)
                ref = 4 * math.pi * (1j ** l) * sp.spherical_jn(l, q * d) * np.conj(Yc[i]) * math.exp(-q * q / (8 * a))
                assert abs(R[k, i] - ref) < 1e-12, (q, l, m, R[k, i], ref)


def test_truncated_sum_converges_to_cartesian_f(oracle_mod):
    """The spherical grid f = sum_{l <= lmax} R Y approaches the Cartesian f
    as lmax grows (config-0 molecule, |q| = 2.5)."""
    W = wl.make_config(0)
    q = 2.5
    rng = np.random.Generator(np.random.PCG64(6))
    th = rng.uniform(0, np.pi, 6)
    ph = rng.uniform(0, 2 * np.pi, 6)
    pts = q * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    ref = oracle_mod.eval_points(W.mol, W.T, pts)[0]
    R = oracle_mod.spherical_R(W.mol, W.T, [q], 44, n_theta=70)
    errs = []
    for lmax in (8, 20, 44):
        Y = oracle_mod.sph_harm_table(lmax, th, ph)
        f = R[0, 0, : (lmax + 1) ** 2] @ Y
        errs.append(np.abs(f - ref).max() / np.abs(ref).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-10, errs


def test_angular_average_parseval(oracle_mod):
    """sum |R_lm|^2 / 4 pi equals the quadrature average of |f|^2 over the sphere."""
    W = wl.make_config(0)
    q = 1.5
    R = oracle_mod.spherical_R(W.mol, W.T, [q], 40, n_theta=60)
    avg_R = oracle_mod.angular_average_from_R(R)[0, 0]
    t, p, w = oracle_mod.sphere_rule(60)
    pts = q * np.stack([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)], axis=1)
    f = oracle_mod.eval_points(W.mol, W.T, pts)[0]
    avg_q = (w * np.abs(f) ** 2).sum() / (4 * math.pi)
    assert abs(avg_R - avg_q) <= 1e-12 * avg_q, (avg_R, avg_q)
