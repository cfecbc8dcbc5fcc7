"""The paper's own closed form for one primitive pair, written from Sec. 4.

Used only as a pin for the oracle: the oracle reduces the same integral by
complex-shifted Gaussian moments, this module follows the paper's route
(widths sigma, eq. sigmaTidbits; centre X_ij, eq. positionTidbits;
b-coefficients, eq. bCoefficients; prefactor M_ij, eq. Mij; probabilists'
Hermite polynomials by recurrence; V-tensors, eq. CartesianVector; their
product, eq. CartesianMethod) and App. A's primitive normalisation with
the Gamma-function form of N_alpha.
"""
from __future__ import annotations

import math

import numpy as np


def sigma_of(alpha):
    # App. A: exp(-r^2 / (2 sigma^2)) = exp(-alpha r^2)
    return 1.0 / math.sqrt(2.0 * alpha)


def norm_app_a(sigma, pw):
    """N_alpha of App. A for a single monomial (every k_i = 1)."""
    s = 1.0
    for k in pw:
        kk = 2 * k
        s *= sigma ** (1 + kk) * math.gamma((kk + 1) / 2.0)
    return s ** -0.5


def hermite_he(n, x):
    """Probabilists' Hermite polynomials He_0..He_n at x (recurrence He_{k+1} = x He_k - k He_{k-1})."""
    out = [np.ones_like(x), x]
    for k in range(1, n):
        out.append(x * out[k] - k * out[k - 1])
    return out[: n + 1]


def b_coeffs(ai, aj, Xij, xi, xj):
    """eq. bCoefficients: coefficients of x^A in (x + X - x_i)^{a_i} (x + X - x_j)^{a_j}."""
    alpha = ai + aj
    out = []
    for A in range(alpha + 1):
        s = 0.0
        for k in range(max(0, ai - A), min(ai, alpha - A) + 1):
            s += math.comb(ai, k) * math.comb(aj, alpha - k - A) * (Xij - xi) ** k * \
                (Xij - xj) ** (alpha - k - A)
        out.append(s)
    return out


def v_tensor(ai, aj, xi, xj, sig_i, sig_j, q):
    """eq. CartesianVector for one axis."""
    sbar = math.sqrt(sig_i ** 2 + sig_j ** 2)
    sij = sig_i * sig_j / sbar
    Xij = sij ** 2 * (xi / sig_i ** 2 + xj / sig_j ** 2)
    b = b_coeffs(ai, aj, Xij, xi, xj)
    he = hermite_he(ai + aj, q * sij)
    poly = sum(b[A] * (1j * sij) ** A * he[A] for A in range(ai + aj + 1))
    return np.exp(1j * q * Xij - q ** 2 * sij ** 2 / 2.0) * poly


def pair_form_factor(ri, rj, alpha_i, alpha_j, pw_i, pw_j, d_i, d_j, q):
    """(2 pi)^{3/2} M_ij V^x V^y V^z for one primitive pair (eqs. Mij, CartesianMethod without sqrt 2)."""
    si, sj = sigma_of(alpha_i), sigma_of(alpha_j)
    sbar2 = si ** 2 + sj ** 2
    sij = si * sj / math.sqrt(sbar2)
    rij2 = float(np.sum((np.asarray(ri) - np.asarray(rj)) ** 2))
    M = d_i * d_j * norm_app_a(si, pw_i) * norm_app_a(sj, pw_j) * sij ** 3 * math.exp(-rij2 / (2 * sbar2))
    q = np.atleast_2d(q)
    v = np.ones(q.shape[0], dtype=complex)
    for ax in range(3):
        v *= v_tensor(pw_i[ax], pw_j[ax], ri[ax], rj[ax], si, sj, q[:, ax])
    return (2 * math.pi) ** 1.5 * M * v


def c_coefficients(ai, aj, xi, xj, sig_i, sig_j):
    """eq. Ccoefficients (monomial form of the V polynomial): C^u, u = 0..a_i+a_j (complex)."""
    sbar = math.sqrt(sig_i ** 2 + sig_j ** 2)
    sij = sig_i * sig_j / sbar
    Xij = sij ** 2 * (xi / sig_i ** 2 + xj / sig_j ** 2)
    b = b_coeffs(ai, aj, Xij, xi, xj)
    alpha = ai + aj
    out = []
    for u in range(alpha + 1):
        s = 0.0
        for m in range((alpha - u) // 2 + 1):
            s += b[u + 2 * m] * sij ** (2 * (u + m)) * math.factorial(u + 2 * m) / \
                (math.factorial(m) * math.factorial(u) * 2 ** m)
        out.append((1j) ** u * s)
    return out, sij, Xij
