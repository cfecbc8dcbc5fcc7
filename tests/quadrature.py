"""Independent real-space quadrature used to pin the oracle.

Nothing here shares code with the oracle or with the HIP library.  The
integrals are evaluated numerically on uniform grids with the trapezoid
rule, which converges exponentially fast for smooth integrands that decay
like Gaussians on the real line (the sampling error is set by the spacing
h through aliasing, ~exp(-(2 pi/h - |q|)^2 / (4 p)), and the truncation by
the window).
"""
from __future__ import annotations

import numpy as np

from workload import CART_ORDER


def components(mol):
    """List of (atom, powers, prim slice) in the documented AO order."""
    out = []
    off = 0
    for s in range(mol.n_shells):
        l, n = int(mol.shell_l[s]), int(mol.shell_nprim[s])
        for pw in CART_ORDER[l]:
            out.append((int(mol.shell_atom[s]), pw, slice(off, off + n)))
        off += n
    return out


def _axis_grid(centre, p, h_scale=0.004, width=11.0):
    L = width / np.sqrt(p)
    n = int(np.ceil(2 * L / (h_scale / np.sqrt(p)))) | 1
    x = np.linspace(centre - L, centre + L, n)
    return x, x[1] - x[0]


def integral_1d(i, j, A, B, a, b, q, extra_power=0):
    """int (x-A)^i (x-B)^j x^extra e^{-a(x-A)^2 - b(x-B)^2} e^{iqx} dx by trapezoid."""
    p = a + b
    P = (a * A + b * B) / p
    x, h = _axis_grid(P, p)
    g = (x - A) ** i * (x - B) ** j * x ** extra_power * np.exp(-a * (x - A) ** 2 - b * (x - B) ** 2)
    return h * np.sum(g * np.exp(1j * q * x))


def self_norm_1d(i, a):
    """int (x)^{2i} e^{-2 a x^2} dx by trapezoid."""
    return integral_1d(i, i, 0.0, 0.0, a, a, 0.0).real


def prim_norm(a, pw):
    return 1.0 / np.sqrt(np.prod([self_norm_1d(pw[k], a) for k in range(3)]))


def contracted_norm(mol, comp):
    atom, pw, sl = comp
    ex, co = mol.exps[sl], mol.coefs[sl]
    s = 0.0
    for k in range(len(ex)):
        for l in range(len(ex)):
            t = 1.0
            for ax in range(3):
                t *= integral_1d(pw[ax], pw[ax], 0.0, 0.0, ex[k], ex[l], 0.0).real
            s += co[k] * co[l] * prim_norm(ex[k], pw) * prim_norm(ex[l], pw) * t
    return 1.0 / np.sqrt(s)


def omega(mol, m, n, q, normalise=True, dipole_axis=None):
    """Omega_{mn}(q) = int phi_m phi_n e^{iq.r} (optionally times r_axis) by products of 1D quadratures."""
    comps = components(mol)
    cm, cn = comps[m], comps[n]
    A, B = mol.xyz[cm[0]], mol.xyz[cn[0]]
    exm, com = mol.exps[cm[2]], mol.coefs[cm[2]]
    exn, con = mol.exps[cn[2]], mol.coefs[cn[2]]
    acc = 0.0 + 0.0j
    for k in range(len(exm)):
        for l in range(len(exn)):
            v = com[k] * con[l] * prim_norm(exm[k], cm[1]) * prim_norm(exn[l], cn[1])
            for ax in range(3):
                v = v * integral_1d(cm[1][ax], cn[1][ax], A[ax], B[ax], exm[k], exn[l], q[ax],
                                    extra_power=1 if dipole_axis == ax else 0)
            acc += v
    if normalise:
        acc *= contracted_norm(mol, cm) * contracted_norm(mol, cn)
    return acc


def basis_values(mol, pts, normalise=True):
    """phi_mu at points [n, 3] -> [n, nbf] (direct evaluation of the documented basis)."""
    comps = components(mol)
    out = np.zeros((pts.shape[0], len(comps)))
    for mu, c in enumerate(comps):
        atom, pw, sl = c
        d = pts - mol.xyz[atom][None, :]
        r2 = np.sum(d * d, axis=1)
        poly = d[:, 0] ** pw[0] * d[:, 1] ** pw[1] * d[:, 2] ** pw[2]
        rad = np.zeros(pts.shape[0])
        for a, co in zip(mol.exps[sl], mol.coefs[sl]):
            rad += co * prim_norm(a, pw) * np.exp(-a * r2)
        nrm = contracted_norm(mol, c) if normalise else 1.0
        out[:, mu] = nrm * poly * rad
    return out
