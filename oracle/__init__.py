"""FP64 CPU oracle for the molecular transition form factor (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It is the checker that the
HIP library is compared against, not a fallback for it: it shares no code
with ``paper_2512_18010_amd`` and is never called by the product path.

The arithmetic lives in ``scff_oracle.c`` (plain C99, FP64, OpenMP over
q-points); its header states each step and the passage of the paper it
follows.  This wrapper only builds that file with gcc and marshals arrays.

The FFT method (Sec. 3, Sec. 5.2) is here too: the transition density on a
real-space grid (C, FP64) and its transform by the paper's steps, with
numpy's FFT as the library step (``fft_form_factor``).  And the spherical
method's result (Sec. 4 eqs. SphericalMethod, RTensor; Sec. 5.4) from its
plain definition: R_lm(q) is the projection of f on the sphere of radius q
onto the complex spherical harmonic Y_lm, computed with a product quadrature
(Gauss-Legendre in cos theta, uniform in phi) of the Cartesian f above, and
the spherical grid is the truncated sum over l <= lmax (``spherical_R``,
``spherical_grid``).

Parity unpinned: nothing.  Every function here is pinned by tests against
closed forms, real-space quadrature, the paper's Hermite form, a direct DFT
sum, the analytic form factor and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scff_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-D_GNU_SOURCE",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i = ctypes.c_double, ctypes.c_int
        lib.scffo_eval.argtypes = [i, P(d), i, P(i), P(i), P(i), P(d), P(d), i, i, P(d), i,
                                   P(d), d, P(d), i]
        lib.scffo_eval.restype = i
        lib.scffo_pair_matrix.argtypes = [i, P(d), i, P(i), P(i), P(i), P(d), P(d), i, P(d),
                                          P(d)]
        lib.scffo_pair_matrix.restype = i
        lib.scffo_norms.argtypes = [i, P(i), P(i), P(i), P(d), P(d), P(d)]
        lib.scffo_norms.restype = i
        lib.scffo_density.argtypes = [i, P(d), i, P(i), P(i), P(i), P(d), P(d), i, i, P(d), i,
                                      P(d), d, P(d), i]
        lib.scffo_density.restype = i
        lib.scffo_ao_values.argtypes = [i, P(d), i, P(i), P(i), P(i), P(d), P(d), i, i, P(d), P(d)]
        lib.scffo_ao_values.restype = i
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _mol_args(mol):
    xyz = np.ascontiguousarray(mol.xyz, dtype=np.float64)
    sa = np.ascontiguousarray(mol.shell_atom, dtype=np.int32)
    sl = np.ascontiguousarray(mol.shell_l, dtype=np.int32)
    sn = np.ascontiguousarray(mol.shell_nprim, dtype=np.int32)
    ex = np.ascontiguousarray(mol.exps, dtype=np.float64)
    co = np.ascontiguousarray(mol.coefs, dtype=np.float64)
    return xyz, sa, sl, sn, ex, co


def eval_points(mol, T: np.ndarray, q: np.ndarray, normalise: bool = True,
                spin_factor: float = 1.0, n_threads: Optional[int] = None) -> np.ndarray:
    """f_s(q) for every state s and every row of q ([n_q, 3], a.u.) -> complex128 [n_states, n_q]."""
    lib = _load()
    xyz, sa, sl, sn, ex, co = _mol_args(mol)
    T = np.ascontiguousarray(T, dtype=np.float64)
    if T.ndim == 2:
        T = T[None]
    q = np.ascontiguousarray(np.atleast_2d(q), dtype=np.float64)
    ns, nq = T.shape[0], q.shape[0]
    out = np.zeros((ns, nq, 2), dtype=np.float64)
    if n_threads is None:
        n_threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    rc = lib.scffo_eval(mol.n_atoms, _dptr(xyz), mol.n_shells, _iptr(sa), _iptr(sl), _iptr(sn),
                        _dptr(ex), _dptr(co), int(bool(normalise)), ns, _dptr(T), nq, _dptr(q),
                        float(spin_factor), _dptr(out), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle: malformed input (code {rc})")
    return out[..., 0] + 1j * out[..., 1]


def pair_matrix(mol, q, normalise: bool = True) -> np.ndarray:
    """Omega_{mu nu}(q) for all component pairs at one q -> complex128 [nbf, nbf]."""
    lib = _load()
    xyz, sa, sl, sn, ex, co = _mol_args(mol)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
    nbf = mol.nbf
    out = np.zeros((nbf, nbf, 2))
    rc = lib.scffo_pair_matrix(mol.n_atoms, _dptr(xyz), mol.n_shells, _iptr(sa), _iptr(sl),
                               _iptr(sn), _dptr(ex), _dptr(co), int(bool(normalise)), _dptr(q),
                               _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle: malformed input (code {rc})")
    return out[..., 0] + 1j * out[..., 1]


def norms(mol) -> np.ndarray:
    """Contracted normalisation constants c_mu -> float64 [nbf]."""
    lib = _load()
    xyz, sa, sl, sn, ex, co = _mol_args(mol)
    out = np.zeros(mol.nbf)
    rc = lib.scffo_norms(mol.n_shells, _iptr(sa), _iptr(sl), _iptr(sn), _dptr(ex), _dptr(co),
                         _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle: malformed input (code {rc})")
    return out


def eval_grid(mol, T, grid, normalise=True, spin_factor=1.0, n_threads=None) -> np.ndarray:
    """f on a full grid -> complex128 [n_states, nx, ny, nz]."""
    f = eval_points(mol, T, grid.points(), normalise, spin_factor, n_threads)
    return f.reshape((f.shape[0],) + tuple(grid.n))


# ------------------------------------------------------------------ FFT method


def ao_values(mol, r, normalise=True) -> np.ndarray:
    """phi_mu at points r ([n, 3], bohr) -> float64 [n, nbf]."""
    lib = _load()
    xyz, sa, sl, sn, ex, co = _mol_args(mol)
    r = np.ascontiguousarray(np.atleast_2d(r), dtype=np.float64)
    out = np.zeros((r.shape[0], mol.nbf))
    rc = lib.scffo_ao_values(mol.n_atoms, _dptr(xyz), mol.n_shells, _iptr(sa), _iptr(sl), _iptr(sn),
                             _dptr(ex), _dptr(co), int(bool(normalise)), r.shape[0], _dptr(r), _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle: malformed input (code {rc})")
    return out


def density(mol, T, r, normalise=True, spin_factor=1.0, n_threads=None) -> np.ndarray:
    """Transition density Phi_s(r) (eq. PhiTDM, AO form) -> float64 [n_states, n]."""
    lib = _load()
    xyz, sa, sl, sn, ex, co = _mol_args(mol)
    T = np.ascontiguousarray(T, dtype=np.float64)
    if T.ndim == 2:
        T = T[None]
    r = np.ascontiguousarray(np.atleast_2d(r), dtype=np.float64)
    out = np.zeros((T.shape[0], r.shape[0]))
    if n_threads is None:
        n_threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    rc = lib.scffo_density(mol.n_atoms, _dptr(xyz), mol.n_shells, _iptr(sa), _iptr(sl), _iptr(sn),
                           _dptr(ex), _dptr(co), int(bool(normalise)), T.shape[0], _dptr(T), r.shape[0],
                           _dptr(r), float(spin_factor), _dptr(out), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle: malformed input (code {rc})")
    return out


def real_space_axes(n, xmin, L):
    """x_a = xmin + a L / N, a = 0..N-1 per axis (the periodic sampling of Sec. 3)."""
    return [xmin[a] + np.arange(n[a]) * (L[a] / n[a]) for a in range(3)]


def density_grid(mol, T, n, xmin, L, normalise=True, spin_factor=1.0, n_threads=None) -> np.ndarray:
    """Phi_s on the real-space grid -> float64 [n_states, nx, ny, nz] (z fastest)."""
    ax = real_space_axes(n, xmin, L)
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    phi = density(mol, T, pts, normalise, spin_factor, n_threads)
    return phi.reshape((phi.shape[0],) + tuple(n))


def fft_q_axes(n, L):
    """q_alpha = 2 pi alpha / L for alpha = -floor(N/2) .. ceil(N/2)-1 (eq. qabc, most negative first)."""
    return [2.0 * np.pi * (np.arange(n[a]) - n[a] // 2) / L[a] for a in range(3)]


def fft_form_factor(mol, T, n, xmin, L, normalise=True, spin_factor=1.0, n_threads=None, phi=None):
    """The FFT method of Sec. 3 on the box [xmin, xmin + L) sampled at N points per axis.

    1. Phi_s tabulated on x_abc (``density_grid``);
    2. F*_abg = forward DFT of the conjugate array (eq. Falbega; numpy's FFT);
    3. cycle each axis so the most negative frequencies come first;
    4. f*_s(q) = V_pix e^{-i q.x_min} F*_abg at q = 2 pi alpha / L (eq. fftABC
       applied to Phi*, eq. qabc), so f_s is its complex conjugate.
    Returns (f [n_states, nx, ny, nz] complex128, phi [n_states, nx, ny, nz]).
    """
    if phi is None:
        phi = density_grid(mol, T, n, xmin, L, normalise, spin_factor, n_threads)
    Fs = np.fft.fftn(np.conj(phi), axes=(1, 2, 3))
    Fs = np.fft.fftshift(Fs, axes=(1, 2, 3))
    vpix = float(np.prod(np.asarray(L, float) / np.asarray(n, float)))
    q = fft_q_axes(n, L)
    QX, QY, QZ = np.meshgrid(q[0], q[1], q[2], indexing="ij")
    qx = QX * xmin[0] + QY * xmin[1] + QZ * xmin[2]
    f_conj = vpix * np.exp(-1j * qx)[None] * Fs
    return np.conj(f_conj), phi


def parseval_sums(phi, f, n, L):
    """(int |Phi|^2 d^3r, int |f|^2 d^3q / (2 pi)^3) per state, both as grid sums (Sec. 7 check)."""
    vpix = float(np.prod(np.asarray(L, float) / np.asarray(n, float)))
    dq3 = float(np.prod(2.0 * np.pi / np.asarray(L, float)))
    ns = phi.shape[0]
    a = (np.abs(phi.reshape(ns, -1)) ** 2).sum(axis=1) * vpix
    b = (np.abs(f.reshape(ns, -1)) ** 2).sum(axis=1) * dq3 / (2.0 * np.pi) ** 3
    return a, b


# ------------------------------------------------------------ spherical method


def ylm_index(l, m):
    return l * l + l + m


def sph_harm_table(lmax, theta, phi):
    """Complex spherical harmonics Y_l^m(theta, phi), orthonormal on the unit
    sphere, with the Condon-Shortley phase, for l <= lmax -> complex128
    [(lmax+1)^2, n] (index l^2 + l + m).  Associated Legendre functions by the
    standard upward recurrences in l from P_m^m; Y_l^{-m} = (-1)^m conj(Y_l^m)."""
    theta = np.asarray(theta, np.float64).reshape(-1)
    phi = np.asarray(phi, np.float64).reshape(-1)
    x, sx = np.cos(theta), np.sin(theta)
    out = np.zeros(((lmax + 1) ** 2, theta.size), np.complex128)
    # normalised P~_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m, P_l^m with Condon-Shortley phase
    pmm = np.full(theta.size, np.sqrt(1.0 / (4.0 * np.pi)))
    for m in range(lmax + 1):
        if m > 0:
            pmm = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sx * pmm
        plm2, plm1 = None, pmm
        e = np.exp(1j * m * phi)
        for l in range(m, lmax + 1):
            if l == m:
                cur = pmm
            elif l == m + 1:
                cur = np.sqrt(2.0 * m + 3.0) * x * pmm
            else:
                a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                cur = a * (x * plm1 - b * plm2)
            if l > m:
                plm2, plm1 = plm1, cur
            y = cur * e
            out[ylm_index(l, m)] = y
            if m > 0:
                out[ylm_index(l, -m)] = (-1) ** m * np.conj(y)
    return out


def sphere_rule(n_theta, n_phi=None):
    """Product rule on the unit sphere: Gauss-Legendre nodes in cos(theta),
    n_phi = 2 n_theta equally spaced azimuths.  Exact for Y_l^m products of
    total degree < 2 n_theta (and |m| < n_phi).  Returns (theta, phi, w)."""
    if n_phi is None:
        n_phi = 2 * n_theta
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    T, P = np.meshgrid(np.arccos(xg), ph, indexing="ij")
    W = np.repeat(wg[:, None], n_phi, axis=1) * (2.0 * np.pi / n_phi)
    return T.ravel(), P.ravel(), W.ravel()


def spherical_R(mol, T, qs, lmax, n_theta, normalise=True, spin_factor=1.0, n_threads=None):
    """R_lm(q) = int dOmega Y_l^m*(q^) f(q q^) for each radius in qs (a.u.):
    the coefficients of eq. SphericalMethod, from the Cartesian f of this
    oracle on a product quadrature with n_theta Gauss-Legendre nodes (choose
    n_theta above lmax plus the band limit of f on the sphere, about
    q * max|r| + 30).  Returns complex128 [n_states, n_q, (lmax+1)^2]."""
    th, ph, w = sphere_rule(n_theta)
    Y = sph_harm_table(lmax, th, ph)
    dirs = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    qs = np.asarray(qs, np.float64).reshape(-1)
    T = np.asarray(T, np.float64)
    if T.ndim == 2:
        T = T[None]
    out = np.zeros((T.shape[0], qs.size, (lmax + 1) ** 2), np.complex128)
    for k, q in enumerate(qs):
        f = eval_points(mol, T, q * dirs, normalise, spin_factor, n_threads)   # [s, n_pts]
        out[:, k, :] = (f * w[None, :]) @ np.conj(Y).T
    return out


def spherical_grid(R, lmax, theta, phi):
    """f_s(q, theta_i, phi_j) = sum_{l <= lmax, m} R_lm(q) Y_l^m(theta_i, phi_j)
    -> complex128 [n_states, n_q, n_theta, n_phi]."""
    th, ph = np.meshgrid(np.asarray(theta, float), np.asarray(phi, float), indexing="ij")
    Y = sph_harm_table(lmax, th.ravel(), ph.ravel())
    f = R[..., : (lmax + 1) ** 2] @ Y
    return f.reshape(R.shape[0], R.shape[1], th.shape[0], th.shape[1])


def angular_average_from_R(R):
    """<|f|^2>_Omega(q) = sum_lm |R_lm(q)|^2 / (4 pi) (Sec. 4) -> [n_states, n_q]."""
    return (np.abs(R) ** 2).sum(axis=-1) / (4.0 * np.pi)
