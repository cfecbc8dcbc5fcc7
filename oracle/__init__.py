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
numpy's FFT as the library step (``fft_form_factor``).

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
