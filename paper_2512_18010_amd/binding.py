"""Thin ctypes binding of libscarff.so (the C ABI in include/scarff.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  The raw entry points are exposed under their C names
(``scff_create``, ``scff_eval_grid``, ...); ``Context`` wraps them for
numpy / torch callers.  PyTorch is used only to allocate device memory and
to name the current HIP stream.

If the library is missing this module raises at import: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscarff.so")

SCFF_OK, SCFF_EINVAL, SCFF_ENOMEM, SCFF_EDEVICE, SCFF_ESTATE, SCFF_EBUSY, SCFF_ECANCELLED = 0, -1, -2, -3, -4, -5, -6
SCFF_FP32, SCFF_BF16X3 = 0, 1
PRECISIONS = {"fp32": SCFF_FP32, "bf16x3": SCFF_BF16X3}
ERROR_NAMES = {0: "SCFF_OK", -1: "SCFF_EINVAL", -2: "SCFF_ENOMEM", -3: "SCFF_EDEVICE",
               -4: "SCFF_ESTATE", -5: "SCFF_EBUSY", -6: "SCFF_ECANCELLED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2512_18010_amd.build` "
                      "(the engine has no non-HIP fallback)")
# PyTorch ships its own HIP and HSA runtimes under the same sonames as the
# system ones the library links against.  Whichever is loaded first serves the
# whole process; if the library came first, PyTorch would load a second copy
# of each and find no GPU.  Load PyTorch's first when it is installed, so one
# HIP runtime serves both PyTorch (device memory, streams) and this library.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)

P = ctypes.POINTER
c_int, c_double, c_float, c_size_t, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p
c_longlong, c_ulonglong = ctypes.c_longlong, ctypes.c_ulonglong


class scff_grid(ctypes.Structure):
    _fields_ = [("n", c_int * 3), ("qmin", c_double * 3), ("qmax", c_double * 3)]


class scff_fft_grid(ctypes.Structure):
    _fields_ = [("n", c_int * 3), ("xmin", c_double * 3), ("L", c_double * 3)]


class scff_info(ctypes.Structure):
    _fields_ = [("nbf", c_int), ("n_shells", c_int), ("n_states", c_int),
                ("shell_pairs_total", c_longlong), ("pairs_total", c_longlong),
                ("pairs_kept", c_longlong), ("prim_pairs_total", c_longlong),
                ("prim_comp_pairs_kept", c_longlong), ("device_bytes", c_size_t),
                ("work_units", c_longlong), ("work_chunks", c_longlong)]


class scff_request(ctypes.Structure):
    _fields_ = [("n_atoms", c_int), ("xyz_bohr", P(c_double)), ("n_shells", c_int),
                ("shell_atom", P(c_int)), ("shell_l", P(c_int)), ("shell_nprim", P(c_int)),
                ("exps", P(c_double)), ("coefs", P(c_double)), ("normalise", c_int),
                ("n_states", c_int), ("T", P(c_double)), ("grid", scff_grid),
                ("precision", c_int), ("screen_eps", c_double), ("spin_factor", c_double),
                ("f", P(c_float)), ("f2", P(c_float))]


class scff_server_stats(ctypes.Structure):
    _fields_ = [("submitted", c_longlong), ("completed", c_longlong), ("failed", c_longlong),
                ("cancelled", c_longlong), ("queued", c_longlong), ("inflight", c_longlong),
                ("admitted_bytes", c_size_t), ("budget_bytes", c_size_t),
                ("peak_admitted_bytes", c_size_t), ("peak_inflight", c_longlong),
                ("mol_cache_hits", c_longlong), ("ns_stage", c_longlong * 5),
                ("batches", c_longlong), ("batched_requests", c_longlong),
                ("graphs_instantiated", c_longlong), ("graphs_updated", c_longlong),
                ("eager_batches", c_longlong)]


def _fn(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


scff_version = _fn("scff_version", ctypes.c_char_p, [])
scff_last_error = _fn("scff_last_error", ctypes.c_char_p, [])
scff_create = _fn("scff_create", c_int, [c_int, c_size_t, P(c_void_p)])
scff_destroy = _fn("scff_destroy", None, [c_void_p])
scff_load_molecule = _fn("scff_load_molecule", c_int,
                         [c_void_p, c_int, P(c_double), c_int, P(c_int), P(c_int), P(c_int),
                          P(c_double), P(c_double), c_int, P(c_int)])
scff_load_transitions = _fn("scff_load_transitions", c_int, [c_void_p, c_int, P(c_double)])
scff_load_transitions_device = _fn("scff_load_transitions_device", c_int, [c_void_p, c_int, c_void_p, c_void_p])
scff_set_options = _fn("scff_set_options", c_int, [c_void_p, c_double, c_double])
scff_eval_grid = _fn("scff_eval_grid", c_int,
                     [c_void_p, P(scff_grid), c_int, c_void_p, c_void_p, c_int, c_void_p])
scff_eval_grid_noalloc = _fn("scff_eval_grid_noalloc", c_int,
                             [c_void_p, P(scff_grid), c_int, c_void_p, c_void_p, c_void_p])
scff_eval_points = _fn("scff_eval_points", c_int,
                       [c_void_p, c_int, P(c_double), c_int, c_void_p, c_void_p, c_int, c_void_p])
scff_query = _fn("scff_query", c_int, [c_void_p, P(scff_info)])
scff_set_timing = _fn("scff_set_timing", c_int, [c_void_p, c_int])
scff_set_symmetry = _fn("scff_set_symmetry", c_int, [c_void_p, c_int])
scff_last_timing = _fn("scff_last_timing", c_int, [c_void_p, P(c_float), P(c_float), P(c_float)])
scff_export_vtensors = _fn("scff_export_vtensors", c_int,
                           [c_void_p, P(scff_grid), P(c_longlong), c_void_p, c_void_p, c_void_p,
                            c_void_p])
scff_eval_separable = _fn("scff_eval_separable", c_int,
                          [c_void_p, P(scff_grid), P(c_double), P(c_double), P(c_double), P(c_double)])
scff_eval_fft = _fn("scff_eval_fft", c_int,
                    [c_void_p, P(scff_fft_grid), c_int, c_void_p, c_void_p, c_void_p, P(c_double), c_int,
                     c_void_p])
scff_eval_spherical = _fn("scff_eval_spherical", c_int,
                          [c_void_p, c_int, c_int, P(c_double), c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                           c_int, c_void_p])
scff_last_sph_timing = _fn("scff_last_sph_timing", c_int, [c_void_p, P(c_float), P(c_float), P(c_float)])
scff_last_fft_timing = _fn("scff_last_fft_timing", c_int, [c_void_p, P(c_float), P(c_float), P(c_float)])
scff_dipole = _fn("scff_dipole", c_int, [c_void_p, P(c_double), P(c_double), P(c_double)])
scff_dipole_fit = _fn("scff_dipole_fit", c_int, [c_void_p, c_double, P(c_double), P(c_double), P(c_double)])
scff_server_create = _fn("scff_server_create", c_int, [c_int, c_size_t, c_int, P(c_void_p)])
scff_server_submit = _fn("scff_server_submit", c_int, [c_void_p, P(scff_request), P(c_ulonglong)])
scff_server_wait = _fn("scff_server_wait", c_int,
                       [c_void_p, c_ulonglong, c_longlong, P(c_int), P(c_longlong)])
scff_server_cancel = _fn("scff_server_cancel", c_int, [c_void_p, c_ulonglong])
scff_server_stats_get = _fn("scff_server_stats_get", c_int, [c_void_p, P(scff_server_stats)])
scff_server_last_failure = _fn("scff_server_last_failure", c_int, [c_void_p, ctypes.c_char_p, c_size_t])
scff_server_destroy = _fn("scff_server_destroy", None, [c_void_p])


class ScffError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc):
    if rc != SCFF_OK:
        raise ScffError(rc, scff_last_error().decode())
    return rc


def _d(a):
    return a.ctypes.data_as(P(c_double))


def _i(a):
    return a.ctypes.data_as(P(c_int))


def _molecule_arrays(mol):
    """Contiguous copies of a molecule's arrays, with their lengths checked
    against each other (the C side trusts the lengths it is given); returns
    (arrays, nbf)."""
    arrs = [np.ascontiguousarray(mol.xyz, np.float64), np.ascontiguousarray(mol.shell_atom, np.int32),
            np.ascontiguousarray(mol.shell_l, np.int32), np.ascontiguousarray(mol.shell_nprim, np.int32),
            np.ascontiguousarray(mol.exps, np.float64), np.ascontiguousarray(mol.coefs, np.float64)]
    xyz, sa, sl, sn, ex, co = arrs
    if xyz.ndim != 2 or xyz.shape[1] != 3:
        raise ValueError(f"xyz must be [n_atoms, 3], got {xyz.shape}")
    if not (sa.ndim == sl.ndim == sn.ndim == 1 and sa.shape == sl.shape == sn.shape):
        raise ValueError("shell_atom, shell_l and shell_nprim must be 1D arrays of one length")
    if np.any(sn < 0) or np.any((sl < 0) | (sl > 2)):
        raise ValueError("shell_nprim must be >= 0 and shell_l in 0..2")
    nprim = int(sn.sum())
    if ex.shape != (nprim,) or co.shape != (nprim,):
        raise ValueError(f"exps and coefs must hold sum(shell_nprim) = {nprim} values each")
    nbf = int(sum((l + 1) * (l + 2) // 2 for l in sl.tolist()))
    return arrs, nbf


def _check_T(T, nbf):
    if T.ndim != 3 or T.shape[1:] != (nbf, nbf):
        raise ValueError(f"T must be [n_states, {nbf}, {nbf}], got {T.shape}")


def _check_device_tensor(t, name, dtype, shape, device):
    """A torch tensor the C side will write or read through a raw pointer:
    exact dtype and shape, contiguous, on the context's GPU."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device.type != "cuda" or (t.device.index if t.device.index is not None else 0) != device:
        raise ValueError(f"{name} must be on cuda:{device}, got {t.device}")


def make_grid(n, qmin, qmax) -> scff_grid:
    g = scff_grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.qmin[a] = float(qmin[a])
        g.qmax[a] = float(qmax[a])
    return g


def make_fft_grid(n, xmin, L) -> scff_fft_grid:
    g = scff_fft_grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.xmin[a] = float(xmin[a])
        g.L[a] = float(L[a])
    return g


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One engine context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = c_void_p()
        check(scff_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.nbf = 0
        self.n_states = 0

    def close(self):
        if getattr(self, "_h", None):
            scff_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- loads
    def load_molecule(self, mol, normalise: bool = True) -> int:
        self._mol_keep, _ = _molecule_arrays(mol)
        xyz, sa, sl, sn, ex, co = self._mol_keep
        nbf = c_int()
        check(scff_load_molecule(self._h, xyz.shape[0], _d(xyz), sl.shape[0], _i(sa), _i(sl), _i(sn),
                                 _d(ex), _d(co), int(bool(normalise)), ctypes.byref(nbf)))
        self.nbf = nbf.value
        return self.nbf

    def load_transitions(self, T):
        T = np.ascontiguousarray(T, np.float64)
        if T.ndim == 2:
            T = T[None]
        _check_T(T, self.nbf)
        check(scff_load_transitions(self._h, T.shape[0], _d(T)))
        self.n_states = T.shape[0]

    def load_transitions_device(self, T_dev, stream=None):
        """T_dev: a contiguous float64 device tensor [n_states, nbf, nbf] (e.g. torch on 'cuda')."""
        import torch
        ns = int(T_dev.shape[0]) if T_dev.dim() == 3 else -1
        _check_device_tensor(T_dev, "T_dev", torch.float64, (ns, self.nbf, self.nbf), self.device)
        check(scff_load_transitions_device(self._h, ns, ctypes.c_void_p(T_dev.data_ptr()), _stream_ptr(stream)))
        self.n_states = ns

    def set_options(self, screen_eps: float = 0.0, spin_factor: float = 1.0):
        check(scff_set_options(self._h, float(screen_eps), float(spin_factor)))

    def set_timing(self, enable: bool = True):
        check(scff_set_timing(self._h, int(bool(enable))))

    def set_symmetry(self, enable: bool = True):
        """Evaluate half of a grid symmetric about q = 0 and mirror f(-q) = f(q)*."""
        check(scff_set_symmetry(self._h, int(bool(enable))))

    def last_timing(self):
        """(prep_ms, vtable_ms, grid_ms) of the last timed evaluation (HIP events on its stream)."""
        p, a, b = c_float(), c_float(), c_float()
        check(scff_last_timing(self._h, ctypes.byref(p), ctypes.byref(a), ctypes.byref(b)))
        return p.value, a.value, b.value

    def query(self) -> dict:
        info = scff_info()
        check(scff_query(self._h, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in scff_info._fields_}

    # ---- evaluation
    def eval_grid_host(self, grid, precision="fp32", want_f=True, want_f2=True):
        """Host outputs: (f complex64 [s,nx,ny,nz] or None, f2 float32 [s,nx,ny,nz] or None)."""
        n = tuple(grid.n)
        shape = (self.n_states,) + n
        f = np.empty(shape + (2,), np.float32) if want_f else None
        f2 = np.empty(shape, np.float32) if want_f2 else None
        g = make_grid(grid.n, grid.qmin, grid.qmax)
        check(scff_eval_grid(self._h, ctypes.byref(g), PRECISIONS[precision],
                             f.ctypes.data if f is not None else None,
                             f2.ctypes.data if f2 is not None else None, 0, None))
        return (f.view(np.complex64)[..., 0] if f is not None else None), f2

    def eval_grid_device(self, grid, f=None, f2=None, precision="fp32", stream=None):
        """Device outputs into torch tensors f ([s,nx,ny,nz,2] float32) / f2 ([s,nx,ny,nz] float32)."""
        import torch
        shape = (self.n_states,) + tuple(int(x) for x in grid.n)
        if f is not None:
            _check_device_tensor(f, "f", torch.float32, shape + (2,), self.device)
        if f2 is not None:
            _check_device_tensor(f2, "f2", torch.float32, shape, self.device)
        g = make_grid(grid.n, grid.qmin, grid.qmax)
        check(scff_eval_grid(self._h, ctypes.byref(g), PRECISIONS[precision],
                             f.data_ptr() if f is not None else None,
                             f2.data_ptr() if f2 is not None else None, 1, _stream_ptr(stream)))
        return f, f2

    def eval_fft_host(self, n, xmin, L, want_f=True, want_f2=True, want_phi=False, parseval=True,
                      precision="fp32"):
        """FFT method on the box [xmin, xmin + L) sampled at n points per axis (host outputs):
        (f complex64 [s,n0,n1,n2] or None, f2 or None, phi float32 [s,n0,n1,n2] or None,
        parseval float64 [s, 2] or None).  precision: "fp32" or "bf16x3" (density contraction)."""
        g = make_fft_grid(n, xmin, L)
        shape = (self.n_states,) + tuple(int(x) for x in n)
        f = np.empty(shape + (2,), np.float32) if want_f else None
        f2 = np.empty(shape, np.float32) if want_f2 else None
        phi = np.empty(shape, np.float32) if want_phi else None
        ps = np.empty((self.n_states, 2), np.float64) if parseval else None
        check(scff_eval_fft(self._h, ctypes.byref(g), PRECISIONS[precision],
                            f.ctypes.data if f is not None else None,
                            f2.ctypes.data if f2 is not None else None,
                            phi.ctypes.data if phi is not None else None,
                            _d(ps) if ps is not None else None, 0, None))
        return (f.view(np.complex64)[..., 0] if f is not None else None), f2, phi, ps

    def eval_fft_device(self, n, xmin, L, f=None, f2=None, phi=None, stream=None, precision="fp32"):
        """FFT method into torch tensors f ([s,n0,n1,n2,2] float32), f2 / phi ([s,n0,n1,n2] float32)."""
        import torch
        g = make_fft_grid(n, xmin, L)
        shape = (self.n_states,) + tuple(int(x) for x in n)
        if f is not None:
            _check_device_tensor(f, "f", torch.float32, shape + (2,), self.device)
        if f2 is not None:
            _check_device_tensor(f2, "f2", torch.float32, shape, self.device)
        if phi is not None:
            _check_device_tensor(phi, "phi", torch.float32, shape, self.device)
        check(scff_eval_fft(self._h, ctypes.byref(g), PRECISIONS[precision],
                            f.data_ptr() if f is not None else None,
                            f2.data_ptr() if f2 is not None else None,
                            phi.data_ptr() if phi is not None else None, None, 1, _stream_ptr(stream)))
        return f, f2, phi

    def eval_spherical_host(self, lmax, qs, n_theta=0, n_phi=0, want_R=True, want_f=False, want_f2=False,
                            want_avg=True):
        """Spherical method (host outputs): (R complex128 [s, n_q, (lmax+1)^2] or None,
        f complex64 [s, n_q, n_theta, n_phi] or None, f2 or None, avg float64 [s, n_q] or None)."""
        qs = np.ascontiguousarray(np.asarray(qs, np.float64).reshape(-1))
        ns, nq, nl = self.n_states, qs.shape[0], (int(lmax) + 1) ** 2
        R = np.empty((ns, nq, nl, 2), np.float64) if want_R else None
        f = np.empty((ns, nq, n_theta, n_phi, 2), np.float32) if want_f else None
        f2 = np.empty((ns, nq, n_theta, n_phi), np.float32) if want_f2 else None
        avg = np.empty((ns, nq), np.float64) if want_avg else None
        check(scff_eval_spherical(self._h, int(lmax), nq, _d(qs), int(n_theta), int(n_phi),
                                  R.ctypes.data if R is not None else None,
                                  f.ctypes.data if f is not None else None,
                                  f2.ctypes.data if f2 is not None else None,
                                  avg.ctypes.data if avg is not None else None, 0, None))
        return ((R[..., 0] + 1j * R[..., 1]) if R is not None else None,
                (f.view(np.complex64)[..., 0] if f is not None else None), f2, avg)

    def eval_spherical_device(self, lmax, qs, n_theta, n_phi, f=None, f2=None, R=None, avg=None, stream=None):
        """Spherical method into torch tensors: f [s,n_q,n_theta,n_phi,2] / f2 [s,n_q,n_theta,n_phi] float32,
        R [s,n_q,(lmax+1)^2,2] / avg [s,n_q] float64."""
        import torch
        qs = np.ascontiguousarray(np.asarray(qs, np.float64).reshape(-1))
        ns, nq, nl = self.n_states, qs.shape[0], (int(lmax) + 1) ** 2
        if f is not None:
            _check_device_tensor(f, "f", torch.float32, (ns, nq, n_theta, n_phi, 2), self.device)
        if f2 is not None:
            _check_device_tensor(f2, "f2", torch.float32, (ns, nq, n_theta, n_phi), self.device)
        if R is not None:
            _check_device_tensor(R, "R", torch.float64, (ns, nq, nl, 2), self.device)
        if avg is not None:
            _check_device_tensor(avg, "avg", torch.float64, (ns, nq), self.device)
        check(scff_eval_spherical(self._h, int(lmax), nq, _d(qs), int(n_theta), int(n_phi),
                                  R.data_ptr() if R is not None else None,
                                  f.data_ptr() if f is not None else None,
                                  f2.data_ptr() if f2 is not None else None,
                                  avg.data_ptr() if avg is not None else None, 1, _stream_ptr(stream)))
        return f, f2, R, avg

    def last_sph_timing(self):
        """(geom_ms, contraction_ms, rest_ms) of the last timed spherical evaluation."""
        a, b, t = c_float(), c_float(), c_float()
        check(scff_last_sph_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t)))
        return a.value, b.value, t.value

    def last_fft_timing(self):
        """(pack_ms, density_ms, transform_ms) of the last timed FFT evaluation."""
        a, b, t = c_float(), c_float(), c_float()
        check(scff_last_fft_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t)))
        return a.value, b.value, t.value

    def eval_points(self, q, precision="fp32"):
        q = np.ascontiguousarray(np.atleast_2d(q), np.float64)
        nq = q.shape[0]
        f = np.empty((self.n_states, nq, 2), np.float32)
        f2 = np.empty((self.n_states, nq), np.float32)
        check(scff_eval_points(self._h, nq, _d(q), PRECISIONS[precision], f.ctypes.data,
                               f2.ctypes.data, 0, None))
        return f.view(np.complex64)[..., 0], f2

    def eval_separable(self, grid, wx, wy, wz):
        """sum over the grid of wx[ix] wy[iy] wz[iz] f_s(q) per transition (complex128 [n_states])."""
        ws = []
        for a, w in enumerate((wx, wy, wz)):
            w = np.ascontiguousarray(np.asarray(w, np.complex128).reshape(-1))
            if w.shape[0] != int(grid.n[a]):
                raise ValueError(f"weights of axis {a} must have {grid.n[a]} values, got {w.shape[0]}")
            ws.append(w)
        out = np.empty(self.n_states, np.complex128)
        g = make_grid(grid.n, grid.qmin, grid.qmax)
        check(scff_eval_separable(self._h, ctypes.byref(g), *[w.view(np.float64).ctypes.data_as(P(c_double))
                                                              for w in ws],
                                  out.view(np.float64).ctypes.data_as(P(c_double))))
        return out

    def dipole(self, dE=None):
        """(mu [n_states, 3], f0 [n_states] or None): transition dipoles and oscillator strengths."""
        mu = np.empty((self.n_states, 3), np.float64)
        f0 = None
        dEa = None
        if dE is not None:
            dEa = np.ascontiguousarray(np.asarray(dE, np.float64).reshape(-1))
            if dEa.shape[0] != self.n_states:
                raise ValueError(f"dE must hold {self.n_states} values")
            f0 = np.empty(self.n_states, np.float64)
        check(scff_dipole(self._h, _d(dEa) if dEa is not None else None, _d(mu),
                          _d(f0) if f0 is not None else None))
        return mu, f0

    def dipole_fit(self, q_fit, dE=None):
        """(coef [n_states, 3] = A, B, C of <|f|^2> = A + B q^2 + C q^4, f0_fit or None)."""
        coef = np.empty((self.n_states, 3), np.float64)
        f0 = None
        dEa = None
        if dE is not None:
            dEa = np.ascontiguousarray(np.asarray(dE, np.float64).reshape(-1))
            if dEa.shape[0] != self.n_states:
                raise ValueError(f"dE must hold {self.n_states} values")
            f0 = np.empty(self.n_states, np.float64)
        check(scff_dipole_fit(self._h, float(q_fit), _d(dEa) if dEa is not None else None, _d(coef),
                              _d(f0) if f0 is not None else None))
        return coef, f0

    def export_vtensors(self, grid):
        g = make_grid(grid.n, grid.qmin, grid.qmax)
        nt = c_longlong()
        check(scff_export_vtensors(self._h, ctypes.byref(g), ctypes.byref(nt), None, None, None, None))
        R = nt.value
        vs = [np.empty((R, grid.n[a], 2), np.float32) for a in range(3)]
        tp = np.empty((self.n_states, R), np.float32)
        check(scff_export_vtensors(self._h, ctypes.byref(g), ctypes.byref(nt), vs[0].ctypes.data,
                                   vs[1].ctypes.data, vs[2].ctypes.data, tp.ctypes.data))
        return [v.view(np.complex64)[..., 0] for v in vs], tp


class Server:
    """Continuous-batching request server (scff_server_*).  device = -1 is the
    scheduler test mode (no GPU work; outputs are left untouched)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_inflight: int = 4):
        h = c_void_p()
        check(scff_server_create(int(device), int(hbm_budget_bytes), int(max_inflight), ctypes.byref(h)))
        self._h = h
        self._outs = {}

    def submit(self, mol, T, grid, precision="fp32", screen_eps=0.0, spin_factor=1.0,
               want_f=True, want_f2=True, normalise=True, precision_code=None) -> int:
        T = np.ascontiguousarray(T, np.float64)
        if T.ndim == 2:
            T = T[None]
        arrs, nbf = _molecule_arrays(mol)
        _check_T(T, nbf)
        shape = (T.shape[0],) + tuple(grid.n)
        f = np.empty(shape + (2,), np.float32) if want_f else None
        f2 = np.empty(shape, np.float32) if want_f2 else None
        r = scff_request()
        r.n_atoms = arrs[0].shape[0]
        r.xyz_bohr = _d(arrs[0])
        r.n_shells = arrs[2].shape[0]
        r.shell_atom, r.shell_l, r.shell_nprim = _i(arrs[1]), _i(arrs[2]), _i(arrs[3])
        r.exps, r.coefs = _d(arrs[4]), _d(arrs[5])
        r.normalise = int(bool(normalise))
        r.n_states = T.shape[0]
        r.T = _d(T)
        r.grid = make_grid(grid.n, grid.qmin, grid.qmax)
        r.precision = PRECISIONS[precision] if precision_code is None else int(precision_code)
        r.screen_eps = float(screen_eps)
        r.spin_factor = float(spin_factor)
        r.f = f.ctypes.data_as(P(c_float)) if f is not None else None
        r.f2 = f2.ctypes.data_as(P(c_float)) if f2 is not None else None
        t = c_ulonglong()
        check(scff_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._outs[t.value] = (f, f2)
        return t.value

    def wait(self, ticket: int, timeout_ns: int = -1):
        """(status, latency_ns, f complex64 or None, f2 or None); raises ScffError(SCFF_EBUSY) on timeout."""
        status, lat = c_int(), c_longlong()
        check(scff_server_wait(self._h, c_ulonglong(ticket), c_longlong(timeout_ns), ctypes.byref(status),
                               ctypes.byref(lat)))
        f, f2 = self._outs.pop(ticket, (None, None))
        fc = f.view(np.complex64)[..., 0] if f is not None else None
        return status.value, lat.value, fc, f2

    def cancel(self, ticket: int):
        check(scff_server_cancel(self._h, c_ulonglong(ticket)))

    def stats(self) -> dict:
        st = scff_server_stats()
        check(scff_server_stats_get(self._h, ctypes.byref(st)))
        d = {k: getattr(st, k) for k, _ in scff_server_stats._fields_}
        d["ns_stage"] = list(d["ns_stage"])
        return d

    def last_failure(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        check(scff_server_last_failure(self._h, buf, 1024))
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None):
            scff_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
