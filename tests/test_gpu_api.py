"""GPU tests of the rest of the C ABI: exported 1D V-tensors, options,
single-output calls, device-resident T, and error paths on a real device.

Numerical checks are against the FP64 oracle (tolerances as in the parity
tests: 1e-6 peak-normalised |f|^2 for FP32 arithmetic) or against exact
invariants of the method.
"""
import os
import sys

import numpy as np
import pytest

import workload as wl
from tests.metrics import TOL_F2, errors

pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def binding():
    import torch  # noqa: F401  (initialises HIP the same way the benchmark does)
    from paper_2512_18010_amd import binding as b
    return b


def small_case():
    W = wl.make_config(0)
    W.grid = wl.Grid(n=(9, 11, 13), qmin=(-5.0, -4.5, -5.0), qmax=(5.0, 4.0, 5.5))
    return W


def test_export_vtensors_rebuild_f(binding, oracle_mod):
    """The exported V-tensors and packed weights rebuild f (the separable sum
    of Sec. 4, evaluated here in FP64 numpy) to the oracle's value."""
    W = small_case()
    log("case export_vtensors", W.grid.n)
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        (vx, vy, vz), tp = ctx.export_vtensors(W.grid)
        info = ctx.query()
    R = vx.shape[0]
    assert R == info["prim_comp_pairs_kept"] == info["prim_pairs_total"]
    vx, vy, vz, tp = (np.asarray(a, np.complex128 if np.iscomplexobj(a) else np.float64) for a in (vx, vy, vz, tp))
    f = np.einsum("st,ti,tj,tk->sijk", tp, vx, vy, vz, optimize=True)
    ref = oracle_mod.eval_grid(W.mol, W.T, W.grid, n_threads=NTH)
    e = errors(f, ref)
    log(f"[export] R={R}: peak-normalised |f|^2 err {e['f2_peak_norm'].max():.3e}")
    assert e["f2_peak_norm"].max() <= TOL_F2["fp32"]


def test_spin_factor_scales_f(binding):
    """f is linear in the spin factor: f(sqrt 2) = sqrt 2 f(1)."""
    W = small_case()
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f1, _ = ctx.eval_grid_host(W.grid, "fp32")
        ctx.set_options(0.0, np.sqrt(2.0))
        f2, _ = ctx.eval_grid_host(W.grid, "fp32")
    scale = np.abs(f1).max()
    assert np.abs(f2 - np.sqrt(2.0) * f1).max() <= 2e-6 * scale


def test_translation_phase(binding):
    """Translating the molecule by d multiplies f by exp(i q.d): |f|^2 is
    unchanged and the phase follows (d of 20 bohr stresses the FP64 phase)."""
    W = small_case()
    d = np.array([20.0, -13.0, 7.5])
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f0, _ = ctx.eval_grid_host(W.grid, "fp32")
        ctx.load_molecule(W.mol.translated(d))
        ctx.load_transitions(W.T)
        f1, _ = ctx.eval_grid_host(W.grid, "fp32")
    q = W.grid.points().reshape(W.grid.n + (3,))
    phase = np.exp(1j * (q @ d))
    scale = np.abs(f0).max()
    assert np.abs(f1 - phase[None] * f0).max() <= 2e-6 * scale


def test_single_outputs_and_device_T(binding):
    """f only, |f|^2 only, and T taken from device memory give the same
    numbers as the full host call."""
    import torch
    W = small_case()
    ns = W.T.shape[0]
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f_ref, f2_ref = ctx.eval_grid_host(W.grid, "fp32")
        T_dev = torch.from_numpy(np.ascontiguousarray(W.T)).to("cuda:0")
        ctx.load_transitions_device(T_dev)
        f = torch.empty((ns,) + W.grid.n + (2,), dtype=torch.float32, device="cuda:0")
        f2 = torch.empty((ns,) + W.grid.n, dtype=torch.float32, device="cuda:0")
        ctx.eval_grid_device(W.grid, f, None)
        ctx.eval_grid_device(W.grid, None, f2)
        torch.cuda.synchronize()
        fh = f.cpu().numpy()
        fc = fh[..., 0] + 1j * fh[..., 1]
        assert np.array_equal(fc, f_ref)
        assert np.array_equal(f2.cpu().numpy(), f2_ref)


def test_error_paths_on_device(binding):
    """State and budget errors on a real device leave the context usable."""
    W = small_case()
    with binding.Context(0) as ctx:
        with pytest.raises(binding.ScffError) as ei:
            ctx.eval_grid_host(W.grid, "fp32")
        assert ei.value.code == binding.SCFF_ESTATE
        ctx.load_molecule(W.mol)
        with pytest.raises(binding.ScffError) as ei:
            ctx.eval_grid_host(W.grid, "fp32")     # no transitions yet
        assert ei.value.code == binding.SCFF_ESTATE
        ctx.load_transitions(W.T)
        f, _ = ctx.eval_grid_host(W.grid, "fp32")
        assert np.isfinite(f).all()
    # a 64 KiB budget cannot hold the tables and outputs: some step must refuse
    with binding.Context(0, hbm_budget_bytes=64 << 10) as tiny:
        with pytest.raises(binding.ScffError) as ei:
            tiny.load_molecule(W.mol)
            tiny.load_transitions(W.T)
            tiny.eval_grid_host(W.grid, "fp32")
        assert ei.value.code == binding.SCFF_ENOMEM


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_split_falls_back_under_budget(binding, oracle_mod, precision):
    """A grid of few tiles splits its pair sums over several workgroups per
    tile (an FP64 partial buffer, reserved last).  A context whose HBM budget
    is one byte short of that evaluation's footprint evaluates the grid
    unsplit instead: no error, the same values up to the order of the FP64
    sums, and both within the tolerance of the oracle."""
    W = small_case()
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f_split, f2_split = ctx.eval_grid_host(W.grid, precision)
        full = ctx.query()["device_bytes"]
    with binding.Context(0, hbm_budget_bytes=full - 1) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f_one, f2_one = ctx.eval_grid_host(W.grid, precision)
        held = ctx.query()["device_bytes"]
    log(f"[split fallback] {precision}: footprint split {full} B, unsplit {held} B")
    assert held < full
    ref = oracle_mod.eval_grid(W.mol, W.T, W.grid, n_threads=NTH)
    for f, f2 in ((f_split, f2_split), (f_one, f2_one)):
        e = errors(f, ref)
        assert e["f2_peak_norm"].max() <= TOL_F2[precision], e["f2_peak_norm"]
        np.testing.assert_allclose(f2, np.abs(f) ** 2, rtol=2e-6, atol=1e-12 * np.abs(f).max() ** 2)
    scale = np.abs(f_split).max()
    assert np.abs(f_one - f_split).max() <= 1e-5 * scale


def test_points_match_grid(binding):
    """eval_points at the grid's own points equals eval_grid (same sums,
    evaluated point-wise with on-the-fly V-tensors)."""
    W = small_case()
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        fg, _ = ctx.eval_grid_host(W.grid, "fp32")
        fp, _ = ctx.eval_points(W.grid.points())
    fg = fg.reshape(fg.shape[0], -1)
    scale = np.abs(fg).max()
    assert np.abs(fp - fg).max() <= 2e-6 * scale


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("nx", [13, 12])
def test_symmetric_grid_mode(binding, oracle_mod, precision, nx):
    """Symmetric-grid mode: on a grid symmetric about q = 0 the planes
    ix < ceil(nx/2) are the full evaluation's values bit for bit, every other
    plane is exactly the conjugate of its mirror (f(-q) = f(q)* for real T),
    and the whole grid matches the oracle; a grid that is not symmetric is
    evaluated in full, bit for bit as without the mode."""
    W = wl.make_config(0)
    sym = wl.Grid(n=(nx, 10, 37), qmin=(-5.0, -4.5, -6.0), qmax=(5.0, 4.5, 6.0))
    asym = small_case().grid
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f_full, _ = ctx.eval_grid_host(sym, precision)
        fa_full, fa2_full = ctx.eval_grid_host(asym, precision)
        ctx.set_symmetry(True)
        f_sym, f2_sym = ctx.eval_grid_host(sym, precision)
        fa_sym, fa2_sym = ctx.eval_grid_host(asym, precision)
    h = (nx + 1) // 2
    assert np.array_equal(f_sym[:, :h], f_full[:, :h])
    mirror = f_sym[:, nx - h - 1::-1, ::-1, ::-1] if nx - h > 0 else f_sym[:, :0]
    assert np.array_equal(f_sym[:, h:], np.conj(mirror))
    assert np.array_equal(f2_sym[:, h:], f2_sym[:, nx - h - 1::-1, ::-1, ::-1])
    assert np.array_equal(fa_sym, fa_full) and np.array_equal(fa2_sym, fa2_full)
    e = errors(f_sym, oracle_mod.eval_grid(W.mol, W.T, sym, n_threads=NTH))
    log(f"[symmetric nx={nx}] {precision}: peak-normalised |f|^2 err {e['f2_peak_norm'].max():.3e}")
    assert e["f2_peak_norm"].max() <= TOL_F2[precision]


@pytest.mark.parametrize("qy", [4.5, 0.0])
def test_symmetric_mode_one_point_axis(binding, oracle_mod, qy):
    """A one-point axis holds the single value q_min.  With q_y = -4.5 (and
    q_max = +4.5, unused) the grid is not symmetric about q = 0, so the mode
    must evaluate it in full (bit for bit as without the mode); with q_y = 0
    it is symmetric and the mirrored planes must still match the oracle."""
    W = wl.make_config(0)
    g = wl.Grid(n=(12, 1, 37), qmin=(-5.0, -qy, -6.0), qmax=(5.0, qy, 6.0))
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)
        ctx.set_options(0.0, 1.0)
        f_full, f2_full = ctx.eval_grid_host(g, "fp32")
        ctx.set_symmetry(True)
        f_sym, f2_sym = ctx.eval_grid_host(g, "fp32")
    if qy != 0.0:
        assert np.array_equal(f_sym, f_full) and np.array_equal(f2_sym, f2_full)
    e = errors(f_sym, oracle_mod.eval_grid(W.mol, W.T, g, n_threads=NTH))
    log(f"[one-point axis q_y={-qy}] peak-normalised |f|^2 err {e['f2_peak_norm'].max():.3e}")
    assert e["f2_peak_norm"].max() <= TOL_F2["fp32"]


def test_validated_precompute_tables(binding, monkeypatch):
    """With SCFF_VALIDATE set when the context is created, every precompute's
    term slots and chunk table are checked on the host before a kernel reads
    them; the engine's own tables pass, across screening levels, and the
    results equal an unvalidated context's bit for bit."""
    W = wl.make_config(0)
    g = small_case().grid
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SCFF_VALIDATE", flag)
        with binding.Context(0) as ctx:
            ctx.load_molecule(W.mol)
            ctx.load_transitions(W.T)
            res = []
            for eps in (0.0, 1e-9, 1e-6):
                ctx.set_options(eps, 1.0)
                res.append(ctx.eval_grid_host(g, "fp32"))
            outs.append(res)
    for (fa, f2a), (fb, f2b) in zip(*outs):
        assert np.array_equal(fa, fb) and np.array_equal(f2a, f2b)
