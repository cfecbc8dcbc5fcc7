"""The allocation-free evaluation entry point (scff_eval_grid_noalloc),
called through the C ABI and checked against scff_eval_grid's output on the
same context: two calls in a row, the second on a smaller problem (the
static scratch keeps the first call's contents, so stale data would show),
in both precisions; plus its refusals (no precompute yet, tables larger than
the scratch) and that the context's device memory does not grow."""
import ctypes

import numpy as np
import pytest

import workload as wl
from tests.metrics import TOL_F2, errors

pytestmark = pytest.mark.gpu


def raw_noalloc(binding, ctx, grid, precision, f, f2, stream):
    g = binding.make_grid(grid.n, grid.qmin, grid.qmax)
    return binding.scff_eval_grid_noalloc(ctx._h, ctypes.byref(g), binding.PRECISIONS[precision],
                                          f.data_ptr() if f is not None else None,
                                          f2.data_ptr() if f2 is not None else None,
                                          ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_noalloc_matches_eval_grid_twice(precision):
    import torch
    from paper_2512_18010_amd import binding
    big = wl.make_config(1)                      # 190 functions, 12 transitions, 64^3
    small = wl.make_config(0)
    small.grid = wl.Grid(n=(13, 11, 37), qmin=(-5.0, -4.0, -5.5), qmax=(5.0, 4.5, 5.0))   # split pair sums
    stream = torch.cuda.current_stream()
    with binding.Context(0) as ctx:
        for W in (big, small):
            print(f"noalloc {precision}: nbf={W.mol.nbf} grid={W.grid.n}", flush=True)
            ctx.load_molecule(W.mol)
            ctx.load_transitions(W.T)
            ctx.set_options(1e-9, 1.0)
            ctx.query()                          # runs the precompute (which allocates)
            shape = (W.T.shape[0],) + tuple(W.grid.n)
            f_ref = torch.empty(shape + (2,), dtype=torch.float32, device="cuda")
            f2_ref = torch.empty(shape, dtype=torch.float32, device="cuda")
            ctx.eval_grid_device(W.grid, f_ref, f2_ref, precision=precision, stream=stream)
            torch.cuda.synchronize()
            held = ctx.query()["device_bytes"]
            f = torch.full(shape + (2,), float("nan"), dtype=torch.float32, device="cuda")
            f2 = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
            rc = raw_noalloc(binding, ctx, W.grid, precision, f, f2, stream)
            assert rc == binding.SCFF_OK, binding.scff_last_error()
            torch.cuda.synchronize()
            assert ctx.query()["device_bytes"] == held
            fa, fb = f.cpu().numpy(), f_ref.cpu().numpy()
            e = errors(fa[..., 0] + 1j * fa[..., 1], fb[..., 0] + 1j * fb[..., 1])
            print(f"  against scff_eval_grid: peak-normalised |f|^2 difference {e['f2_peak_norm'].max():.3e}, "
                  f"identical {np.array_equal(fa, fb) and np.array_equal(f2.cpu().numpy(), f2_ref.cpu().numpy())}",
                  flush=True)
            assert np.isfinite(fa).all() and e["f2_peak_norm"].max() <= TOL_F2[precision]
            # the same split plan and kernels: the same bits
            assert np.array_equal(fa, fb) and np.array_equal(f2.cpu().numpy(), f2_ref.cpu().numpy())


def test_noalloc_refusals():
    import torch
    from paper_2512_18010_amd import binding
    W = wl.make_config(0)
    stream = torch.cuda.current_stream()
    with binding.Context(0) as ctx:
        ctx.load_molecule(W.mol)
        ctx.load_transitions(W.T)           # no precompute has run yet
        f2 = torch.empty((1,) + tuple(W.grid.n), dtype=torch.float32, device="cuda")
        assert raw_noalloc(binding, ctx, W.grid, "fp32", None, f2, stream) == binding.SCFF_ESTATE
        ctx.query()
        huge = wl.Grid(n=(4096, 4, 4), qmin=(-5.0,) * 3, qmax=(5.0,) * 3)   # tables beyond the scratch
        assert raw_noalloc(binding, ctx, huge, "fp32", None, None, stream) == binding.SCFF_EINVAL
        assert raw_noalloc(binding, ctx, W.grid, "fp32", None, f2, stream) == binding.SCFF_OK
        torch.cuda.synchronize()
