"""The Python binding checks every buffer it hands to the C side as a raw
pointer (dtype, shape against the loaded problem, contiguity, device) and
raises ValueError before any call into the library.  CPU only: the checks
fire before a device is touched."""
import numpy as np
import pytest
import torch

import workload as wl
from paper_2512_18010_amd import binding


def fake_context(nbf=44, n_states=2):
    """A Context object with a loaded-problem state but no library handle:
    any call that reached the C side would fail on the NULL context."""
    ctx = object.__new__(binding.Context)
    ctx._h = None
    ctx.device = 0
    ctx.nbf = nbf
    ctx.n_states = n_states
    return ctx


GRID = wl.Grid(n=(4, 5, 6), qmin=(-1.0,) * 3, qmax=(1.0,) * 3)


def test_device_outputs_are_checked():
    ctx = fake_context()
    shape = (2, 4, 5, 6)
    bad = [
        dict(f=torch.empty(shape + (2,), dtype=torch.float32)),                    # host tensor
        dict(f2=torch.empty(shape, dtype=torch.float32)),                          # host tensor
        dict(f=torch.empty(shape + (2,), dtype=torch.float16)),                    # dtype
        dict(f=torch.empty((2, 4, 5, 5, 2), dtype=torch.float32)),                 # undersized
        dict(f2=torch.empty((1,) + shape[1:], dtype=torch.float32)),               # too few states
        dict(f2=torch.empty((2, 4, 6, 5), dtype=torch.float32).transpose(2, 3)),   # not contiguous
        dict(f=np.empty(shape + (2,), np.float32)),                                # not a tensor
    ]
    for kw in bad:
        with pytest.raises(ValueError):
            ctx.eval_grid_device(GRID, **kw)


def test_device_transitions_are_checked():
    ctx = fake_context()
    for T in (torch.zeros((2, 44, 44), dtype=torch.float64),          # host tensor
              torch.zeros((2, 44, 44), dtype=torch.float32),          # dtype
              torch.zeros((2, 44, 43), dtype=torch.float64),          # shape
              torch.zeros((44, 44), dtype=torch.float64)):            # no state axis
        with pytest.raises(ValueError):
            ctx.load_transitions_device(T)


def test_host_transitions_are_checked():
    ctx = fake_context()
    with pytest.raises(ValueError):
        ctx.load_transitions(np.zeros((2, 44, 40)))
    with pytest.raises(ValueError):
        ctx.load_transitions(np.zeros((44, 45)))


def test_molecule_array_lengths_are_checked():
    W = wl.make_config(0)
    arrs, nbf = binding._molecule_arrays(W.mol)
    assert nbf == W.mol.nbf == 44
    import dataclasses
    for bad in (dataclasses.replace(W.mol, exps=W.mol.exps[:-1]),
                dataclasses.replace(W.mol, coefs=np.concatenate([W.mol.coefs, [1.0]])),
                dataclasses.replace(W.mol, shell_l=W.mol.shell_l[:-1]),
                dataclasses.replace(W.mol, xyz=W.mol.xyz[:, :2])):
        with pytest.raises(ValueError):
            binding._molecule_arrays(bad)


def test_server_submit_checks_T_against_the_basis():
    W = wl.make_config(0)
    with binding.Server(-1, 1 << 30, 2) as srv:   # scheduler test mode: no GPU
        with pytest.raises(ValueError):
            srv.submit(W.mol, np.zeros((1, 44, 43)), W.grid)
        t = srv.submit(W.mol, W.T, W.grid)        # a well-formed request still goes through
        st, _, _, _ = srv.wait(t)
        assert st == 0
