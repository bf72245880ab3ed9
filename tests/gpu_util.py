"""GPU-test plumbing: build plans through the C-ABI binding and move arrays."""
from __future__ import annotations

import numpy as np

from helpers import share_ranks, share_values


def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def dev_tensor(a):
    torch = torch_mod()
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def make_plan(w, first=0, alpha=None):
    from paper_2510_08536_amd import Plan
    alpha = w.n_ranks - first if alpha is None else alpha
    return Plan(w.part.n_cells, first, alpha, share_ranks(w, first, alpha))


def update(plan, vals, where="device", lower=False):
    """vals: list of per-rank dicts (diag, upper, iface[, lower])."""
    conv = dev_tensor if where == "device" else (lambda a: np.ascontiguousarray(a, dtype=np.float64))
    plan.update([conv(v["diag"]) for v in vals], [conv(v["upper"]) for v in vals],
                [conv(v["iface"]) for v in vals],
                lower=[conv(v["lower"]) for v in vals] if lower else None)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype.itemsize == 8 else np.uint32)


def assert_bits_equal(got, want, what):
    got, want = np.asarray(got), np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    diff = np.nonzero(bits(got) != bits(want))[0]
    assert diff.size == 0, f"{what}: {diff.size} mismatches, first at {diff[:5]}: {got[diff[:5]]} vs {want[diff[:5]]}"
