"""rp_update_values_noalloc against rp_update_values.

The allocation-free update keeps its pointer table in a fixed device array
shared by every call on the GPU, so this checks two calls in a row, the
second on a smaller plan (fewer ranks, shorter table) after the first left a
longer table behind: each result must equal the plan-memory update's bit for
bit (val64, val32, dinv64, dinv32), and the error reporting must match (a
non-finite value, a non-symmetric update).  Host arrays and shares above the
table's size are refused before any device work."""
import numpy as np
import pytest

import synth
from helpers import share_values
from gpu_util import torch_mod, dev_tensor, make_plan, assert_bits_equal

pytestmark = pytest.mark.gpu


def _dev(vals, lower=False):
    d = [dev_tensor(v["diag"]) for v in vals]
    u = [dev_tensor(v["upper"]) for v in vals]
    i = [dev_tensor(v["iface"]) for v in vals]
    lo = [dev_tensor(v["lower"]) for v in vals] if lower else None
    return d, u, i, lo


_loaded = [False]


def _noalloc(plan, d, u, i, lo=None):
    """One rp_update_values_noalloc call.  The first call in the process loads
    the library's code object holding the fixed array (the runtime maps it
    once per GPU); every later call must leave the device's free memory
    unchanged."""
    torch = torch_mod()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan.update_noalloc(d, u, i, lower=lo)
    torch.cuda.synchronize()
    if _loaded[0]:
        assert torch.cuda.mem_get_info()[0] == free0, "the call allocated device memory"
    _loaded[0] = True


def _both(w, vals, lower=False):
    """values after rp_update_values and after rp_update_values_noalloc"""
    d, u, i, lo = _dev(vals, lower)
    ref_plan = make_plan(w)
    ref_plan.update(d, u, i, lower=lo)
    want = ref_plan.get_values()
    ref_plan.close()
    plan = make_plan(w)
    _noalloc(plan, d, u, i, lo)
    got = plan.get_values()
    return plan, got, want


def test_noalloc_matches_update_twice_second_smaller():
    big = synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True)
    small = synth.small((9, 6, 5), ("blocks", 3, 1, 1), kappa=(1e-2, 1.0), seed=5)
    assert small.n_ranks < big.n_ranks
    for w, lower in ((big, False), (small, False), (big, True), (small, True)):
        vals = share_values(w) if not lower else share_values(w, values=w.momentum_values())
        plan, got, want = _both(w, vals, lower)
        for g, wv, what in zip(got, want, ("val64", "val32", "dinv64", "dinv32")):
            assert_bits_equal(g, wv, f"{w.n_ranks} ranks lower={lower} {what}")
        plan.close()


def test_noalloc_reports_value_and_symmetry_errors():
    from paper_2510_08536_amd import RP_ERR_VALUE, RP_ERR_UNSUPPORTED, RpError
    w = synth.small((9, 6, 5), ("blocks", 3, 1, 1), kappa=(1e-2, 1.0), seed=5)
    plan = make_plan(w)
    b = dev_tensor(w.rhs())
    vals = share_values(w)
    bad = [dict(v) for v in vals]
    bad[1] = dict(bad[1], upper=bad[1]["upper"].copy())
    bad[1]["upper"][2] = np.inf
    d, u, i, _ = _dev(bad)
    _noalloc(plan, d, u, i)
    with pytest.raises(RpError) as e:
        plan.solve(b)
    assert e.value.code == RP_ERR_VALUE
    mv = share_values(w, values=w.momentum_values())
    d, u, i, lo = _dev(mv, lower=True)
    _noalloc(plan, d, u, i, lo)
    with pytest.raises(RpError) as e:
        plan.solve(b)
    assert e.value.code == RP_ERR_UNSUPPORTED
    d, u, i, _ = _dev(vals)
    _noalloc(plan, d, u, i)
    x, info = plan.solve(b)
    assert info["status"] == 0
    plan.close()


def test_noalloc_refuses_host_arrays_and_large_shares():
    from paper_2510_08536_amd import RP_ERR_ARG, RpError
    from paper_2510_08536_amd.rp import RP_NOALLOC_MAX_RANKS
    w = synth.small((9, 6, 5), ("blocks", 3, 1, 1), kappa=(1e-2, 1.0), seed=5)
    plan = make_plan(w)
    vals = share_values(w)
    host = [np.ascontiguousarray(v["diag"]) for v in vals]
    d, u, i, _ = _dev(vals)
    with pytest.raises(RpError) as e:
        plan.update_noalloc(host, u, i)
    assert e.value.code == RP_ERR_ARG
    plan.close()
    # a chain of one-cell ranks, one more than the table holds
    n = RP_NOALLOC_MAX_RANKS + 1
    wc = synth.small((n, 1, 1), ("blocks", n, 1, 1), seed=2, walls=(True, False, False))
    plan = make_plan(wc)
    vals = share_values(wc)
    d, u, i, _ = _dev(vals)
    with pytest.raises(RpError) as e:
        plan.update_noalloc(d, u, i)
    assert e.value.code == RP_ERR_ARG and "at most" in str(e.value)
    plan.close()
