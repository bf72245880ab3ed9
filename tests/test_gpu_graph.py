"""CG iteration chunks replayed as HIP graphs (rp_solve_opts.graph = 1).

A replayed chunk runs the same kernels with the same arguments as the eager
launches, except that K2 and K3 read the iteration number from the device
state, so every replay must give the eager solve's x bit for bit, with the
same iteration counts and residual.  Each test replays the cached graph
several times, with eager solves and value updates between the replays."""
import numpy as np
import pytest

import synth
from helpers import share_values
from gpu_util import torch_mod, dev_tensor, make_plan, update, assert_bits_equal
from paper_2510_08536_amd import default_opts, RP_KERNEL_SPMV64

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda: synth.build("c1"),
    # oblique cut planes: some row groups offset-coded, the rest CSR
    "rcb_mixed": lambda: synth.small((40, 20, 12), ("rcb", 3), kappa=(1e-2, 1.0), seed=24),
    "ragged_rcb7": lambda: synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True),
}


def _scaled(vals, s):
    return [{k: (v * s if k in ("diag", "upper", "iface", "lower") else v) for k, v in r.items()} for r in vals]


def _solve(plan, b, x, **kw):
    x.zero_()
    o = default_opts(x0_zero=1, **kw)
    x, info = plan.solve(b, x=x, opts=o, check=False)
    return x.cpu().numpy(), info


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_rr"])
def test_graph_replays_match_eager(name, precision):
    torch = torch_mod()
    w = CASES[name]()
    plan = make_plan(w)
    v1 = share_values(w)
    v2 = _scaled(v1, 2.0)
    b = dev_tensor(w.rhs())
    x = torch.empty_like(b)
    kw = dict(tol=1e-8, precision=precision, check_every=16)
    update(plan, v1)
    xe1, ie1 = _solve(plan, b, x, **kw)
    update(plan, v2)
    xe2, ie2 = _solve(plan, b, x, **kw)
    assert ie1["status"] == 0 and ie2["status"] == 0, (ie1, ie2)
    for rep in range(3):
        update(plan, v1)
        xg, ig = _solve(plan, b, x, graph=1, **kw)
        assert_bits_equal(xg, xe1, f"{name} {precision} replay {rep} (values 1)")
        assert (ig["iters"], ig["outer_iters"], ig["rel_res"]) == (ie1["iters"], ie1["outer_iters"], ie1["rel_res"])
        # eager work between the replays
        xe, _ = _solve(plan, b, x, **kw)
        assert_bits_equal(xe, xe1, f"{name} {precision} eager after replay {rep}")
        update(plan, v2)
        xg, ig = _solve(plan, b, x, graph=1, **kw)
        assert_bits_equal(xg, xe2, f"{name} {precision} replay {rep} (values 2)")
        assert ig["iters"] == ie2["iters"]
    # another output vector: the graph is captured again
    x_other = torch.empty_like(b)
    xg, ig = _solve(plan, b, x_other, graph=1, **kw)
    assert_bits_equal(xg, xe2, f"{name} {precision} new x")
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("check_every", [1, 16])
def test_graph_budget_not_a_multiple_of_the_chunk(precision, check_every):
    """max_iter = 45: the last replay runs past the budget and its kernels must
    do nothing, leaving the eager result and count."""
    torch = torch_mod()
    w = synth.build("c1")
    plan = make_plan(w)
    update(plan, share_values(w))
    b = dev_tensor(w.rhs())
    x = torch.empty_like(b)
    kw = dict(tol=1e-14, precision=precision, check_every=check_every, max_iter=45)
    xe, ie = _solve(plan, b, x, **kw)
    assert ie["status_name"] == "RP_NOT_CONVERGED" and ie["iters"] == 45, ie
    for rep in range(2):
        xg, ig = _solve(plan, b, x, graph=1, **kw)
        assert ig["status"] == ie["status"] and ig["iters"] == 45, ig
        assert_bits_equal(xg, xe, f"{precision} chunk {check_every} replay {rep}")
        assert ig["rel_res"] == ie["rel_res"]
    plan.close()


def test_graph_on_a_side_stream():
    torch = torch_mod()
    w = synth.build("c1")
    plan = make_plan(w)
    update(plan, share_values(w))
    b = dev_tensor(w.rhs())
    x = torch.empty_like(b)
    xe, ie = _solve(plan, b, x, tol=1e-8)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for rep in range(2):
        with torch.cuda.stream(s):
            x.zero_()
            o = default_opts(x0_zero=1, tol=1e-8, graph=1)
            xs, ig = plan.solve(b, x=x, opts=o, stream=s)
        s.synchronize()
        assert_bits_equal(xs.cpu().numpy(), xe, f"side stream replay {rep}")
        assert ig["iters"] == ie["iters"]
    plan.close()


def test_graph_ignored_while_timing():
    """Kernel timing needs events around each SpMV: the solve launches eagerly
    and every SpMV is counted."""
    torch = torch_mod()
    w = synth.build("c1")
    plan = make_plan(w)
    update(plan, share_values(w))
    b = dev_tensor(w.rhs())
    x = torch.empty_like(b)
    xe, ie = _solve(plan, b, x, tol=1e-8)
    plan.set_timing(True)
    xg, ig = _solve(plan, b, x, tol=1e-8, graph=1)
    n, ms = plan.kernel_stats(RP_KERNEL_SPMV64)
    plan.set_timing(False)
    assert_bits_equal(xg, xe, "timed")
    assert n == ig["iters"] and ms > 0, (n, ig["iters"], ms)
    plan.close()


def test_graph_option_is_checked():
    torch = torch_mod()
    w = synth.build("c1")
    plan = make_plan(w)
    update(plan, share_values(w))
    b = dev_tensor(w.rhs())
    x, info = plan.solve(b, opts=default_opts(graph=2), check=False)
    assert info["status_name"] == "RP_ERR_ARG"
    plan.close()
