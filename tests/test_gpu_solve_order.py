"""CG and the mixed solvers on the reverse Cuthill-McKee solve order
(rp_plan_set_solve_order), against the oracle on the fused system.

The renumbered matrix is Q A Q^T, so the solve must meet the same bar as in
fused order: true relative residual <= 1e-8 by the oracle's own SpMV and
solution error <= 1e-6 against the oracle's x; iteration counts may differ
from the fused-order solve by rounding only (a few)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from helpers import share_values, share_ranks, oracle_system
from gpu_util import torch_mod, dev_tensor, make_plan, update, assert_bits_equal
from paper_2510_08536_amd import default_opts

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda: synth.build("c1"),
    "ragged_rcb7": lambda: synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True),
    "stretched": lambda: synth.small((12, 12, 20), ("rcb", 6), kappa=(1e-3, 1.0), seed=22, scramble=True,
                                     stretch=100.0),
    "rcb_mixed": lambda: synth.small((40, 20, 12), ("rcb", 3), kappa=(1e-2, 1.0), seed=24),
}


def _setup(name):
    w = CASES[name]()
    m, buf, val64, *_ = oracle_system(w)
    plan = make_plan(w)
    return w, m, val64, plan


def _check_against_oracle(m, val64, b, x, info, it_or=None):
    xh = x.cpu().numpy() if hasattr(x, "cpu") else x
    x_or = oracle.pcg(m, val64, b, tol=1e-8)[0]
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    assert info["status"] == 0 and rr <= 1e-8, (info, rr)
    assert abs(info["rel_res"] - rr) <= 1e-3 * rr + 1e-15
    assert err <= 1e-6, err


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_rr"])
def test_solve_in_rcm_order_matches_oracle(name, precision):
    w, m, val64, plan = _setup(name)
    plan.set_solve_order("rcm")          # before the first update
    update(plan, share_values(w))
    b = w.rhs()
    x, info = plan.solve(dev_tensor(b), tol=1e-8, precision=precision)
    _check_against_oracle(m, val64, b, x, info)
    if precision == "fp64":
        plan.set_solve_order("fused")
        x0, i0 = plan.solve(dev_tensor(b), tol=1e-8)
        assert abs(info["iters"] - i0["iters"]) <= max(3, int(0.02 * i0["iters"])), (info, i0)
    plan.close()


def test_order_is_a_permutation_that_narrows_the_band():
    w = CASES["ragged_rcb7"]()
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, share_ranks(w, 0, w.n_ranks))
    plan = make_plan(w)
    assert plan.solve_order() == (0, None)
    plan.set_solve_order(1)
    mode, perm = plan.solve_order()
    assert mode == 1 and np.array_equal(np.sort(perm), np.arange(m.n_rows))
    A = sp.csr_matrix((np.ones(m.nnz_local), np.asarray(m.col), np.asarray(m.row_ptr)), shape=(m.n_rows,) * 2)
    c, cp = A.tocoo(), A[perm][:, perm].tocoo()
    assert np.abs(cp.row - cp.col).max() * 4 < np.abs(c.row - c.col).max()
    # the plan's order is the host routine's on the fused pattern
    import paper_2510_08536_amd as rp
    assert np.array_equal(perm, rp.rcm_order(np.asarray(m.row_ptr), np.asarray(m.col)))
    plan.close()


def test_values_follow_updates_and_warm_start():
    """Enable after values exist, then change the values: the next solve
    gathers the new ones.  A warm start from the previous x is permuted in."""
    torch = torch_mod()
    w, m, val64, plan = _setup("ragged_rcb7")
    vals = share_values(w)
    update(plan, vals)
    plan.set_solve_order(1)
    b = w.rhs()
    x1, i1 = plan.solve(dev_tensor(b), tol=1e-8)
    _check_against_oracle(m, val64, b, x1, i1)
    vals2 = [{k: (v * 3.0 if k in ("diag", "upper", "iface") else v) for k, v in r.items()} for r in vals]
    update(plan, vals2)
    x2, i2 = plan.solve(dev_tensor(b), tol=1e-8)
    # 3 A x = b: x = x1 / 3, to the accuracy both solves reach (1e-6 against the oracle)
    x1h, x2h = x1.cpu().numpy(), x2.cpu().numpy()
    assert i2["status"] == 0
    assert np.linalg.norm(x2h - x1h / 3.0) <= 2e-6 * np.linalg.norm(x1h / 3.0)
    # warm start: x0 = the answer for these values needs (almost) no iterations
    x3 = x2.clone()
    o = default_opts(tol=1e-8, x0_zero=0)
    x3, i3 = plan.solve(dev_tensor(b), x=x3, opts=o)
    assert i3["status"] == 0 and i3["iters"] <= 2, i3
    plan.close()


def test_fused_order_unchanged_after_toggling():
    """Switching the solve order on and back off leaves the fused-order
    solve bit-identical to a plan that never used it."""
    torch = torch_mod()
    w = CASES["rcb_mixed"]()
    b = dev_tensor(w.rhs())
    ref = make_plan(w)
    update(ref, share_values(w))
    xr, ir = ref.solve(b, tol=1e-8)
    plan = make_plan(w)
    update(plan, share_values(w))
    plan.set_solve_order(1)
    plan.solve(b, tol=1e-8)
    plan.set_solve_order(0)
    x, i = plan.solve(b, tol=1e-8)
    assert_bits_equal(x.cpu().numpy(), xr.cpu().numpy(), "fused after toggling")
    assert i["iters"] == ir["iters"]
    ref.close()
    plan.close()


def test_graph_replay_in_rcm_order():
    torch = torch_mod()
    w, m, val64, plan = _setup("stretched")
    update(plan, share_values(w))
    plan.set_solve_order(1)
    b = dev_tensor(w.rhs())
    xe, ie = plan.solve(b, tol=1e-8, check_every=8)
    for rep in range(2):
        xg, ig = plan.solve(b, tol=1e-8, check_every=8, graph=1)
        assert_bits_equal(xg.cpu().numpy(), xe.cpu().numpy(), f"graph replay {rep}")
        assert ig["iters"] == ie["iters"]
    plan.close()


@pytest.mark.parametrize("transpose", [0, 1])
def test_bicgstab_in_rcm_order_matches_oracle(transpose):
    """Non-symmetric (convection-diffusion) values on a scrambled mesh:
    BiCGStab on the solve order, plain and transposed, against the oracle's
    BiCGStab on the fused system (or its explicit transpose)."""
    w = CASES["stretched"]()
    v = w.momentum_values(pe=4.0, sigma=1.0)
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, share_ranks(w))
    vals = share_values(w, values=v)
    val64, *_ = oracle.update(m, oracle.receive_buffer(vals))
    plan = make_plan(w)
    plan.set_solve_order(1)
    update(plan, vals, lower=True)
    A = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(m.n_rows,) * 2)
    if transpose:
        A = A.T.tocsr()
        A.sort_indices()
    b = w.rhs()
    x_or, st, *_ = oracle.bicgstab_csr(A.indptr, A.indices, A.data, b, tol=1e-8)
    assert st == 0
    x, info = plan.solve(dev_tensor(b), tol=1e-8, method="bicgstab", transpose=transpose)
    xh = x.cpu().numpy()
    rr = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
    assert info["status"] == 0 and rr <= 1e-8 * (1 + 1e-6), (info, rr)
    assert np.linalg.norm(xh - x_or) <= 1e-6 * np.linalg.norm(x_or)
    plan.close()


def test_bad_solve_order_is_refused():
    w, m, val64, plan = _setup("ragged_rcb7")
    import paper_2510_08536_amd.rp as low
    with pytest.raises(low.RpError):
        plan.set_solve_order(2)
    with pytest.raises(low.RpError):
        plan.set_solve_order(-1)
    assert plan.solve_order() == (0, None)
    plan.close()
