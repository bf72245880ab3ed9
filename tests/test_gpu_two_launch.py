"""The two-launch CG iteration against the three-launch one and the oracle.

With rp_solve_opts.fused_loop = RP_LOOP_AUTO (the default), a Jacobi CG
solve on at most RP_LOOP_TWO_MAX_ROWS rows runs each iteration as two
launches: the r update, then the x and p update of that iteration fused with
the SpMV of the next one, where every row forms the new p of its columns
itself.  The fused kernel takes every p entry by the same operations as the
three-launch x and p update, gives rows to blocks as the SpMV does and sums
each row in column order, so the bar against RP_LOOP_THREE is bit-identical
x, iteration counts and residuals.  Against the oracle the solve bars hold:
true relative residual <= 1e-8 by the oracle's SpMV, error <= 1e-6 against
the oracle's x, iteration count within rounding of the oracle's, and for a
fixed iteration budget the iterate within 1e-10 of the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from helpers import share_values, oracle_system
from gpu_util import dev_tensor, make_plan, update, torch_mod
from paper_2510_08536_amd import RP_LOOP_AUTO, RP_LOOP_THREE, RP_LOOP_TWO_MAX_ROWS, RP_NOT_CONVERGED

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda: synth.build("c1"),
    "c4fd": lambda: synth.build("c4fd"),
    "ragged_rcb7": lambda: synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True),
    "stretched": lambda: synth.small((12, 12, 20), ("rcb", 6), kappa=(1e-3, 1.0), seed=22, scramble=True,
                                     stretch=100.0),
    "chain": lambda: synth.small((300, 1, 1), ("blocks", 5, 1, 1), seed=23, walls=(True, False, False)),
    "box27": lambda: synth.small((10, 9, 8), ("blocks", 2, 1, 1), kappa=(1e-2, 1.0), seed=25, stencil=27),
    "single_row_groups": lambda: synth.small((3, 2, 1), ("blocks", 1, 1, 1), seed=27),
}

KEYS = ("status", "iters", "outer_iters", "restarts", "rel_res")


def _setup(w):
    m, buf, val64, *_ = oracle_system(w)
    plan = make_plan(w)
    update(plan, share_values(w))
    return m, val64, plan


def _same(a, b):
    (xa, ia), (xb, ib) = a, b
    torch = torch_mod()
    assert torch.equal(xa, xb), float((xa - xb).abs().max())
    assert all(ia[k] == ib[k] for k in KEYS), (ia, ib)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_rr"])
def test_two_launch_equals_three_and_meets_the_oracle(name, precision):
    w = CASES[name]()
    m, val64, plan = _setup(w)
    assert plan.n_rows <= RP_LOOP_TWO_MAX_ROWS
    b = w.rhs()
    x_or, st, it_or, rs_or, _ = oracle.pcg(m, val64, b, tol=1e-8)
    assert st == 0 and rs_or == 0
    res = {fl: plan.solve(dev_tensor(b), tol=1e-8, precision=precision, fused_loop=fl)
           for fl in (RP_LOOP_AUTO, RP_LOOP_THREE)}
    _same(res[RP_LOOP_AUTO], res[RP_LOOP_THREE])
    x, info = res[RP_LOOP_AUTO]
    xh = x.cpu().numpy()
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    print(f"{name} {precision}: {info['iters']} it (oracle {it_or}), {info['outer_iters']} outer, "
          f"rel.res {rr:.2e}, err {err:.2e}")
    assert info["status"] == 0 and info["restarts"] == 0 and rr <= 1e-8, (info, rr)
    assert err <= 1e-6, err
    if precision == "fp64":
        assert abs(info["iters"] - it_or) <= max(3, int(0.02 * it_or)), (info["iters"], it_or)
    plan.close()


@pytest.mark.parametrize("max_iter", [1, 2, 5, 37])
@pytest.mark.parametrize("check_every", [1, 3, 32])
def test_two_launch_budgets_and_chunks(max_iter, check_every):
    """An iteration budget that ends inside or at the end of a host chunk:
    the iterate is the three-launch one and the oracle's after max_iter."""
    w = CASES["c4fd"]()
    m, val64, plan = _setup(w)
    b = w.rhs()
    xo, st, it, *_ = oracle.pcg(m, val64, b, tol=1e-8, max_iter=max_iter)
    assert st == 1 and it == max_iter
    res = {fl: plan.solve(dev_tensor(b), tol=1e-8, max_iter=max_iter, check_every=check_every, fused_loop=fl,
                          check=False) for fl in (RP_LOOP_AUTO, RP_LOOP_THREE)}
    _same(res[RP_LOOP_AUTO], res[RP_LOOP_THREE])
    x, info = res[RP_LOOP_AUTO]
    assert info["status"] == RP_NOT_CONVERGED and info["iters"] == max_iter, info
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    plan.close()


def test_two_launch_largest_size():
    """64^3 = RP_LOOP_TWO_MAX_ROWS rows, the largest system that takes two
    launches, in FP64 and both mixed forms."""
    w = synth.small((64, 64, 64), ("blocks", 2, 2, 2), kappa=(1e-2, 1.0), seed=28)
    m, val64, plan = _setup(w)
    assert plan.n_rows == RP_LOOP_TWO_MAX_ROWS
    b = w.rhs()
    x_or, st, it_or, *_ = oracle.pcg(m, val64, b, tol=1e-8)
    assert st == 0
    for precision in ("fp64", "mixed", "mixed_rr"):
        res = {fl: plan.solve(dev_tensor(b), tol=1e-8, precision=precision, fused_loop=fl)
               for fl in (RP_LOOP_AUTO, RP_LOOP_THREE)}
        _same(res[RP_LOOP_AUTO], res[RP_LOOP_THREE])
        x, info = res[RP_LOOP_AUTO]
        xh = x.cpu().numpy()
        rr = oracle.true_relres(m, val64, b, xh)
        err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
        print(f"64^3 {precision}: {info['iters']} it (oracle {it_or}), rel.res {rr:.2e}, err {err:.2e}")
        assert info["status"] == 0 and rr <= 1e-8 and err <= 1e-6, (info, rr, err)
    plan.close()


def test_two_launch_repeated_solves_keep_no_state():
    """Solves on one plan in turn with two and three launches, from zero and
    warm-started: each equals the three-launch solve of the same input."""
    w = CASES["ragged_rcb7"]()
    m, val64, plan = _setup(w)
    b = dev_tensor(w.rhs())
    ref = plan.solve(b, tol=1e-6, fused_loop=RP_LOOP_THREE)
    x0 = ref[0] * 0.5
    warm = plan.solve(b, x=x0.clone(), tol=1e-9, fused_loop=RP_LOOP_THREE)
    for fl in (RP_LOOP_AUTO, RP_LOOP_THREE, RP_LOOP_AUTO, RP_LOOP_AUTO):
        _same(plan.solve(b, tol=1e-6, fused_loop=fl), ref)
        _same(plan.solve(b, x=x0.clone(), tol=1e-9, fused_loop=fl), warm)
    plan.close()


def test_two_launch_on_the_solve_order():
    """The reverse Cuthill-McKee solve order: plain CSR rows of the
    renumbered copy, two launches against three."""
    w = CASES["stretched"]()
    m, val64, plan = _setup(w)
    plan.set_solve_order("rcm")
    b = w.rhs()
    for precision in ("fp64", "mixed_rr"):
        res = {fl: plan.solve(dev_tensor(b), tol=1e-8, precision=precision, fused_loop=fl)
               for fl in (RP_LOOP_AUTO, RP_LOOP_THREE)}
        _same(res[RP_LOOP_AUTO], res[RP_LOOP_THREE])
        x, info = res[RP_LOOP_AUTO]
        assert info["status"] == 0 and oracle.true_relres(m, val64, b, x.cpu().numpy()) <= 1e-8
    plan.close()


def test_two_launch_breakdown_on_indefinite_matrix():
    """diag 1, coupling -2, b the eigenvector of eigenvalue -1: (p, A p) < 0
    at the first iteration, reported as the oracle reports it."""
    from paper_2510_08536_amd import Plan, RP_ERR_BREAKDOWN
    n = 2
    ranks = [dict(owner=np.array([0], np.int32), neighbour=np.array([1], np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    plan = Plan([n], 0, 1, ranks)
    plan.update([np.array([1.0, 1.0])], [np.array([-2.0])], [np.zeros(0)])
    b = np.array([1.0, 1.0])
    m = oracle.merge([n], 0, 1, ranks)
    v64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=[1.0, 1.0], upper=[-2.0], iface=[])]))
    xo, st, it, *_ = oracle.pcg(m, v64, b)
    assert st == -6
    x, info = plan.solve(dev_tensor(b), fused_loop=RP_LOOP_AUTO, check=False)
    assert info["status"] == RP_ERR_BREAKDOWN and info["iters"] == it, (info, it)
    plan.close()
