"""GPU Jacobi-PCG (FP64) and mixed FP32/FP64 refinement against the oracle.

Tolerances: the solve must reach a true relative residual <= 1e-8 (computed
by the oracle's own SpMV on the GPU answer) and, on the moderately
conditioned cases here, a solution error <= 1e-6 against the oracle's x.
Iteration counts of GPU and oracle may differ by rounding (different
reduction order), by a few iterations at most."""
import numpy as np
import pytest

import oracle
import synth
from helpers import share_values, oracle_system, random_ldu_values
from gpu_util import torch_mod, dev_tensor, make_plan, update

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda: synth.build("c1"),
    "c4fd": lambda: synth.build("c4fd"),
    "ragged_rcb7": lambda: synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True),
    "stretched": lambda: synth.small((12, 12, 20), ("rcb", 6), kappa=(1e-3, 1.0), seed=22, scramble=True,
                                     stretch=100.0),
    "chain": lambda: synth.small((300, 1, 1), ("blocks", 5, 1, 1), seed=23, walls=(True, False, False)),
    # oblique cut planes: some row groups offset-coded, the rest CSR
    "rcb_mixed": lambda: synth.small((40, 20, 12), ("rcb", 3), kappa=(1e-2, 1.0), seed=24),
}


def _setup(name):
    w = CASES[name]()
    m, buf, val64, *_ = oracle_system(w)
    plan = make_plan(w)
    update(plan, share_values(w))
    return w, m, val64, plan


def _iters_close(a, b):
    return abs(a - b) <= max(3, int(0.02 * b))


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_rr"])
def test_solve_matches_oracle(name, precision):
    w, m, val64, plan = _setup(name)
    b = w.rhs()
    x_or, st, it_or, rs_or, rr_or = oracle.pcg(m, val64, b, tol=1e-8)
    assert st == 0 and rs_or == 0
    x, info = plan.solve(dev_tensor(b), tol=1e-8, precision=precision)
    xh = x.cpu().numpy()
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    assert info["status"] == 0 and rr <= 1e-8, (info, rr)
    assert info["restarts"] == 0, info
    assert abs(info["rel_res"] - rr) <= 1e-3 * rr + 1e-15
    assert err <= 1e-6, err
    if precision == "fp64":
        assert _iters_close(info["iters"], it_or), (info["iters"], it_or)
    else:
        assert info["outer_iters"] >= 1
    plan.close()


def test_sine_eigenvector_one_iteration():
    N = 16
    w = synth.small((N, N, N), ("blocks", 2, 2, 1), seed=1)
    m, buf, val64, *_ = oracle_system(w)
    plan = make_plan(w)
    update(plan, share_values(w))
    h = 1.0 / (N + 1)
    nat = np.arange(w.n_cells)
    i, j, k = nat % N + 1, (nat // N) % N + 1, nat // (N * N) + 1
    v = w.merged(np.sin(np.pi * 3 * i * h) * np.sin(np.pi * j * h) * np.sin(np.pi * 2 * k * h))
    lam = 6 - 2 * np.cos(np.pi * 3 * h) - 2 * np.cos(np.pi * h) - 2 * np.cos(np.pi * 2 * h)
    x, info = plan.solve(dev_tensor(v), tol=1e-10)
    assert info["iters"] == 1
    assert np.max(np.abs(x.cpu().numpy() - v / lam)) < 1e-13
    plan.close()


def test_tridiagonal_closed_form():
    N = 200
    w = synth.small((N, 1, 1), ("blocks", 4, 1, 1), seed=3, walls=(True, False, False))
    m, buf, val64, *_ = oracle_system(w)
    plan = make_plan(w)
    update(plan, share_values(w))
    idx = np.arange(1, N + 1)
    Ainv = np.minimum.outer(idx, idx) * (N + 1 - np.maximum.outer(idx, idx)) / (N + 1)
    b = np.random.default_rng(6).uniform(-1, 1, N)
    for prec in ("fp64", "mixed", "mixed_rr"):
        x, info = plan.solve(dev_tensor(b), tol=1e-12 if prec == "fp64" else 1e-10, precision=prec)
        ref = Ainv @ b
        assert np.max(np.abs(x.cpu().numpy() - ref)) <= 1e-8 * np.max(np.abs(ref)), prec
    plan.close()


def test_deterministic_and_chunk_independent():
    w, m, val64, plan = _setup("ragged_rcb7")
    b = dev_tensor(w.rhs())
    runs = []
    for ce in (1, 7, 32, 1000):
        x, info = plan.solve(b, tol=1e-8, check_every=ce)
        runs.append((x.cpu().numpy(), info["iters"]))
    for x, it in runs[1:]:
        assert it == runs[0][1]
        assert np.array_equal(x.view(np.uint64), runs[0][0].view(np.uint64))
    plan.close()


def test_windows_do_not_change_solves():
    """Staging x through LDS windows changes where x is read, not the result:
    FP64 and mixed solves are bit-identical either way."""
    w, m, val64, plan = _setup("c1")
    b = dev_tensor(w.rhs())
    for prec in ("fp64", "mixed"):
        plan.set_spmv_windows(False)
        x0, i0 = plan.solve(b, precision=prec)
        plan.set_spmv_windows(True)
        x1, i1 = plan.solve(b, precision=prec)
        assert i0["iters"] == i1["iters"] and torch_mod().equal(x0, x1), prec
    plan.close()


FORM_CASES = {
    # 27-point stencil: more offsets than a coded group holds (CSR groups only)
    "box27": lambda: synth.small((10, 9, 8), ("blocks", 2, 1, 1), kappa=(1e-2, 1.0), seed=25, stencil=27),
    # rank rows of 64 cells: offsets +-1, +-64, +-384 in every coded group
    "rows64": lambda: synth.small((64, 6, 8), ("blocks", 1, 1, 2), kappa=(1e-3, 1.0), seed=26),
}


@pytest.mark.parametrize("name", ["c1", "rcb_mixed", "ragged_rcb7", "chain", "stretched", "box27", "rows64"])
def test_spmv_form_does_not_change_solves(name):
    """The offset-coded and the CSR index form give the same products and row
    sums, so FP64 and both mixed solves are bit-identical in either form (and
    with the x windows of the CSR groups on), with three and with two launches
    per iteration."""
    from paper_2510_08536_amd import RP_LOOP_THREE
    if name in FORM_CASES:
        w = FORM_CASES[name]()
        plan = make_plan(w)
        update(plan, share_values(w))
    else:
        w, m, val64, plan = _setup(name)
    b = dev_tensor(w.rhs())
    for prec in ("fp64", "mixed", "mixed_rr"):
        runs = []
        for coded, windows, fl in ((True, False, 0), (False, False, 0), (False, True, 0), (True, True, 0),
                                   (True, False, RP_LOOP_THREE), (False, False, RP_LOOP_THREE)):
            plan.set_spmv_format(coded)
            plan.set_spmv_windows(windows)
            x, info = plan.solve(b, precision=prec, fused_loop=fl)
            runs.append((x, info["iters"], info["outer_iters"]))
        for x, it, outer in runs[1:]:
            assert (it, outer) == runs[0][1:] and torch_mod().equal(x, runs[0][0]), (name, prec)
    plan.close()


def test_zero_rhs_and_warm_start():
    torch = torch_mod()
    w, m, val64, plan = _setup("stretched")
    b = w.rhs()
    x0 = dev_tensor(np.ones(m.n_rows))
    x, info = plan.solve(dev_tensor(np.zeros(m.n_rows)), x=x0)
    assert info["status"] == 0 and info["iters"] == 0 and (x.cpu().numpy() == 0).all()
    x_or, *_ = oracle.pcg(m, val64, b, tol=1e-12)
    x, info = plan.solve(dev_tensor(b), x=dev_tensor(x_or), tol=1e-8)
    assert info["status"] == 0 and info["iters"] == 0
    # warm start from a nearby x converges in fewer iterations than from zero
    x_cold, info_cold = plan.solve(dev_tensor(b), tol=1e-8)
    x_w, info_w = plan.solve(dev_tensor(b), x=dev_tensor(x_or * (1 + 1e-4)), tol=1e-8)
    assert info_w["iters"] < info_cold["iters"]
    for prec in ("fp64", "mixed", "mixed_rr"):
        x, info = plan.solve(torch.zeros(m.n_rows, dtype=torch.float64, device="cuda:0"), precision=prec)
        assert info["status"] == 0 and (x.cpu().numpy() == 0).all()
    plan.close()


def test_iteration_budget():
    from paper_2510_08536_amd import RP_NOT_CONVERGED
    w, m, val64, plan = _setup("c4fd")
    b = w.rhs()
    x, info = plan.solve(dev_tensor(b), tol=1e-8, max_iter=5, check=False)
    xo, st, it, *_ = oracle.pcg(m, val64, b, tol=1e-8, max_iter=5)
    assert info["status"] == RP_NOT_CONVERGED and st == 1 and info["iters"] == it == 5
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    plan.close()


def test_value_errors_reported():
    from paper_2510_08536_amd import RP_ERR_VALUE, RP_ERR_UNSUPPORTED, RpError
    w = CASES["ragged_rcb7"]()
    plan = make_plan(w)
    b = dev_tensor(w.rhs())
    vals = share_values(w)
    bad = [dict(v) for v in vals]
    bad[1] = dict(bad[1], upper=bad[1]["upper"].copy())
    bad[1]["upper"][3] = np.nan
    update(plan, bad)
    with pytest.raises(RpError) as e:
        plan.solve(b)
    assert e.value.code == RP_ERR_VALUE
    with pytest.raises(RpError) as e:
        plan.sync()
    assert e.value.code == RP_ERR_VALUE
    neg = [dict(v) for v in vals]
    neg[0] = dict(neg[0], diag=-neg[0]["diag"])
    update(plan, neg)
    with pytest.raises(RpError) as e:
        plan.solve(b)
    assert e.value.code == RP_ERR_VALUE
    # non-symmetric: lower differs from upper, and interface partners differ
    rng = np.random.default_rng(0)
    update(plan, random_ldu_values(w, rng), lower=True)
    with pytest.raises(RpError) as e:
        plan.solve(b)
    assert e.value.code == RP_ERR_UNSUPPORTED
    asym = [dict(v) for v in vals]
    asym[2] = dict(asym[2], iface=asym[2]["iface"] * 1.5)
    update(plan, asym)
    with pytest.raises(RpError) as e:
        plan.solve(b)
    assert e.value.code == RP_ERR_UNSUPPORTED
    # a good update clears the errors
    update(plan, vals)
    x, info = plan.solve(b)
    assert info["status"] == 0
    plan.close()


def test_nonlocal_share_not_solvable():
    from paper_2510_08536_amd import RP_ERR_UNSUPPORTED, RpError
    w = CASES["ragged_rcb7"]()
    plan = make_plan(w, 1, 3)
    assert plan.nnz_nonlocal > 0
    update(plan, share_values(w, None, 1, 3))
    with pytest.raises(RpError) as e:
        plan.solve(dev_tensor(np.ones(plan.n_rows)))
    assert e.value.code == RP_ERR_UNSUPPORTED
    plan.close()


def test_breakdown_on_indefinite_matrix():
    """diag 1, coupling -2: eigenvalues -1 and 3, so (p, A p) can be <= 0."""
    from paper_2510_08536_amd import Plan, RP_ERR_BREAKDOWN
    n = 2
    ranks = [dict(owner=np.array([0], np.int32), neighbour=np.array([1], np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    plan = Plan([n], 0, 1, ranks)
    plan.update([np.array([1.0, 1.0])], [np.array([-2.0])], [np.zeros(0)])
    b = np.array([1.0, 1.0])   # eigenvector of eigenvalue -1: (p, A p) < 0 at once
    x, info = plan.solve(dev_tensor(b), check=False)
    m = oracle.merge([n], 0, 1, ranks)
    v64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=[1.0, 1.0], upper=[-2.0], iface=[])]))
    xo, st, *_ = oracle.pcg(m, v64, b)
    assert info["status"] == RP_ERR_BREAKDOWN and st == -6
    plan.close()


def test_kernel_timing_counts_iterations():
    from paper_2510_08536_amd import RP_KERNEL_SPMV64, RP_KERNEL_SPMV32, RP_KERNEL_SCATTER
    w, m, val64, plan = _setup("c1")
    plan.set_timing(True)
    update(plan, share_values(w))
    x, info = plan.solve(dev_tensor(w.rhs()), tol=1e-8, check_every=16)
    n, ms = plan.kernel_stats(RP_KERNEL_SPMV64)
    assert n == info["iters"] and ms > 0
    n, ms = plan.kernel_stats(RP_KERNEL_SCATTER)
    assert n == 1 and ms > 0
    x, info = plan.solve(dev_tensor(w.rhs()), tol=1e-8, precision="mixed")
    n32, _ = plan.kernel_stats(RP_KERNEL_SPMV32)
    assert n32 == info["iters"]
    plan.set_timing(False)
    plan.close()


@pytest.mark.parametrize("stride", [3, 8])
@pytest.mark.parametrize("check_every", [5, 32])
def test_kernel_timing_stride(stride, check_every):
    """Timing every stride-th launch: the launches 0, stride, 2 stride, ...
    of the solve that did work are recorded (those past the stop inside the
    last host chunk are not), and their mean matches timing every launch."""
    from paper_2510_08536_amd import RP_KERNEL_SPMV64, RpError
    w, m, val64, plan = _setup("c1")
    b = dev_tensor(w.rhs())
    plan.set_timing(1)
    x1, info1 = plan.solve(b, tol=1e-8, check_every=check_every)
    n1, ms1 = plan.kernel_stats(RP_KERNEL_SPMV64)
    assert n1 == info1["iters"]
    plan.set_timing(stride)
    x, info = plan.solve(b, tol=1e-8, check_every=check_every)
    n, ms = plan.kernel_stats(RP_KERNEL_SPMV64)
    assert info["iters"] == info1["iters"] and torch_mod().equal(x, x1)
    assert n == -(-info["iters"] // stride) and ms > 0, (n, info["iters"], stride)
    assert 0.5 < (ms / n) / (ms1 / n1) < 2.0
    plan.set_timing(False)
    with pytest.raises(RpError):
        plan.set_timing(-1)
    plan.close()


def test_update_and_solve_on_a_side_stream():
    """The library enqueues on the stream it is given (torch's current one by
    default): the same update and solve on a second stream give the same
    bits as on the default stream."""
    torch = torch_mod()
    w, m, val64, plan = _setup("c1")
    b = dev_tensor(w.rhs())
    x0, i0 = plan.solve(b, tol=1e-8)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        update(plan, share_values(w))
        x1, i1 = plan.solve(b, tol=1e-8)
        x2, i2 = plan.solve(b, tol=1e-8, method="bicgstab")
    side.synchronize()
    assert i0["iters"] == i1["iters"] and torch.equal(x0, x1)
    assert i2["status"] == 0 and oracle.true_relres(m, val64, w.rhs(), x2.cpu().numpy()) <= 1e-8
    plan.close()
