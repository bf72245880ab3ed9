"""Rows with far more couplings than a 7-point stencil.

A 27-point mesh (every cell coupled to its 26 neighbours, as polyhedral
finite-volume cells can be) gives 27 entries per interior row, so every
256-row group holds about 3,000 value pairs: more than the 1,024 pairs the
SpMV stages in LDS, and more than 16 distinct column offsets, so every group
is read as CSR through the unstaged per-thread loop.  The SpMV must still be
bit-exact against the oracle's serial definition (FP64), within the FP32
rounding bound (FP32), and every solve within the solve tolerances of
test_gpu_solve (true relative residual <= 1e-8, error <= 1e-6 against the
oracle's x, no restart)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import share_values, oracle_system
from gpu_util import dev_tensor, make_plan, update, assert_bits_equal

pytestmark = pytest.mark.gpu

CASES = {
    "box27_blocks": lambda: synth.small((14, 12, 10), ("blocks", 2, 2, 1), kappa=(1e-2, 1.0), seed=31, stencil=27),
    "box27_rcb": lambda: synth.small((13, 11, 9), ("rcb", 5), kappa=(1e-3, 1.0), seed=32, stencil=27,
                                     scramble=True),
}


def _setup(name):
    w = CASES[name]()
    m, buf, val64, val32, *_ = oracle_system(w)
    assert (np.diff(m.row_ptr) > 8).mean() > 0.5
    groups = [(m.row_ptr[min(g + 256, m.n_rows)] - m.row_ptr[g]) // 2 for g in range(0, m.n_rows, 256)]
    assert max(groups) > 1024, groups
    plan = make_plan(w)
    update(plan, share_values(w))
    return w, m, val64, val32, plan


@pytest.mark.parametrize("name", sorted(CASES))
def test_wide_rows_spmv(name):
    w, m, val64, val32, plan = _setup(name)
    f = plan.spmv_format()
    assert f["coded_groups"] == 0, f
    rng = np.random.default_rng(5)
    for trial in range(3):
        x = rng.uniform(-1, 1, m.n_rows)
        assert_bits_equal(plan.spmv(dev_tensor(x)).cpu().numpy(), oracle.spmv(m, val64, x), f"{name} spmv64")
    x32 = rng.uniform(-1, 1, m.n_rows).astype(np.float32)
    y = plan.spmv(dev_tensor(x32)).cpu().numpy().astype(np.float64)
    exact = oracle.spmv(m, val32.astype(np.float64), x32.astype(np.float64))
    absrow = oracle.spmv(m, np.abs(val32.astype(np.float64)), np.abs(x32.astype(np.float64)))
    k = np.diff(m.row_ptr).astype(np.float64)
    u = 2.0 ** -24
    assert (np.abs(y - exact) <= (k + 1) * u / (1 - (k + 1) * u) * absrow).all()
    plan.close()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_rr"])
def test_wide_rows_solve(name, precision):
    w, m, val64, val32, plan = _setup(name)
    b = w.rhs()
    x_or, st, it_or, rs_or, _ = oracle.pcg(m, val64, b, tol=1e-8)
    assert st == 0 and rs_or == 0
    x, info = plan.solve(dev_tensor(b), tol=1e-8, precision=precision)
    xh = x.cpu().numpy()
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    assert info["status"] == 0 and info["restarts"] == 0 and rr <= 1e-8, (info, rr)
    assert err <= 1e-6, err
    if precision == "fp64":
        assert abs(info["iters"] - it_or) <= max(3, int(0.02 * it_or)), (info["iters"], it_or)
    plan.close()


@pytest.mark.parametrize("name", sorted(CASES))
def test_wide_rows_bicgstab(name):
    """Non-symmetric values on the wide rows: each upper / lower pair drawn
    apart, the diagonal the row's sum of off-diagonal magnitudes plus 1
    (strictly diagonally dominant), BiCGStab against the oracle's."""
    w = CASES[name]()
    rng = np.random.default_rng(8)
    vals = []
    for r in range(w.n_ranks):
        d = w.part.rank(r)
        nf, ni = len(d["owner"]), len(d["iface_cell"])
        vals.append(dict(upper=-rng.uniform(0.1, 1.0, nf), lower=-rng.uniform(0.1, 1.0, nf), iface=None,
                         diag=None, d=d))
    # interface entries: A(row, col) on each side, drawn per side
    for v in vals:
        v["iface"] = -rng.uniform(0.1, 1.0, len(v["d"]["iface_cell"]))
    for v in vals:
        d = v["d"]
        diag = np.ones(d["n_cells"])
        np.add.at(diag, d["owner"], np.abs(v["upper"]))
        np.add.at(diag, d["neighbour"], np.abs(v["lower"]))
        np.add.at(diag, d["iface_cell"], np.abs(v["iface"]))
        v["diag"] = diag
        del v["d"]
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, [w.part.rank(r) for r in range(w.n_ranks)])
    val64, *_ = oracle.update(m, oracle.receive_buffer(vals))
    plan = make_plan(w)
    update(plan, vals, lower=True)
    b = w.rhs()
    x_or, st, it_or, rs_or, _ = oracle.bicgstab(m, val64, b, tol=1e-8)
    assert st == 0 and rs_or == 0
    x, info = plan.solve(dev_tensor(b), tol=1e-8, method="bicgstab")
    xh = x.cpu().numpy()
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    assert info["status"] == 0 and info["restarts"] == 0 and rr <= 1e-8 and err <= 1e-6, (info, rr, err)
    plan.close()
