"""Block-Jacobi preconditioner on the GPU against the oracle.

The block inverses are built on the GPU from the fused values by the same
Gauss-Jordan steps as the oracle's, each operation one IEEE rounding in the
same order, so the packed inverses must match bit for bit (FP64, and the
FP32 copy is their RNE rounding).  Solves: FP64 PCG with the preconditioner
against the oracle's block-Jacobi PCG, true relative residual <= 1e-8 by the
oracle's SpMV, error <= 1e-6 against the oracle's x, iteration counts within
rounding, no restart; both mixed forms reach the same residual and error
bound against the oracle's FP64 solution."""
import numpy as np
import pytest

import oracle
import synth
from helpers import share_values, oracle_system
from gpu_util import dev_tensor, make_plan, update, assert_bits_equal, torch_mod

pytestmark = pytest.mark.gpu

CASES = {
    "c4fd": lambda: synth.build("c4fd"),
    "ragged_rcb7": lambda: synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True),
    "stretched": lambda: synth.small((12, 12, 20), ("rcb", 6), kappa=(1e-3, 1.0), seed=22, scramble=True,
                                     stretch=100.0),
    "blocks_odd": lambda: synth.small((15, 9, 7), ("blocks", 3, 1, 1), kappa=(1e-3, 1.0), seed=23),
    "box27": lambda: synth.small((10, 9, 8), ("blocks", 2, 1, 1), kappa=(1e-2, 1.0), seed=24, stencil=27),
}


def _setup(name):
    w = CASES[name]()
    m, buf, val64, val32, d64, d32 = oracle_system(w)
    plan = make_plan(w)
    update(plan, share_values(w))
    return w, m, val64, d64, plan


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("bs", [1, 2, 3, 4, 8])
def test_block_inverse_bit_exact(name, bs):
    w, m, val64, d64, plan = _setup(name)
    start_or = oracle.block_starts(w.part.n_cells, bs)
    minv_or = oracle.block_jacobi_inverse(m, val64, start_or, bs)
    start, m64, m32 = plan.block_jacobi(bs)
    assert np.array_equal(start, start_or)
    assert_bits_equal(m64, minv_or, f"{name} bs={bs} minv64")
    assert_bits_equal(m32, minv_or.astype(np.float32), f"{name} bs={bs} minv32")
    if bs == 1:
        assert_bits_equal(m64, d64, f"{name} bs=1 is 1/diag")
    plan.close()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("bs", [2, 4, 8])
def test_block_jacobi_pcg_matches_oracle(name, bs):
    w, m, val64, d64, plan = _setup(name)
    b = w.rhs()
    x_or, st, it_or, rs_or, _ = oracle.pcg_block_jacobi(m, val64, b, w.part.n_cells, bs, tol=1e-8)
    _, _, it_j, _, _ = oracle.pcg(m, val64, b, tol=1e-8)
    assert st == 0 and rs_or == 0
    x, info = plan.solve(dev_tensor(b), tol=1e-8, precond="block_jacobi", block_size=bs)
    xh = x.cpu().numpy()
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    print(f"{name} bs={bs}: {info['iters']} it (oracle {it_or}, Jacobi {it_j}), rel.res {rr:.2e}, err {err:.2e}")
    assert info["status"] == 0 and info["restarts"] == 0 and rr <= 1e-8, (info, rr)
    assert err <= 1e-6
    assert abs(info["iters"] - it_or) <= max(3, int(0.02 * it_or)), (info["iters"], it_or)
    plan.close()


@pytest.mark.parametrize("name", ["c4fd", "ragged_rcb7", "blocks_odd"])
@pytest.mark.parametrize("precision", ["mixed", "mixed_rr"])
def test_block_jacobi_mixed(name, precision):
    w, m, val64, d64, plan = _setup(name)
    b = w.rhs()
    x_or, st, *_ = oracle.pcg(m, val64, b, tol=1e-12)
    assert st == 0
    x, info = plan.solve(dev_tensor(b), tol=1e-8, precision=precision, precond="block_jacobi", block_size=4)
    xh = x.cpu().numpy()
    rr = oracle.true_relres(m, val64, b, xh)
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    assert info["status"] == 0 and rr <= 1e-8 and err <= 1e-6, (info, rr, err)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_block_jacobi_graph_replay_bit_identical(precision):
    torch = torch_mod()
    w, m, val64, d64, plan = _setup("ragged_rcb7")
    b = dev_tensor(w.rhs())
    kw = dict(tol=1e-8, precision=precision, precond="block_jacobi", block_size=4, check_every=8)
    xe, ie = plan.solve(b, **kw)
    for rep in range(3):
        xg, ig = plan.solve(b, graph=1, **kw)
        assert ig["iters"] == ie["iters"] and torch.equal(xg, xe), rep
        xe2, _ = plan.solve(b, **kw)
        assert torch.equal(xe2, xe)
    plan.close()


def test_block_jacobi_follows_updates():
    """The inverses are rebuilt after every update: solves after an update
    with other values match the oracle's for those values."""
    w = synth.build("c2", shape=(24, 20, 16), decomp=("blocks", 2, 2, 1), timesteps=3)
    plan = make_plan(w)
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, [w.part.rank(r) for r in range(w.n_ranks)])
    b = w.rhs()
    for t in range(3):
        vals = share_values(w, t)
        val64, *_ = oracle.update(m, oracle.receive_buffer(vals))
        update(plan, vals)
        x_or, st, it_or, _, _ = oracle.pcg_block_jacobi(m, val64, b, w.part.n_cells, 4, tol=1e-8)
        x, info = plan.solve(dev_tensor(b), tol=1e-8, precond="block_jacobi", block_size=4)
        xh = x.cpu().numpy()
        assert np.linalg.norm(xh - x_or) <= 1e-6 * np.linalg.norm(x_or), t
        start, m64, _ = plan.block_jacobi(4)
        assert_bits_equal(m64, oracle.block_jacobi_inverse(m, val64, start, 4), f"t={t} minv64")
    plan.close()


def test_block_jacobi_refusals():
    from paper_2510_08536_amd import Plan, RpError, RP_ERR_ARG, RP_ERR_UNSUPPORTED, RP_ERR_BREAKDOWN
    w, m, val64, d64, plan = _setup("ragged_rcb7")
    b = dev_tensor(w.rhs())
    for bs in (0, 9):
        with pytest.raises(RpError) as e:
            plan.solve(b, precond="block_jacobi", block_size=bs)
        assert e.value.code == RP_ERR_ARG
    with pytest.raises(RpError) as e:
        plan.solve(b, precond="block_jacobi", method="bicgstab")
    assert e.value.code == RP_ERR_UNSUPPORTED
    plan.set_solve_order("rcm")
    with pytest.raises(RpError) as e:
        plan.solve(b, precond="block_jacobi")
    assert e.value.code == RP_ERR_UNSUPPORTED
    plan.close()
    # an indefinite 2x2 block: diag 1, coupling -2
    ranks = [dict(owner=np.array([0], np.int32), neighbour=np.array([1], np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    plan = Plan([2], 0, 1, ranks)
    plan.update([np.array([1.0, 1.0])], [np.array([-2.0])], [np.zeros(0)])
    with pytest.raises(RpError) as e:
        plan.solve(dev_tensor(np.ones(2)), precond="block_jacobi", block_size=2)
    assert e.value.code == RP_ERR_BREAKDOWN
    plan.close()
