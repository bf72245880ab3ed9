"""GPU parity of the repartitioning (plan), the value update, the SpMV and the
value gradient against the oracle.  All of these are pure index work or
single roundings taken in the same order, so the bar is bit-exactness."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import share_ranks, share_values, oracle_system, random_ldu_values
from gpu_util import torch_mod, dev_tensor, make_plan, update, assert_bits_equal

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (shape, decomposition, kwargs): several row groups of 256 and ragged tails
CASES = {
    "chain8_4": ((8, 1, 1), ("blocks", 4, 1, 1), dict(walls=(True, False, False))),
    "cube4_8": ((4, 4, 4), ("blocks", 2, 2, 2), dict(kappa=(1e-2, 1.0))),
    "rcb_scrambled": ((5, 4, 3), ("rcb", 3), dict(kappa=(1e-3, 1.0), scramble=True)),
    "stretched_rcb": ((6, 5, 7), ("rcb", 5), dict(kappa=(1e-3, 1.0), scramble=True, stretch=100.0)),
    "ragged_rcb7": ((17, 13, 11), ("rcb", 7), dict(kappa=(1e-2, 1.0), scramble=True)),
    "slabs_c1like": ((32, 32, 32), ("blocks", 1, 1, 4), dict()),
    "one_cell_per_rank": ((9, 1, 1), ("blocks", 9, 1, 1), dict(walls=(True, False, False))),
    "single_rank": ((7, 6, 5), ("blocks", 1, 1, 1), dict(kappa=(1e-2, 1.0), scramble=True)),
    "two_pairs": ((80, 3, 5), ("blocks", 1, 1, 1), dict(kappa=(1e-2, 1.0))),
    "banded_ragged": ((20, 9, 31), ("blocks", 1, 2, 3), dict(kappa=(1e-2, 1.0))),
    # oblique cut planes: 10 of 38 row groups offset-coded, the rest CSR
    "rcb_mixed": ((40, 20, 12), ("rcb", 3), dict(kappa=(1e-2, 1.0))),
}


def _work(name, seed=0):
    shape, decomp, kw = CASES[name]
    kw = dict(kw)
    return synth.small(shape, decomp, kappa=kw.pop("kappa", None), seed=seed, **kw)


def _shares(w):
    out = [(0, w.n_ranks)]
    if w.n_ranks > 2:
        out.append((1, w.n_ranks - 2))   # strict subset: non-local block present
    return out


@pytest.mark.parametrize("name", sorted(CASES))
def test_plan_bit_exact(name):
    w = _work(name)
    for first, alpha in _shares(w):
        m = oracle.merge(w.part.n_cells, first, alpha, share_ranks(w, first, alpha))
        plan = make_plan(w, first, alpha)
        assert (plan.n_rows, plan.nnz, plan.nnz_nonlocal, plan.n_slots) == \
            (m.n_rows, m.nnz_local, m.nnz_nonlocal, m.n_slots)
        assert np.array_equal(plan.slot_off, m.slot_off)
        g = plan.get_csr()
        for k in ("row_ptr", "col", "perm", "nl_row_ptr", "nl_col"):
            want = getattr(m, k)
            assert np.array_equal(g[k], want), (name, first, alpha, k)
        plan.close()


@pytest.mark.parametrize("which", ["alpha2", "rank1_alone"])
def test_plan_golden_chain(which):
    from paper_2510_08536_amd import Plan
    gd = json.load(open(os.path.join(GOLDEN, "alpha2_chain.json")))
    exp = gd[which]
    first, alpha = exp["first"], exp["alpha"]
    ranks = [gd["ranks"][r] for r in range(first, first + alpha)]
    plan = Plan(gd["n_cells_all"], first, alpha, ranks)
    g = plan.get_csr()
    assert g["row_ptr"].tolist() == exp["row_ptr"] and g["col"].tolist() == exp["col"]
    assert g["perm"].tolist() == exp["perm"] and g["nl_col"].tolist() == exp["nl_col"]
    assert g["nl_row_ptr"].tolist() == exp["nl_row_ptr"]
    plan.update([np.array(r["diag"]) for r in ranks], [np.array(r["upper"]) for r in ranks],
                [np.array(r["iface"]) for r in ranks], lower=[np.array(r["lower"]) for r in ranks])
    v64, *_ = plan.get_values()
    assert v64.tolist() == exp["val"]
    plan.close()


def test_plan_with_empty_rank():
    """A rank owning no cells (and so no slots) inside the share."""
    from paper_2510_08536_amd import Plan
    gd = json.load(open(os.path.join(GOLDEN, "alpha2_chain.json")))
    ranks = [gd["ranks"][0], dict(owner=[], neighbour=[], iface_cell=[], iface_nbr_rank=[], iface_nbr_cell=[]),
             dict(gd["ranks"][1], iface_nbr_rank=[0])]
    n_cells_all = [2, 0, 2]
    ranks[0] = dict(ranks[0], iface_nbr_rank=[2])
    to_np = lambda r: {k: np.array(r[k], dtype=np.int32) for k in
                       ("owner", "neighbour", "iface_cell", "iface_nbr_rank", "iface_nbr_cell")}
    m = oracle.merge(n_cells_all, 0, 3, [to_np(r) for r in ranks])
    plan = Plan(n_cells_all, 0, 3, [to_np(r) for r in ranks])
    g = plan.get_csr()
    for k in ("row_ptr", "col", "perm"):
        assert np.array_equal(g[k], getattr(m, k)), k
    plan.close()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("where", ["device", "host"])
def test_update_bit_exact(name, where):
    w = _work(name, seed=3)
    rng = np.random.default_rng(11)
    for first, alpha in _shares(w):
        m = oracle.merge(w.part.n_cells, first, alpha, share_ranks(w, first, alpha))
        plan = make_plan(w, first, alpha)
        for step, vals in enumerate([share_values(w, None, first, alpha),
                                     random_ldu_values(w, rng)[first:first + alpha]]):
            lower = step == 1
            buf = oracle.receive_buffer(vals)
            want = oracle.update(m, buf)
            update(plan, vals, where=where, lower=lower)
            got = plan.get_values()
            for gv, wv, what in zip(got, want, ("val64", "val32", "dinv64", "dinv32")):
                assert_bits_equal(gv, wv, f"{name} {where} share({first},{alpha}) step {step} {what}")
        plan.close()


def test_update_slots_bit_exact():
    torch = torch_mod()
    w = _work("ragged_rcb7", seed=5)
    m, buf, *want = oracle_system(w)
    plan = make_plan(w)
    plan.update_slots(dev_tensor(buf))
    got = plan.get_values()
    for gv, wv, what in zip(got, want, ("val64", "val32", "dinv64", "dinv32")):
        assert_bits_equal(gv, wv, what)
    plan.close()
    del torch


def test_spmv_window_detection():
    """The plan finds the long-range stencil offset of blocked natural
    numbering (nx * ny of the rank block) and no windows for scrambled ids."""
    expect = {"slabs_c1like": (1, [1024]), "chain8_4": (0, [])}
    for name, want in expect.items():
        plan = make_plan(_work(name))
        assert plan.spmv_windows() == want, name
        plan.close()
    w = synth.small((30, 30, 30), ("rcb", 3), seed=2, scramble=True)   # random local order
    plan = make_plan(w)
    assert plan.spmv_windows() == (-1, [])
    plan.close()
    w = synth.small((20, 8, 12), ("blocks", 1, 1, 2), seed=1)    # nx = 20 <= 64, nx*ny = 160
    plan = make_plan(w)
    assert plan.spmv_windows() == (1, [160])
    plan.close()
    w = synth.small((80, 3, 4), ("blocks", 1, 1, 1), seed=1)     # nx = 80 > 64: two pairs,
    plan = make_plan(w)                                            # the more frequent first
    assert plan.spmv_windows() == (2, [240, 80])
    plan.close()


def _host_format(row_ptr, col, n):
    """The SpMV form rule restated on the host: a group of 256 rows is
    offset-coded iff its entries use at most 16 distinct col - row and its
    values span at most 1024 aligned pairs and 512 aligned quads."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ng = (n + 255) // 256
    out = dict(n_groups=ng, coded_groups=0, coded_rows=0, coded_nnz=0)
    for g in range(ng):
        r0, r1 = g * 256, min(n, g * 256 + 256)
        s, e = rp[r0], rp[r1]
        rows = np.repeat(np.arange(r0, r1), np.diff(rp[r0:r1 + 1]))
        k = np.unique(np.asarray(col[s:e], dtype=np.int64) - rows).size
        if 0 < k <= 16 and ((e - (s & ~1) + 1) >> 1) <= 1024 and ((e - (s & ~3) + 3) >> 2) <= 512:
            out["coded_groups"] += 1
            out["coded_rows"] += r1 - r0
            out["coded_nnz"] += int(e - s)
    return out


@pytest.mark.parametrize("name", sorted(CASES))
def test_spmv_format_coverage_and_bytes(name):
    """Which groups are offset-coded (integer work: exact), and the bytes
    reported for one y = A x in each form."""
    w = _work(name)
    for first, alpha in _shares(w):
        m = oracle.merge(w.part.n_cells, first, alpha, share_ranks(w, first, alpha))
        plan = make_plan(w, first, alpha)
        f = plan.spmv_format()
        want = _host_format(m.row_ptr, m.col, m.n_rows)
        assert f["enabled"] == 1
        assert {k: f[k] for k in want} == want, (name, first, alpha)
        n, nnz = m.n_rows, m.nnz_local
        cg, cr, cn = want["coded_groups"], want["coded_rows"], want["coded_nnz"]
        for key, sv in (("bytes64", 8), ("bytes32", 4)):
            coded = cn * sv + 2 * cr + 72 * cg + (nnz - cn) * (sv + 4) + 4 * (n - cr) + 2 * n * sv + 4
            assert f[key] == coded, (name, key)
        plan.set_spmv_format(False)
        f = plan.spmv_format()
        assert f["enabled"] == 0
        assert f["bytes64"] == 12 * nnz + 20 * n + 4 and f["bytes32"] == 8 * nnz + 12 * n + 4
        plan.close()


SPMV_MODES = ["coded", "csr", "csr_windows", "coded_windows"]


def _set_mode(plan, mode):
    plan.set_spmv_format(mode.startswith("coded"))
    plan.set_spmv_windows(mode.endswith("windows"))


@pytest.mark.parametrize("name", ["ragged_rcb7", "slabs_c1like", "stretched_rcb", "one_cell_per_rank",
                                  "single_rank", "chain8_4", "two_pairs", "banded_ragged", "rcb_mixed"])
@pytest.mark.parametrize("mode", SPMV_MODES)
def test_spmv_fp64_bit_exact(name, mode):
    w = _work(name, seed=7)
    m, buf, val64, val32, *_ = oracle_system(w)
    plan = make_plan(w)
    assert not plan.spmv_windows_enabled() and plan.spmv_format()["enabled"] == 1
    _set_mode(plan, mode)
    assert plan.spmv_windows_enabled() == (mode.endswith("windows") and plan.spmv_windows()[0] >= 0)
    update(plan, share_values(w))
    rng = np.random.default_rng(2)
    for x in (rng.uniform(-1, 1, m.n_rows), rng.standard_normal(m.n_rows) * 1e3, np.zeros(m.n_rows)):
        y = plan.spmv(dev_tensor(x)).cpu().numpy()
        assert_bits_equal(y, oracle.spmv(m, val64, x), f"{name} spmv64 {mode}")
    plan.close()


def test_spmv_fp32_same_bits_in_both_forms():
    """The FP32 SpMV forms every product and row sum in the same order in
    both index forms, so their results agree bit for bit."""
    torch = torch_mod()
    for name in ("slabs_c1like", "rcb_mixed", "banded_ragged"):
        w = _work(name, seed=9)
        m, *_ = oracle_system(w)
        plan = make_plan(w)
        update(plan, share_values(w))
        x32 = dev_tensor(np.random.default_rng(4).uniform(-1, 1, m.n_rows).astype(np.float32))
        ys = []
        for mode in SPMV_MODES:
            _set_mode(plan, mode)
            ys.append(plan.spmv(x32).cpu().numpy())
        for mode, y in zip(SPMV_MODES[1:], ys[1:]):
            assert_bits_equal(y, ys[0], f"{name} spmv32 {mode} vs coded")
        plan.close()
    del torch


@pytest.mark.parametrize("name", ["ragged_rcb7", "slabs_c1like", "two_pairs", "banded_ragged", "rcb_mixed"])
@pytest.mark.parametrize("mode", SPMV_MODES)
def test_spmv_fp32_error_bound(name, mode):
    """FP32 SpMV: each row sums k products with one rounding each, so
    |y32 - y| <= gamma_{k+1} * sum |a_ij x_j| with gamma_m = m u / (1 - m u),
    u = 2^-24, against the exact (FP64) product of the same FP32 inputs."""
    torch = torch_mod()
    w = _work(name, seed=9)
    m, buf, val64, val32, *_ = oracle_system(w)
    plan = make_plan(w)
    _set_mode(plan, mode)
    update(plan, share_values(w))
    x32 = np.random.default_rng(4).uniform(-1, 1, m.n_rows).astype(np.float32)
    y = plan.spmv(dev_tensor(x32)).cpu().numpy().astype(np.float64)
    exact = oracle.spmv(m, val32.astype(np.float64), x32.astype(np.float64))
    absrow = oracle.spmv(m, np.abs(val32.astype(np.float64)), np.abs(x32.astype(np.float64)))
    k = np.diff(m.row_ptr).astype(np.float64)
    u = 2.0 ** -24
    gamma = (k + 1) * u / (1 - (k + 1) * u)
    assert (np.abs(y - exact) <= gamma * absrow).all()
    plan.close()
    del torch


@pytest.mark.parametrize("name", ["ragged_rcb7", "stretched_rcb"])
def test_value_grad_bit_exact(name):
    w = _work(name, seed=13)
    m, buf, val64, *_ = oracle_system(w)
    plan = make_plan(w)
    rng = np.random.default_rng(8)
    lam, x = rng.uniform(-1, 1, m.n_rows), rng.uniform(-1, 1, m.n_rows)
    g = plan.value_grad(dev_tensor(lam), dev_tensor(x)).cpu().numpy()
    assert_bits_equal(g, oracle.value_grad(m, lam, x), name)
    plan.close()


# --------------------------------------------------------------------------
# error paths (forced from the host: invalid inputs the plan rejects)
# --------------------------------------------------------------------------
def _chain_ranks():
    gd = json.load(open(os.path.join(GOLDEN, "alpha2_chain.json")))
    return [{k: np.array(v, dtype=np.int32) for k, v in r.items()
             if k in ("owner", "neighbour", "iface_cell", "iface_nbr_rank", "iface_nbr_cell")} for r in gd["ranks"]]


@pytest.mark.parametrize("mutation,code", [
    ("self_face", -2), ("owner_range", -2), ("duplicate", -2), ("unpaired", -2),
    ("iface_rank_range", -2), ("iface_self_rank", -2), ("iface_cell_range", -2), ("bad_alpha", -1),
    ("ncells_mismatch", -1)])
def test_plan_rejects_bad_addressing(mutation, code):
    from paper_2510_08536_amd import Plan, RpError
    ranks = _chain_ranks()
    nca, first, alpha = [2, 2], 0, 2
    if mutation == "self_face":
        ranks[0]["neighbour"] = np.array([0], np.int32)
    elif mutation == "owner_range":
        ranks[1]["owner"] = np.array([2], np.int32)
    elif mutation == "duplicate":
        ranks[0]["owner"] = np.array([0, 1], np.int32)
        ranks[0]["neighbour"] = np.array([1, 0], np.int32)
    elif mutation == "unpaired":
        ranks[1]["iface_cell"] = np.array([1], np.int32)
    elif mutation == "iface_rank_range":
        ranks[0]["iface_nbr_rank"] = np.array([5], np.int32)
    elif mutation == "iface_self_rank":
        ranks[0]["iface_nbr_rank"] = np.array([0], np.int32)
    elif mutation == "iface_cell_range":
        ranks[0]["iface_nbr_cell"] = np.array([7], np.int32)
    elif mutation == "bad_alpha":
        alpha = 3
        ranks.append(ranks[0])
    elif mutation == "ncells_mismatch":
        ranks[0]["n_cells"] = 3
    with pytest.raises(RpError) as e:
        Plan(nca, first, alpha, ranks)
    assert e.value.code == code


class _DevArray:
    """A device array the library owns, seen by torch without a copy."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 3}


@pytest.mark.parametrize("name", ["slabs_c1like", "rcb_mixed", "ragged_rcb7"])
def test_device_ptrs(name):
    """rp_plan_device_ptrs: the device arrays hold what rp_plan_get_csr and
    rp_plan_get_values return (pattern, P, values in CSR order, Jacobi
    inverses), in either SpMV form."""
    torch = torch_mod()
    w = _work(name)
    m, buf, val64, val32, d64, d32 = oracle_system(w)
    plan = make_plan(w)
    update(plan, share_values(w))
    dev = lambda ptr, n, t: torch.as_tensor(_DevArray(ptr, n, t), device="cuda").cpu().numpy()
    for coded in (True, False):
        plan.set_spmv_format(coded)
        ptrs = plan.device_ptrs()
        assert np.array_equal(dev(ptrs["row_ptr"], m.n_rows + 1, "<i4"), m.row_ptr)
        assert np.array_equal(dev(ptrs["col"], m.nnz_local, "<i4"), m.col)
        assert np.array_equal(dev(ptrs["perm"], m.n_slots, "<i4"), m.perm)
        assert_bits_equal(dev(ptrs["val64"], plan.n_slots, "<f8"), val64, f"{name} device val64")
        assert_bits_equal(dev(ptrs["val32"], plan.n_slots, "<f4"), val32, f"{name} device val32")
        assert_bits_equal(dev(ptrs["dinv64"], m.n_rows, "<f8"), d64, f"{name} device dinv64")
        assert_bits_equal(dev(ptrs["dinv32"], m.n_rows, "<f4"), d32, f"{name} device dinv32")
    plan.close()
