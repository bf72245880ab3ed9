"""Adjoint on the GPU: RepartSolve (torch.autograd.Function) against the
oracle's adjoint and finite differences.

The face-coefficient -> slot-value assembly below is the caller's own code in
plain torch (the part a CFD application owns); the library differentiates the
solve: lambda = A^-1 dL/dx, dL/db = lambda, dL/dv_k = -lambda_row x_col."""
import numpy as np
import pytest

import oracle
import synth
from helpers import share_values, oracle_system, merged_row_of_natural
from gpu_util import torch_mod, dev_tensor, make_plan

pytestmark = pytest.mark.gpu


class Assembly:
    """slot values of the whole-mesh share as a differentiable function of the
    face coefficients c (global face order)."""

    def __init__(self, w, plan):
        torch = torch_mod()
        p = w.part
        n_slots = plan.n_slots
        src = np.full(n_slots, -1, np.int64)
        diag_slot = np.zeros(w.n_cells, np.int64)
        for r in range(w.n_ranks):
            k0 = int(plan.slot_off[r])
            nc = int(p.n_cells[r])
            f0, f1 = p.face_ptr[r], p.face_ptr[r + 1]
            i0, i1 = p.if_ptr[r], p.if_ptr[r + 1]
            nf = f1 - f0
            diag_slot[p.cell_ptr[r]:p.cell_ptr[r + 1]] = np.arange(k0, k0 + nc)
            src[k0 + nc:k0 + nc + nf] = p.face_gid[f0:f1]
            src[k0 + nc + nf:k0 + nc + 2 * nf] = p.face_gid[f0:f1]
            src[k0 + nc + 2 * nf:k0 + nc + 2 * nf + (i1 - i0)] = p.if_gid[i0:i1]
        off = np.nonzero(src >= 0)[0]
        pi = merged_row_of_natural(w)
        fa, fb = w.mesh.face_a, w.mesh.face_b
        inc_row = np.concatenate([pi[fa], pi[fb[fb >= 0]]])
        inc_face = np.concatenate([np.arange(w.mesh.n_faces), np.nonzero(fb >= 0)[0]])
        d = lambda a: torch.as_tensor(a, device="cuda:0")
        self.off_slots, self.off_src = d(off), d(src[off])
        self.diag_slots = d(diag_slot)       # merged row -> its diag slot
        self.inc_row, self.inc_face = d(inc_row), d(inc_face)
        self.n_slots, self.n = n_slots, w.n_cells

    def __call__(self, c):
        torch = torch_mod()
        diag = torch.zeros(self.n, dtype=c.dtype, device=c.device).index_add(0, self.inc_row, c[self.inc_face])
        v = torch.zeros(self.n_slots, dtype=c.dtype, device=c.device)
        v = v.index_put((self.off_slots,), -c[self.off_src])
        v = v.index_put((self.diag_slots,), diag)
        return v


def _oracle_adjoint(w, tol=1e-13):
    m, buf, val64, *_ = oracle_system(w)
    b, xt = w.rhs(), w.target()
    x, st, *_ = oracle.pcg(m, val64, b, tol=tol)
    lam, st2, *_ = oracle.pcg(m, val64, x - xt, tol=tol)
    assert st == 0 and st2 == 0
    pi = merged_row_of_natural(w)
    fb = w.mesh.face_b
    gface = oracle.face_grad(pi[w.mesh.face_a], np.where(fb >= 0, pi[np.maximum(fb, 0)], -1), lam, x)
    return m, val64, x, lam, gface


@pytest.mark.parametrize("precision,tol,bound", [("fp64", 1e-12, 1e-6), ("mixed", 1e-10, 1e-5)])
def test_autograd_matches_oracle_adjoint(precision, tol, bound):
    torch = torch_mod()
    from paper_2510_08536_amd import default_opts
    from paper_2510_08536_amd.autograd import repart_solve
    w = synth.build("c4fd")
    m, val64, x_or, lam_or, g_or = _oracle_adjoint(w)
    plan = make_plan(w)
    asm = Assembly(w, plan)
    c = dev_tensor(w.coefficients()).requires_grad_(True)
    b = dev_tensor(w.rhs()).requires_grad_(True)
    xt = dev_tensor(w.target())
    v = asm(c)
    # the torch assembly reproduces the generator's values (up to summation order of the diagonal)
    assert torch.allclose(v.detach(), dev_tensor(oracle.receive_buffer(share_values(w))), rtol=1e-14, atol=0)
    x = repart_solve(v, b, plan, default_opts(tol=tol, precision=precision))
    L = 0.5 * torch.sum((x - xt) ** 2)
    L.backward()
    gc, gb = c.grad.cpu().numpy(), b.grad.cpu().numpy()
    assert np.max(np.abs(gb - lam_or)) <= bound * max(1.0, np.max(np.abs(lam_or)))
    assert np.max(np.abs(gc - g_or) / np.maximum(1.0, np.abs(g_or))) <= bound
    plan.close()


def test_gradient_finite_difference_on_gpu():
    """Central differences of L(c) through GPU solves (h = 1e-6, FP64)."""
    torch = torch_mod()
    from paper_2510_08536_amd import default_opts
    from paper_2510_08536_amd.autograd import repart_solve
    w = synth.build("c4fd")
    plan = make_plan(w)
    asm = Assembly(w, plan)
    b, xt = dev_tensor(w.rhs()), dev_tensor(w.target())
    opts = lambda: default_opts(tol=1e-13)
    c0 = dev_tensor(w.coefficients())
    c = c0.clone().requires_grad_(True)
    L = 0.5 * torch.sum((repart_solve(asm(c), b, plan, opts()) - xt) ** 2)
    L.backward()
    g = c.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    faces = np.concatenate([rng.choice(w.mesh.n_interior, 24, replace=False),
                            rng.choice(np.arange(w.mesh.n_interior, w.mesh.n_faces), 8, replace=False)])
    h = 1e-6
    with torch.no_grad():
        for f in faces:
            cp, cm = c0.clone(), c0.clone()
            cp[f] += h
            cm[f] -= h
            Lp = 0.5 * torch.sum((repart_solve(asm(cp), b, plan, opts()) - xt) ** 2).item()
            Lm = 0.5 * torch.sum((repart_solve(asm(cm), b, plan, opts()) - xt) ** 2).item()
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[f]) <= 1e-5 * max(1.0, abs(g[f])), (f, fd, g[f])
    plan.close()


def test_backward_after_other_update_uses_saved_values():
    torch = torch_mod()
    from paper_2510_08536_amd import default_opts
    from paper_2510_08536_amd.autograd import repart_solve
    w = synth.build("c4fd", timesteps=2)
    m, val64, x_or, lam_or, g_or = _oracle_adjoint(w)
    plan = make_plan(w)
    asm = Assembly(w, plan)
    c = dev_tensor(w.coefficients()).requires_grad_(True)
    b, xt = dev_tensor(w.rhs()), dev_tensor(w.target())
    x = repart_solve(asm(c), b, plan, default_opts(tol=1e-12))
    # another timestep's values go into the plan before backward runs
    plan.update_slots(dev_tensor(oracle.receive_buffer(share_values(w, t=1))))
    L = 0.5 * torch.sum((x - xt) ** 2)
    L.backward()
    gc = c.grad.cpu().numpy()
    assert np.max(np.abs(gc - g_or) / np.maximum(1.0, np.abs(g_or))) <= 1e-6
    plan.close()


def test_autograd_keeps_caller_opts():
    """The Function works on a copy of the caller's options."""
    torch = torch_mod()
    from paper_2510_08536_amd import default_opts
    from paper_2510_08536_amd.autograd import repart_solve
    w = synth.small((6, 5, 4), ("blocks", 2, 1, 1), kappa=(1e-2, 1.0), seed=77)
    plan = make_plan(w)
    asm = Assembly(w, plan)
    c = torch.as_tensor(w.coefficients(), device="cuda:0").requires_grad_(True)
    b = dev_tensor(w.rhs())
    o = default_opts(tol=1e-10)
    assert o.x0_zero == 0 and o.transpose == 0
    x = repart_solve(asm(c), b, plan, o)
    (0.5 * (x * x).sum()).backward()
    assert o.x0_zero == 0 and o.transpose == 0 and c.grad is not None and torch.isfinite(c.grad).all()
    plan.close()


def test_autograd_nonsymmetric_bicgstab_finite_difference():
    """Non-symmetric (momentum-type) slot values through BiCGStab: the
    backward solves A^T lambda = x - x_t.  Central differences along random
    slot directions (FP64, h = 1e-6, solves to 1e-13) agree with <g, d>."""
    torch = torch_mod()
    from paper_2510_08536_amd import default_opts
    from paper_2510_08536_amd.autograd import repart_solve
    w = synth.small((7, 6, 5), ("rcb", 3), kappa=(1e-2, 1.0), seed=78)
    mv = share_values(w, values=w.momentum_values(pe=6.0))
    buf = oracle.receive_buffer(mv)
    plan = make_plan(w)
    o = default_opts(tol=1e-13, method="bicgstab")
    b, xt = dev_tensor(w.rhs()), dev_tensor(w.target())
    v = torch.as_tensor(buf, device="cuda:0").requires_grad_(True)
    x = repart_solve(v, b, plan, o)
    loss = 0.5 * ((x - xt) ** 2).sum()
    loss.backward()
    g = v.grad.detach()

    def L(vals):
        with torch.no_grad():
            xx = repart_solve(vals, b, plan, o)
            return 0.5 * ((xx - xt) ** 2).sum().item()

    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(4):
        d = torch.as_tensor(rng.uniform(-1, 1, buf.shape[0]) * np.abs(buf), device="cuda:0")
        fd = (L(v.detach() + h * d) - L(v.detach() - h * d)) / (2 * h)
        ad = float((g * d).sum().item())
        assert abs(fd - ad) <= 1e-5 * max(1.0, abs(ad)), (fd, ad)
    # dL/db against the oracle's transposed solve
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, [w.part.rank(r) for r in range(w.n_ranks)])
    val64, *_ = oracle.update(m, buf)
    import scipy.sparse as sp
    AT = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(m.n_rows, m.n_rows)).T.tocsr()
    AT.sort_indices()
    lam_or, st, *_ = oracle.bicgstab_csr(AT.indptr, AT.indices, AT.data, (x - xt).detach().cpu().numpy(), tol=1e-13)
    assert st == 0
    bb = b.clone().requires_grad_(True)
    x2 = repart_solve(v.detach(), bb, plan, o)
    (0.5 * ((x2 - xt) ** 2).sum()).backward()
    lam = bb.grad.cpu().numpy()
    assert np.linalg.norm(lam - lam_or) <= 1e-8 * np.linalg.norm(lam_or)
    plan.close()
