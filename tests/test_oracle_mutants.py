"""Pin strength: plausible mistakes planted in a copy of the oracle source must
each make at least one pin fail.  Runs on the CPU only; the committed oracle
is never modified."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle.oracle as oracle_mod
import test_oracle_amg as amg_pins
import test_oracle_pins as pins

MUTANTS = {
    # merge: upper and lower slots placed at each other's positions
    "upper_lower_swapped": ("slot_row[k] = (int32_t)(row0 + o);\n            slot_col[k] = off[r] + b;",
                            "slot_row[k] = (int32_t)(row0 + b);\n            slot_col[k] = off[r] + o;"),
    # merge: interface column taken in the wrong rank's numbering
    "iface_wrong_rank_offset": ("slot_col[k] = off[q] + d;", "slot_col[k] = off[r] + d;"),
    # merge: rows sorted descending
    "row_sort_descending": ("slot_col[at[base + m - 1]] > cg", "slot_col[at[base + m - 1]] < cg"),
    # merge: off-by-one in the localisation range
    "localise_off_by_one": (">= lo && ", "> lo && "),
    # update: inverse permutation applied instead of P
    "perm_inverted": ("val64[perm[k]] = buf[k];", "val64[k] = buf[perm[k]];"),
    # update: Jacobi diagonal read from the wrong slot
    "dinv_wrong_slot": ("dinv64[i] = 1.0 / buf[diag_slot[i]];", "dinv64[i] = 1.0 / buf[i];"),
    # CG: residual update sign
    "cg_residual_sign": ("r[i] -= a * q[i];", "r[i] += a * q[i];"),
    # CG: beta term dropped (steepest descent)
    "cg_no_beta": ("p[i] = z[i] + beta * p[i];", "p[i] = z[i];"),
    # CG: preconditioner left out of the recurrence (kept in the start-up)
    "cg_precond_only_at_start": ("z[i] = r[i] / diag[i];\n            const double rz_new",
                                 "z[i] = r[i];\n            const double rz_new"),
    # CG: preconditioner left out everywhere
    "cg_no_precond": ("z[i] = r[i] / diag[i];", "z[i] = r[i];"),
    # BiCGStab: the omega v correction left out of the direction update
    "bicg_p_no_omega_v": ("p[i] = r[i] + beta * (p[i] - omega * v[i]);", "p[i] = r[i] + beta * p[i];"),
    # BiCGStab: intermediate residual with the wrong sign
    "bicg_s_sign": ("s[i] = r[i] - alpha * v[i];", "s[i] = r[i] + alpha * v[i];"),
    # BiCGStab: preconditioner left out of the stabilising half step
    "bicg_z_no_precond": ("z[i] = s[i] / diag[i];", "z[i] = s[i];"),
    # BiCGStab: shadow residual replaced by the current residual
    "bicg_rho_uses_r": ("const double rho = dot(n, rh, r);", "const double rho = dot(n, r, r);"),
    # BiCGStab: omega step missing from the solution update
    "bicg_x_no_omega": ("x[i] = (x[i] + alpha * y[i]) + omega * z[i];", "x[i] = x[i] + alpha * y[i];"),
    # adjoint: row and column exchanged
    "grad_transposed": ("-lambda[slot_row[k]] * x[c]", "-lambda[c] * x[slot_row[k]]"),
    # adjoint: interface face gradient sign of the partner term
    "face_grad_sign": ("-(lambda[a] - lambda[b]) * (x[a] - x[b])", "-(lambda[a] + lambda[b]) * (x[a] - x[b])"),
    # block-Jacobi: only the rows below the pivot eliminated (no back elimination)
    "bj_no_back_elimination": ("if (i == k) continue;\n                const double f = W[i][k];",
                               "if (i <= k) continue;\n                const double f = W[i][k];"),
    # block-Jacobi: packed store without the triangle offset
    "bj_packed_index": ("out[i * bs - i * (i - 1) / 2 + (j - i)] = Z[i][j];", "out[i * bs + (j - i)] = Z[i][j];"),
    # block-Jacobi: apply reads the row's entry for j < i from the wrong triangle
    "bj_apply_wrong_triangle": ("const int a = i < j ? i : j, c = i < j ? j : i;", "const int a = i, c = j;"),
    # block-Jacobi: blocks numbered from each rank's start instead of the share's
    "bj_starts_rank_local": ("if (start) start[nb] = (int32_t)(row + c);", "if (start) start[nb] = (int32_t)c;"),
    # AMG: the weakest coupling taken for the strongest
    "amg_weakest_coupling": ("if (a->w != b->w) return a->w > b->w;", "if (a->w != b->w) return a->w < b->w;"),
    # AMG: unmatched rows never join a pair
    "amg_no_joining": ("leader[i] = j >= 0 ? (j < mate[j] ? (int32_t)j : mate[j]) : (int32_t)i;",
                       "leader[i] = (int32_t)i;"),
    # AMG: Galerkin sum keeps only the first contribution of each coarse entry
    "amg_galerkin_first_only": ("for (int64_t t = L->cptr[e]; t < L->cptr[e + 1]; ++t) s += L->val[L->cpos[t]];",
                                "s = L->val[L->cpos[L->cptr[e]]];"),
    # AMG: restriction of the smoothed level takes r instead of the residual t
    "amg_restrict_r_not_t": ("for (int64_t m = L->mem_ptr[I]; m < L->mem_ptr[I + 1]; ++m) s += t[L->mem[m]];",
                             "for (int64_t m = L->mem_ptr[I]; m < L->mem_ptr[I + 1]; ++m) s += r[L->mem[m]];"),
    # AMG: post-smoothing without the damping factor
    "amg_post_no_omega": ("y[i] = x[i] + h->omega * (L->dinv[i] * (r[i] - t[i]));",
                          "y[i] = x[i] + (L->dinv[i] * (r[i] - t[i]));"),
    # AMG: every level smoothed (the odd levels too)
    "amg_all_levels_smoothed": ("if (l % 2 == 1) {", "if (l % 2 == 2) {"),
    # AMG: prolongation adds the coarse correction of the wrong row
    "amg_prolong_wrong_row": ("x[i] = x[i] + ec[L->agg[i]];", "x[i] = x[i] + ec[L->agg[n - 1 - i]];"),
    # AMG: coarsest inverse without back elimination
    "amg_inverse_no_back": ("if (i == k) continue;\n            const double f = W[i * n + k];",
                            "if (i <= k) continue;\n            const double f = W[i * n + k];"),
}

PIN_CALLS = [
    lambda: [pins.test_p1_global_assembly_identity(c) for c in range(len(pins.SMALL_CASES))],
    lambda: [pins.test_p2_brute_force_dense(c, s) for c in range(len(pins.SMALL_CASES)) for s in (False, True)],
    lambda: [pins.test_golden_alpha2_chain(w) for w in ("alpha2", "rank1_alone")],
    lambda: [pins.test_p4_symmetric_positive_definite(c) for c in range(len(pins.SMALL_CASES))],
    pins.test_p3_single_rank_is_plain_ldu_to_csr,
    pins.test_p5_sine_eigenvector_one_iteration,
    pins.test_p5_two_eigenvalues_two_iterations,
    lambda: [pins.test_p6_tridiagonal_inverse(n) for n in (1, 3)],
    lambda: [pins.test_p7_dense_lu(c) for c in range(1, len(pins.SMALL_CASES))],
    pins.test_p9_bicgstab_diagonal_one_iteration,
    pins.test_p9_bicgstab_two_eigenvalues_two_iterations,
    lambda: [pins.test_p9_bicgstab_dense_lu(c) for c in range(1, len(pins.SMALL_CASES))],
    pins.test_p8_slot_gradient_dense,
    pins.test_p8_adjoint_face_gradient_finite_difference,
    pins.test_p11_block_starts_hand_derived,
    lambda: [pins.test_p11_block_inverse_against_lapack(c, bs) for c in range(len(pins.SMALL_CASES))
             for bs in (2, 4)],
    lambda: [pins.test_p11_apply_is_the_block_diagonal_solve(c, 4) for c in range(len(pins.SMALL_CASES))],
    amg_pins.test_p12_chain4_pair_and_joiners,
    amg_pins.test_p12_chain6_two_pairs,
    lambda: [amg_pins.test_p12_galerkin_is_dense_ptap(nm) for nm in ("cube8_const", "box27")],
    lambda: [amg_pins.test_p12_vcycle_is_the_multigrid_product(nm, cm)
             for nm, cm in (("cube8_const", 256), ("box27", 100))],
]


RUNNER = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle.oracle as om
om.LIB = {lib!r}
om._lib = None
import test_oracle_mutants as tm
for call in tm.PIN_CALLS:
    try:
        call()
    except Exception as e:
        print("CAUGHT", type(e).__name__, str(e)[:200])
        sys.exit(0)
print("MISSED")
"""


def _compile(src_text, out_dir):
    src = os.path.join(out_dir, "mutant.c")
    lib = os.path.join(out_dir, "libmutant.so")
    open(src, "w").write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", lib, src, "-lm"])
    return lib


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    before, after = MUTANTS[name]
    text = open(oracle_mod.SRC).read()
    assert text.count(before) >= 1, name
    tests_dir = os.path.dirname(os.path.abspath(__file__))
    with tempfile.TemporaryDirectory() as d:
        lib = _compile(text.replace(before, after), d)
        code = RUNNER.format(root=os.path.dirname(tests_dir), tests=tests_dir, lib=lib)
        p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    # a pin failing, or the mutant crashing the process, both expose the mistake
    assert p.returncode != 0 or "CAUGHT" in p.stdout, f"no pin caught mutant {name}: {p.stdout[-500:]}"
