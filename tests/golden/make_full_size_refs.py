"""Write the oracle reference solutions of the full-size pressure systems.

Run from the repository root:  python tests/golden/make_full_size_refs.py c3 c5

For each named workload this solves the pressure system A x = b (the
unperturbed coefficients for c3, timestep 0 for c5) with the serial oracle
PCG, first to a relative residual of 1e-8 from x = 0 (the tolerance the GPU
solves use) and then on to 1e-12 from that x.  It stores, as text:

  - the oracle's iteration counts, restarts and true relative residuals;
  - ||x_ref||_2 of the 1e-12 solution and the relative 2-norm error of the
    oracle's own 1e-8 solution against it (full vector and on the samples);
  - x_ref at a seeded sample of rows (exact decimal repr of each double).

The GPU tests and the benchmark compare their answers with x_ref on those
rows.  Only the oracle and the seeded input generators are called here.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

N_SAMPLES = 8192
# the system each reference is for: timestep None = the unperturbed kappa_0
SYSTEMS = {"c3": None, "c5": 0}


def sample_rows(name: str, n: int) -> np.ndarray:
    seed = int.from_bytes(name.encode(), "little")
    rng = np.random.default_rng(np.random.SeedSequence([seed, 20251008536]))
    return np.sort(rng.choice(n, size=min(N_SAMPLES, n), replace=False)).astype(np.int64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(name: str) -> dict:
    t = SYSTEMS[name]
    w = synth.build(name)
    ranks = [w.part.rank(r) for r in range(w.n_ranks)]
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, ranks)
    vals = [w.values(t).rank(w.part, r) for r in range(w.n_ranks)]
    val64, *_ = oracle.update(m, oracle.receive_buffer(vals))
    del vals
    b = w.rhs()
    t0 = time.perf_counter()
    x8, st8, it8, rs8, rr8 = oracle.pcg(m, val64, b, tol=1e-8)
    s8 = time.perf_counter() - t0
    print(f"{name}: oracle 1e-8: status {st8}, {it8} iterations, {rs8} restarts, rel.res {rr8:.3e}, {s8:.1f} s",
          flush=True)
    t0 = time.perf_counter()
    xr, str_, itr, rsr, rrr = oracle.pcg(m, val64, b, x0=x8, tol=1e-12)
    sr = time.perf_counter() - t0
    print(f"{name}: oracle 1e-12 (from the 1e-8 x): status {str_}, {itr} iterations, {rsr} restarts, "
          f"rel.res {rrr:.3e}, {sr:.1f} s", flush=True)
    rows = sample_rows(name, m.n_rows)
    out = {
        "workload": name,
        "timestep": t,
        "n_rows": int(m.n_rows),
        "nnz": int(m.nnz_local),
        "oracle_1e-8": {"status": st8, "iters": it8, "restarts": rs8, "rel_res": rr8,
                        "serial_seconds": round(s8, 1),
                        "rel_err_vs_ref": rel(x8, xr), "rel_err_vs_ref_sampled": rel(x8[rows], xr[rows])},
        "reference": {"tol": 1e-12, "status": str_, "iters_after_1e-8": itr, "restarts": rsr, "rel_res": rrr,
                      "norm2": float(np.linalg.norm(xr)), "norm_inf": float(np.abs(xr).max())},
        "rows": rows.tolist(),
        "x_ref": [repr(float(v)) for v in xr[rows]],
    }
    print(f"{name}: oracle 1e-8 error vs reference {out['oracle_1e-8']['rel_err_vs_ref']:.3e} "
          f"(sampled {out['oracle_1e-8']['rel_err_vs_ref_sampled']:.3e})", flush=True)
    return out


def main(names):
    for name in names:
        out = make(name)
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"ref_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
            f.write("\n")
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or sorted(SYSTEMS))
