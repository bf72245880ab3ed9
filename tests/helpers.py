"""Shared test plumbing: carve a share of ranks out of a synthetic workload."""
from __future__ import annotations

import numpy as np


def share_ranks(w, first=0, alpha=None):
    alpha = w.n_ranks - first if alpha is None else alpha
    return [w.part.rank(r) for r in range(first, first + alpha)]


def share_values(w, t=None, first=0, alpha=None, values=None):
    alpha = w.n_ranks - first if alpha is None else alpha
    v = w.values(t) if values is None else values
    return [v.rank(w.part, r) for r in range(first, first + alpha)]


def merged_row_of_natural(w):
    """merged row (whole-mesh share) of every natural cell id"""
    p = w.part
    return p.cell_ptr[p.cell_rank].astype(np.int64) + p.cell_local.astype(np.int64)


def oracle_system(w, t=None, first=0, alpha=None):
    import oracle
    alpha = w.n_ranks - first if alpha is None else alpha
    m = oracle.merge(w.part.n_cells, first, alpha, share_ranks(w, first, alpha))
    buf = oracle.receive_buffer(share_values(w, t, first, alpha))
    val64, val32, d64, d32 = oracle.update(m, buf)
    return m, buf, val64, val32, d64, d32


def random_ldu_values(w, rng, symmetric=False):
    """Arbitrary per-rank values (not an M-matrix) to expose placement errors."""
    out = []
    for r in range(w.n_ranks):
        d = w.part.rank(r)
        nf, ni = len(d["owner"]), len(d["iface_cell"])
        up = rng.uniform(-1, 1, nf)
        out.append(dict(diag=rng.uniform(1, 2, d["n_cells"]), upper=up,
                        lower=up if symmetric else rng.uniform(-1, 1, nf),
                        iface=rng.uniform(-1, 1, ni)))
    return out


def golden_reference(name):
    """The oracle's reference solution of a full-size pressure system
    (tests/golden/ref_<name>.json, written by make_full_size_refs.py): the
    record, the sampled rows and x_ref on them."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"ref_{name}.json")
    with open(path) as f:
        d = json.load(f)
    rows = np.asarray(d["rows"], dtype=np.int64)
    x_ref = np.asarray([float(v) for v in d["x_ref"]], dtype=np.float64)
    return d, rows, x_ref


def sampled_rel_err(x, rows, x_ref):
    """||x - x_ref|| / ||x_ref|| over the sampled rows."""
    return float(np.linalg.norm(np.asarray(x)[rows] - x_ref) / np.linalg.norm(x_ref))
