"""Rank processes hand their values to the GPU owner (Sec. 3 update
procedure): through the owner's device receive buffer mapped by IPC (the
GPU-aware path), and through a receive buffer in shared host memory (the
host-buffer path).  Either way the fused values must equal the oracle's
update bit for bit (val64, val32, dinv64, dinv32), for symmetric and
non-symmetric values, over several timesteps with the workers' values
changing between them."""
import numpy as np
import pytest

import oracle
import synth
from helpers import share_ranks, share_values
from gpu_util import make_plan, assert_bits_equal

pytestmark = pytest.mark.gpu


def _layout(plan, w):
    return [(int(plan.slot_off[r]), int(w.part.n_cells[r]), len(w.part.rank(r)["owner"]),
             len(w.part.rank(r)["iface_cell"])) for r in range(w.n_ranks)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("lower", [False, True])
def test_rank_processes_both_paths_bit_exact(lower):
    from paper_2510_08536_amd.ranks import RankPool
    w = synth.small((17, 13, 11), ("rcb", 7), kappa=(1e-2, 1.0), seed=21, scramble=True, timesteps=3)
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, share_ranks(w))
    plan = make_plan(w)
    pool = RankPool(3, _layout(plan, w))
    try:
        bufs, want = [], []
        for t in range(3):
            vals = share_values(w, values=w.momentum_values(t)) if lower else share_values(w, t)
            buf = oracle.receive_buffer(vals)
            bufs.append(buf)
            want.append(oracle.update(m, buf))
        pool.load(bufs)
        pool.attach_device(plan.export_recv())
        host = pool.host_buffer(plan.n_slots)
        for t in range(3):
            pool.write_device(t)
            plan.update_from_recv()
            got = plan.get_values()
            for g, wv, what in zip(got, want[t], ("val64", "val32", "dinv64", "dinv32")):
                assert_bits_equal(g, wv, f"device path t={t} {what}")
            pool.write_host(t)
            so = plan.slot_off
            views = [host[so[r]:so[r + 1]] for r in range(w.n_ranks)]
            lay = _layout(plan, w)
            d = [v[:nc] for v, (_, nc, nf, ni) in zip(views, lay)]
            u = [v[nc:nc + nf] for v, (_, nc, nf, ni) in zip(views, lay)]
            lo = [v[nc + nf:nc + 2 * nf] for v, (_, nc, nf, ni) in zip(views, lay)]
            i = [v[nc + 2 * nf:] for v, (_, nc, nf, ni) in zip(views, lay)]
            plan.update(d, u, i, lower=lo)
            got = plan.get_values()
            for g, wv, what in zip(got, want[t], ("val64", "val32", "dinv64", "dinv32")):
                assert_bits_equal(g, wv, f"host path t={t} {what}")
    finally:
        pool.close()
        plan.close()
