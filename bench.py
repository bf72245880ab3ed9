"""Benchmark of the repartitioned pressure solve on one MI355X.

Workload (default "c3"): a 256^3 7-point finite-volume system split over 64
CPU ranks (4x4x4 blocks of 64^3 cells, log-uniform face coefficients in
[1e-3, 1]), all 64 ranks fused onto this GPU.  Inputs are seeded and
synthetic (no dataset); every timestep's per-rank coefficients are made on
the host and put in HBM before the timed region.

One step = one timestep of the whole path:
  update     per-rank diag/upper/interface values (device memory) staged into
             the receive buffer and reordered by P (FP64 + FP32 + Jacobi)
  FP64 PCG   A x = b from x = 0 to ||b - A x|| <= 1e-8 ||b||
  mixed      iterative refinement: FP32 inner PCG to 1e-4 under FP64 residual
             and solution, same b, x = 0, same target
  mixed_rr   FP32 PCG with FP64 residual replacement (a variant, reported apart)
  adjoint    lambda = A^-1 (x - x_t) (FP64 PCG) and the slot gradient
  momentum   the plan refreshed with a non-symmetric convection-diffusion
             system on the same ranks, solved with BiCGStab (FP64, 1e-8)
The plan (pattern, U, P) is built once before the steps and timed apart.

Prints one JSON line.  value = median ms per FP64 pressure solve; the mixed
solves, the SpMV bandwidth (HIP events around every FP64 SpMV launch inside
the timed solves), the roofline of that kernel and the oracle timed on the
host are reported beside it.  After the timed steps the unperturbed system
is solved once more by each method (untimed) and every answer is checked on
the host: its true residual by the oracle's SpMV, and its error against the
oracle's 1e-12 solution (tests/golden/ref_<config>.json) on the stored rows.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
TIMING_STRIDE = 8                # kernel timing records every 8th launch (rp_plan_set_timing)
METRIC = "ms per pressure solve to rel.res 1e-8 + SpMV HBM GB/s, FP64 vs mixed, 1 GPU"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=100,
                    help="oracle PCG iterations timed (beyond a 4-iteration run that carries the setup) "
                         "for the CPU baseline sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle's complete FP64 PCG solve to 1e-8 instead of a sample "
                         "(minutes of host time at 256^3)")
    ap.add_argument("--solve-order", default="fused", choices=["fused", "rcm"],
                    help="row order CG and the mixed solvers run in (rcm: the plan's reverse Cuthill-McKee copy)")
    ap.add_argument("--no-loop-legs", action="store_true",
                    help="skip the single-launch CG loop against three-kernel iteration legs")
    ap.add_argument("--no-preconditioners", action="store_true",
                    help="skip the Jacobi vs block-Jacobi leg (shorter profiler runs)")
    ap.add_argument("--rank-procs", type=int, default=8,
                    help="rank processes for the multi-process update leg (0: skip it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 2 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def profiled_traffic(config):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/traffic_<config>.md), or None when there is none or the
    kernel sources changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{config}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+); kernel: [^;]+; sources_sha256_16: ([0-9a-f]+)",
                  open(path).read())
    if not m:
        return None
    h = hashlib.sha256()
    for f in ("spmv.hpp", "cg.hip", "rp_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2510_08536_amd", "csrc", f), "rb").read())
    return int(m.group(1)) if h.hexdigest()[:16] == m.group(2) else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the library runs one plan on one GPU (asked for --gpus {a.gpus}); "
              "splitting the ranks over several GPUs is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import synth
    n_steps_total = a.warmup + a.steps
    t0 = time.time()
    w = synth.build(a.config, timesteps=max(n_steps_total, 1))
    gen_s = time.time() - t0
    p = w.part
    ranks = [p.rank(r) for r in range(w.n_ranks)]
    print(f"[bench] {a.config}: {w.n_cells} cells, {w.n_ranks} ranks, generated in {gen_s:.1f}s", flush=True)

    # rank processes, started before this process touches the GPU
    layout, so = [], 0
    for r in range(w.n_ranks):
        nc, nf, ni = int(p.n_cells[r]), len(ranks[r]["owner"]), len(ranks[r]["iface_cell"])
        layout.append((so, nc, nf, ni))
        so += nc + 2 * nf + ni
    pool, pool_err = None, None
    if a.rank_procs > 0:
        try:
            from paper_2510_08536_amd.ranks import RankPool
            pool = RankPool(min(a.rank_procs, w.n_ranks), layout)
        except Exception as e:  # reported in the JSON line, the rest still runs
            pool_err = f"{type(e).__name__}: {e}"

    import torch
    from paper_2510_08536_amd import (Plan, default_opts, RP_KERNEL_SPMV64, RP_KERNEL_SPMV32, RP_KERNEL_SCATTER,
                                      RP_LOOP_AUTO, RP_LOOP_COOPERATIVE, RP_LOOP_THREE, RP_LOOP_TWO_MAX_ROWS)

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")

    # ---- plan (once) -------------------------------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan(p.n_cells, 0, w.n_ranks, ranks)
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    n, nnz = plan.n_rows, plan.nnz
    print(f"[bench] plan: n={n} nnz={nnz} slots={plan.n_slots} in {plan_ms:.1f} ms", flush=True)
    order_ms = None
    if a.solve_order == "rcm":
        t0 = time.perf_counter()
        plan.set_solve_order("rcm")
        torch.cuda.synchronize()
        order_ms = 1e3 * (time.perf_counter() - t0)
        print(f"[bench] solve order (reverse Cuthill-McKee) built in {order_ms:.1f} ms", flush=True)

    # ---- per-timestep inputs, resident in HBM before timing ------------------
    def to_dev(v):
        return torch.from_numpy(np.ascontiguousarray(v)).to(dev)

    steps_vals = []
    for t in range(n_steps_total):
        v = w.values(t)
        steps_vals.append(([to_dev(v.diag[p.cell_ptr[r]:p.cell_ptr[r + 1]]) for r in range(w.n_ranks)],
                           [to_dev(v.upper[p.face_ptr[r]:p.face_ptr[r + 1]]) for r in range(w.n_ranks)],
                           [to_dev(v.iface[p.if_ptr[r]:p.if_ptr[r + 1]]) for r in range(w.n_ranks)]))
    # the non-symmetric momentum-type system on the same ranks (one set of
    # values, refreshed into the plan every step)
    vm = w.momentum_values()
    mom_vals = ([to_dev(vm.diag[p.cell_ptr[r]:p.cell_ptr[r + 1]]) for r in range(w.n_ranks)],
                [to_dev(vm.upper[p.face_ptr[r]:p.face_ptr[r + 1]]) for r in range(w.n_ranks)],
                [to_dev(vm.iface[p.if_ptr[r]:p.if_ptr[r + 1]]) for r in range(w.n_ranks)],
                [to_dev(vm.lower[p.face_ptr[r]:p.face_ptr[r + 1]]) for r in range(w.n_ranks)])
    del vm
    b = to_dev(w.rhs())
    xt = to_dev(w.target())
    print(f"[bench] {n_steps_total} timesteps of values resident in HBM", flush=True)

    # PCIe-inclusive update from pinned host buffers (reported apart, never `value`)
    vh = w.values(0)
    pin = lambda a_: torch.from_numpy(np.ascontiguousarray(a_)).pin_memory()
    host_vals = ([pin(vh.diag[p.cell_ptr[r]:p.cell_ptr[r + 1]]) for r in range(w.n_ranks)],
                 [pin(vh.upper[p.face_ptr[r]:p.face_ptr[r + 1]]) for r in range(w.n_ranks)],
                 [pin(vh.iface[p.if_ptr[r]:p.if_ptr[r + 1]]) for r in range(w.n_ranks)])
    plan.update(*host_vals)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.update(*host_vals)
    plan.sync()
    update_host_ms = 1e3 * (time.perf_counter() - t0)
    del host_vals

    if a.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    o64 = lambda: default_opts(tol=1e-8, precision="fp64", x0_zero=1)
    omx = lambda: default_opts(tol=1e-8, precision="mixed", x0_zero=1)
    omr = lambda: default_opts(tol=1e-8, precision="mixed_rr", x0_zero=1)
    obi = lambda: default_opts(tol=1e-8, precision="fp64", method="bicgstab", x0_zero=1)
    stream = torch.cuda.current_stream()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    prev = {}

    def one_step(t, rec):
        d, u, i = steps_vals[t]
        e0 = ev()
        plan.update(d, u, i)
        e1 = ev()
        x64, inf64 = plan.solve(b, opts=o64())
        e2 = ev()
        xmx, infmx = plan.solve(b, opts=omx())
        e3 = ev()
        _, infmr = plan.solve(b, opts=omr())
        e3b = ev()
        e3c = ev()
        lam, infl = plan.solve(x64 - xt, opts=o64())
        g = plan.value_grad(lam, x64)
        e4 = ev()
        plan.update(mom_vals[0], mom_vals[1], mom_vals[2], lower=mom_vals[3])
        e5 = ev()
        xbi, infbi = plan.solve(b, opts=obi())
        e6 = ev()
        # warm start: the pressure system again, from the previous timestep's
        # solution (reported apart; the values differ by up to 5 %)
        infw = None
        ew0 = ev()
        if "x" in prev:
            plan.update(d, u, i)
            ew0 = ev()
            xw, infw = plan.solve(b, x=prev["x"].clone(), opts=default_opts(tol=1e-8, precision="fp64"))
        ew1 = ev()
        prev["x"] = x64
        if rec is not None:
            rec.append(dict(ev=(e0, e1, e2, e3, e4, e5, e6), rr_ev=(e3, e3b), adj_ev=(e3c, e4),
                            warm=(ew0, ew1, infw), fp64=inf64, mixed=infmx, mixed_rr=infmr,
                            adj=infl, bicg=infbi, x64=x64, xmx=xmx))
        for info in (inf64, infmx, infmr, infl, infbi) + ((infw,) if infw is not None else ()):
            assert info["status"] == 0 and info["rel_res"] <= 1e-8, info
        return g

    for t in range(a.warmup):
        one_step(t, None)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({a.warmup} steps)", flush=True)

    # HIP events around every TIMING_STRIDE-th launch of the timed kernels: an
    # event pair costs the stream several microseconds, so timing every launch
    # would slow the timed solves it measures
    plan.set_timing(TIMING_STRIDE)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        one_step(a.warmup + k, recs)
        print(f"[bench] step {k + 1}/{a.steps}: fp64 {recs[-1]['fp64']['iters']} it, "
              f"mixed {recs[-1]['mixed']['iters']} inner/{recs[-1]['mixed']['outer_iters']} outer, "
              f"mixed_rr {recs[-1]['mixed_rr']['iters']} inner/{recs[-1]['mixed_rr']['outer_iters']} updates",
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_spmv, ms_spmv = plan.kernel_stats(RP_KERNEL_SPMV64)
    ranks_update = rank_process_update(pool, pool_err, plan, w, layout, torch) if a.rank_procs > 0 else None

    # SpMV alone: 200 launches of y = A x on the last step's pressure matrix
    plan.update(*steps_vals[n_steps_total - 1])
    xs_ = torch.rand(n, dtype=torch.float64, device=dev)
    ys_ = torch.empty_like(xs_)
    for _ in range(5):
        plan.spmv(xs_, y=ys_)
    ts_ = []
    for _ in range(200):
        e_a, e_b = ev(), None
        plan.spmv(xs_, y=ys_)
        e_b = ev()
        ts_.append((e_a, e_b))
    torch.cuda.synchronize()
    spmv_micro_us = float(np.median([1e3 * e_a.elapsed_time(e_b) for e_a, e_b in ts_]))
    n_spmv32, ms_spmv32 = plan.kernel_stats(RP_KERNEL_SPMV32)
    n_scat, ms_scat = plan.kernel_stats(RP_KERNEL_SCATTER)
    plan.set_timing(False)
    # block-Jacobi preconditioner (blocks of consecutive rows inside a rank)
    # against Jacobi on the same system: 3 timed solves each, after one warm-up
    bj = {}
    legs = () if a.no_preconditioners else (("jacobi", dict(precision="fp64")),
                                            ("block_jacobi_4", dict(precision="fp64", precond="block_jacobi",
                                                                    block_size=4)),
                                            ("block_jacobi_8", dict(precision="fp64", precond="block_jacobi",
                                                                    block_size=8)),
                                            ("mixed_block_jacobi_4", dict(precision="mixed", precond="block_jacobi",
                                                                          block_size=4)),
                                            ("amg", dict(precision="fp64", precond="amg")),
                                            ("mixed_amg", dict(precision="mixed", precond="amg")))
    if a.solve_order != "fused":
        # block-Jacobi blocks are runs of fused rows: not in the solve order
        legs = tuple(lg for lg in legs if lg[1].get("precond") != "block_jacobi")
    amg_info = None
    if legs:
        # multigrid hierarchy of the last step's system, built once (the legs
        # below reuse it; a value update only refreshes its coarse values)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.amg_setup()
        torch.cuda.synchronize()
        amg_setup_ms = 1e3 * (time.perf_counter() - t0)
        sizes = [plan.amg_level(l)["n"] for l in range(plan.amg_levels())]
        amg_info = {"setup_ms": round(amg_setup_ms, 2), "levels": len(sizes), "rows_per_level": sizes}
    for label, kw in legs:
        plan.solve(b, opts=default_opts(tol=1e-8, x0_zero=1, **kw))
        ts, its = [], []
        for _ in range(3):
            e_a = ev()
            _, ib = plan.solve(b, opts=default_opts(tol=1e-8, x0_zero=1, **kw))
            e_b = ev()
            torch.cuda.synchronize()
            assert ib["status"] == 0 and ib["rel_res"] <= 1e-8, ib
            ts.append(e_a.elapsed_time(e_b))
            its.append(ib["iters"])
        bj[label] = {"ms_per_solve": round(float(np.median(ts)), 3), "iters": int(np.median(its))}
    for label in bj:
        bj[label]["speedup_vs_jacobi"] = round(bj["jacobi"]["ms_per_solve"] / bj[label]["ms_per_solve"], 3)
    if amg_info is not None:
        # value refresh: new values, then the first multigrid solve
        # refreshes the coarse values (timed against a steady solve)
        plan.update(*steps_vals[0])
        e_a = ev()
        plan.solve(b, opts=default_opts(tol=1e-8, x0_zero=1, precision="fp64", precond="amg"))
        e_b = ev()
        plan.solve(b, opts=default_opts(tol=1e-8, x0_zero=1, precision="fp64", precond="amg"))
        e_c = ev()
        torch.cuda.synchronize()
        amg_info["refresh_ms"] = round(e_a.elapsed_time(e_b) - e_b.elapsed_time(e_c), 2)
        plan.update(*steps_vals[n_steps_total - 1])
        bj["amg_hierarchy"] = amg_info
    print(f"[bench] preconditioners: {bj}", flush=True)
    # launches per CG iteration (kernel timing off in all): three, two (the
    # x and p update fused with the next SpMV; systems of at most
    # RP_LOOP_TWO_MAX_ROWS rows) and one cooperative launch; per-iteration
    # time, on systems of up to 2^20 rows
    loop = {}
    forms = [(RP_LOOP_THREE, "three_kernel"), (RP_LOOP_COOPERATIVE, "single_launch")]
    if n <= RP_LOOP_TWO_MAX_ROWS:
        forms.insert(1, (RP_LOOP_AUTO, "two_launch"))
    for prec in (() if a.no_loop_legs or n > (1 << 20) else ("fp64", "mixed")):
        for fl, label in forms:
            kw = dict(tol=1e-8, x0_zero=1, precision=prec, fused_loop=fl)
            plan.solve(b, opts=default_opts(**kw))
            ts, its = [], []
            for _ in range(3):
                e_a = ev()
                _, ib = plan.solve(b, opts=default_opts(**kw))
                e_b = ev()
                torch.cuda.synchronize()
                assert ib["status"] == 0 and ib["rel_res"] <= 1e-8, ib
                ts.append(e_a.elapsed_time(e_b))
                its.append(ib["iters"])
            ms, it_ = float(np.median(ts)), int(np.median(its))
            loop[f"{prec}_{label}"] = {"ms_per_solve": round(ms, 3), "iters": it_,
                                       "us_per_iter": round(1e3 * ms / max(it_, 1), 2)}
        for _, label in forms[1:]:
            loop[f"{prec}_{label}"]["speedup"] = round(loop[f"{prec}_three_kernel"]["ms_per_solve"]
                                                       / loop[f"{prec}_{label}"]["ms_per_solve"], 3)
    print(f"[bench] cg loop: {loop}", flush=True)

    el = lambda e_a, e_b: e_a.elapsed_time(e_b)
    upd = [el(r["ev"][0], r["ev"][1]) for r in recs]
    f64 = [el(r["ev"][1], r["ev"][2]) for r in recs]
    mx = [el(r["ev"][2], r["ev"][3]) for r in recs]
    mr = [el(*r["rr_ev"]) for r in recs]
    adj = [el(*r["adj_ev"]) for r in recs]
    mupd = [el(r["ev"][4], r["ev"][5]) for r in recs]
    warm = [(el(r["warm"][0], r["warm"][1]), r["warm"][2]["iters"]) for r in recs if r["warm"][2] is not None]
    bic = [el(r["ev"][5], r["ev"][6]) for r in recs]
    itbi = [r["bicg"]["iters"] for r in recs]
    it64 = [r["fp64"]["iters"] for r in recs]
    itmx = [r["mixed"]["iters"] for r in recs]
    itmr = [r["mixed_rr"]["iters"] for r in recs]
    restarts = {k: int(sum(r[k]["restarts"] for r in recs)) for k in ("fp64", "mixed", "mixed_rr", "adj", "bicg")}
    last = recs[-1]
    diff = (torch.linalg.vector_norm(last["x64"] - last["xmx"]) / torch.linalg.vector_norm(last["x64"])).item()

    # ---- accuracy (untimed): the unperturbed system by every method ----------
    v0 = w.values(None)
    plan.update([to_dev(v0.diag[p.cell_ptr[r]:p.cell_ptr[r + 1]]) for r in range(w.n_ranks)],
                [to_dev(v0.upper[p.face_ptr[r]:p.face_ptr[r + 1]]) for r in range(w.n_ranks)],
                [to_dev(v0.iface[p.if_ptr[r]:p.if_ptr[r + 1]]) for r in range(w.n_ranks)])
    answers = {}
    for label, mk in (("fp64", o64), ("mixed", omx), ("mixed_rr", omr)):
        xa, ia = plan.solve(b, opts=mk())
        answers[label] = (xa.cpu().numpy(), ia)
    del xa

    # algorithmic bytes per unit of work (each array read once, ideal reuse of
    # x): the CSR SpMV moves val + col per entry, row_ptr, x and y; a PCG
    # iteration adds the vector kernels.  The kernels move less where row
    # groups are offset-coded (no col array); those bytes are reported beside.
    fmt = plan.spmv_format()
    spmv64_bytes = 12 * nnz + 20 * n + 4
    spmv32_bytes = 8 * nnz + 12 * n + 4
    iter64_bytes = 12 * nnz + 108 * n
    iter32_bytes = 8 * nnz + 56 * n
    # BiCGStab iteration: two CSR SpMVs plus 168 n of vectors (p, y, v, rh, s, z, t, x, r)
    iterbi_bytes = 2 * (12 * nnz + 20 * n) + 168 * n
    kern64_fused = fmt["bytes64"]            # what the SpMV kernels read and write in the form in use
    # the solves' SpMV: the fused form, or plain CSR groups on the solve-order copy
    rcm = a.solve_order == "rcm"
    kern64_bytes = spmv64_bytes if rcm else fmt["bytes64"]
    kern32_bytes = spmv32_bytes if rcm else fmt["bytes32"]
    spmv_avg_ms = ms_spmv / max(n_spmv, 1)
    spmv32_avg_ms = ms_spmv32 / max(n_spmv32, 1)
    spmv_gbs = spmv64_bytes / (spmv_avg_ms * 1e-3) / 1e9
    spmv32_gbs = spmv32_bytes / (spmv32_avg_ms * 1e-3) / 1e9
    med = lambda v: float(np.median(v))

    out = {
        "metric": METRIC,
        "value": round(med(f64), 3),
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * wall / a.steps, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {w.recipe.note}", "n_rows": n, "nnz": nnz, "alpha": w.n_ranks,
                   "tol": 1e-8, "x0": "zero", "solve_order": a.solve_order,
                   "step": "update + FP64 PCG + mixed PCG + adjoint (lambda solve + slot gradient) + "
                           "momentum update + BiCGStab"},
        "fp64": {"ms_per_solve": round(med(f64), 3), "iters": int(np.median(it64)),
                 "ms_per_iter": round(med(f64) / max(np.median(it64), 1), 4),
                 "iter_GBps_alg": round(iter64_bytes * np.median(it64) / (med(f64) * 1e-3) / 1e9, 1)},
        "mixed": {"method": "iterative refinement: FP32 inner PCG to 1e-4, FP64 residual and solution",
                  "ms_per_solve": round(med(mx), 3), "inner_iters": int(np.median(itmx)),
                  "outer_iters": int(last["mixed"]["outer_iters"]),
                  "speedup_vs_fp64": round(med(f64) / med(mx), 3),
                  "rel_diff_vs_fp64_solution": diff,
                  "inner_iter_GBps_alg": round(iter32_bytes * np.median(itmx) / (med(mx) * 1e-3) / 1e9, 1)},
        "mixed_rr": {"method": "FP32 PCG with FP64 residual replacement every 0.1 reduction (variant)",
                     "ms_per_solve": round(med(mr), 3), "inner_iters": int(np.median(itmr)),
                     "fp64_updates": int(last["mixed_rr"]["outer_iters"]),
                     "speedup_vs_fp64": round(med(f64) / med(mr), 3)},
        "restarts_in_timed_solves": restarts,
        "preconditioners": dict(bj, note="last timestep's system, x0 = 0, tol 1e-8, 3 solves each (median); "
                                         "block_jacobi_b: blocks of b consecutive rows inside each rank; "
                                         "amg: one aggregation-multigrid V-cycle per iteration (hierarchy "
                                         "built once: amg_hierarchy.setup_ms; a value update refreshes the "
                                         "coarse values: refresh_ms)"),
        "cg_loop": dict(loop, note="last timestep's system, x0 = 0, tol 1e-8, 3 solves each (median); "
                                   "three_kernel: one launch per phase; two_launch: the x and p update "
                                   "fused with the next SpMV (systems of at most 2^18 rows); single_launch: "
                                   "the iterations in one cooperative launch with grid-wide barriers")
        if loop else None,
        "fp64_warm_start": ({"ms_per_solve": round(float(np.median([wm for wm, _ in warm])), 3),
                             "iters": int(np.median([wi for _, wi in warm])),
                             "note": "x0 = previous timestep's x; values differ by up to 5 % between timesteps"}
                            if warm else None),
        "momentum_bicgstab": {"ms_per_solve": round(med(bic), 3), "iters": int(np.median(itbi)),
                              "ms_per_iter": round(med(bic) / max(np.median(itbi), 1), 4),
                              "iter_GBps_alg": round(iterbi_bytes * np.median(itbi) / (med(bic) * 1e-3) / 1e9, 1),
                              "update_ms": round(med(mupd), 3)},
        "adjoint_ms": round(med(adj), 3),
        "adjoint_iters": int(np.median([r["adj"]["iters"] for r in recs])),
        "update_ms": round(med(upd), 3),
        "update_scatter_ms": round(ms_scat / max(n_scat, 1), 4),
        "update_host_staged_ms": round(update_host_ms, 3),
        "update_from_rank_processes": ranks_update,
        "plan_ms": round(plan_ms, 1),
        "solve_order_build_ms": None if order_ms is None else round(order_ms, 1),
        "spmv_GBps": round(spmv_gbs, 1),
        "spmv32_GBps": round(spmv32_gbs, 1),
        "spmv_alone": {"median_us": round(spmv_micro_us, 2), "launches": 200,
                       "GBps": round(spmv64_bytes / (spmv_micro_us * 1e-6) / 1e9, 1),
                       "kernel_GBps": round(kern64_fused / (spmv_micro_us * 1e-6) / 1e9, 1)},
        "spmv_format": {"coded_groups": fmt["coded_groups"], "n_groups": fmt["n_groups"],
                        "coded_nnz_frac": round(fmt["coded_nnz"] / max(nnz, 1), 4),
                        "kernel_bytes64": kern64_bytes, "kernel_GBps64": round(kern64_bytes / (spmv_avg_ms * 1e-3) / 1e9, 1),
                        "kernel_bytes32": kern32_bytes,
                        "kernel_GBps32": round(kern32_bytes / (spmv32_avg_ms * 1e-3) / 1e9, 1)},
        "roofline": {"bound": "hbm",
                     "kernel": "cg_spmv_pq<double> (FP64 SpMV + p.q; " + (
                         "CSR groups on the reverse Cuthill-McKee solve order)" if rcm else "offset-coded row groups)"),
                     "achieved": round(spmv_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(spmv_gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": spmv64_bytes, "bytes_basis": "12 nnz + 20 n + 4 (FP64 CSR SpMV)",
                     "kernel_bytes_per_launch": kern64_bytes, "avg_launch_ms": round(spmv_avg_ms, 5),
                     "launches": n_spmv, "timed_launches": f"HIP events around every {TIMING_STRIDE}th launch "
                                                           "of the timed steps", "traffic": None if rcm else profiled_traffic(a.config),
                     "traffic_note": "HBM bytes/launch from FETCH_SIZE+WRITE_SIZE (profiles/traffic_c3.md), "
                                     "scaled by a 2 GiB copy; null if the kernel changed since"},
    }

    out["accuracy"] = accuracy(w, a.config, answers)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_iters, a.cpu_full, med(f64), int(np.median(it64)),
                                           answers["fp64"][1]["iters"])
    print(json.dumps(out), flush=True)
    plan.close()


def rank_process_update(pool, pool_err, plan, w, layout, torch):
    """The update with the ranks' values in other processes (timesteps 0-2,
    each twice, the second timed): every process writes its ranks' slot
    blocks into the plan's device receive buffer through its IPC handle and
    the plan reorders that buffer (GPU-aware path), or writes them into a
    shared host buffer that rp_update_values copies to the device, one copy
    per rank array (host-buffer path).  Wall time from the request to the
    reordered matrix."""
    if pool is None:
        return {"error": pool_err or "no rank processes"}
    try:
        T = min(3, len(w.step_seqs))
        bufs = []
        for t in range(T):
            v = w.values(t)
            parts = []
            for r, (off, nc, nf, ni) in enumerate(layout):
                c0, f0, i0 = w.part.cell_ptr[r], w.part.face_ptr[r], w.part.if_ptr[r]
                up = v.upper[f0:f0 + nf]
                parts += [v.diag[c0:c0 + nc], up, up, v.iface[i0:i0 + ni]]
            bufs.append(np.concatenate(parts))
            del v, parts
        t0 = time.perf_counter()
        pool.load(bufs)
        load_s = time.perf_counter() - t0
        del bufs
        pool.attach_device(plan.export_recv())
        host = pool.host_buffer(plan.n_slots)
        views = [host[off:off + nc + 2 * nf + ni] for off, nc, nf, ni in layout]
        hd = [vw[:nc] for vw, (_, nc, nf, ni) in zip(views, layout)]
        hu = [vw[nc:nc + nf] for vw, (_, nc, nf, ni) in zip(views, layout)]
        hl = [vw[nc + nf:nc + 2 * nf] for vw, (_, nc, nf, ni) in zip(views, layout)]
        hi = [vw[nc + 2 * nf:] for vw, (_, nc, nf, ni) in zip(views, layout)]
        dev_ms, host_ms, dev_w, host_w = [], [], [], []
        for rep in range(2):
            for t in range(T):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ww = pool.write_device(t)
                plan.update_from_recv()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                wh = pool.write_host(t)
                plan.update(hd, hu, hi, lower=hl)      # host arrays: copies + reorder, synchronised
                t2 = time.perf_counter()
                if rep == 1:
                    dev_ms.append(1e3 * (t1 - t0))
                    host_ms.append(1e3 * (t2 - t1))
                    dev_w.append(1e3 * ww)
                    host_w.append(1e3 * wh)
        out = {"processes": len(pool.procs), "ranks": len(layout),
               "gpu_aware_ipc_ms": round(float(np.median(dev_ms)), 3),
               "gpu_aware_ipc_worker_write_ms": round(float(np.median(dev_w)), 3),
               "host_buffer_ms": round(float(np.median(host_ms)), 3),
               "host_buffer_worker_write_ms": round(float(np.median(host_w)), 3),
               "speedup_ipc_vs_host": round(float(np.median(host_ms)) / float(np.median(dev_ms)), 3),
               "values_load_s": round(load_s, 2),
               "note": "wall time from the request to the reordered matrix, median of 3 timesteps; values "
                       "start in each rank process's own (pageable) memory"}
    except Exception as e:
        out = {"error": f"{type(e).__name__}: {e}"}
    finally:
        pool.close()
    return out


def accuracy(w, config, answers):
    """Host check of the untimed answers on the unperturbed system: the true
    relative residual of each by the oracle's SpMV, and its error against the
    oracle's 1e-12 solution on the stored rows (when a reference exists)."""
    import oracle
    ranks = [w.part.rank(r) for r in range(w.n_ranks)]
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, ranks)
    vals = w.values(None)
    val64, *_ = oracle.update(m, oracle.receive_buffer([vals.rank(w.part, r) for r in range(w.n_ranks)]))
    del vals
    b = w.rhs()
    ref_path = os.path.join(ROOT, "tests", "golden", f"ref_{config}.json")
    ref = None
    if os.path.exists(ref_path):
        with open(ref_path) as f:
            ref = json.load(f)
        if ref.get("timestep") is not None:
            ref = None          # the reference is for another timestep's values
    out = {"system": "unperturbed coefficients (kappa_0), x0 = 0, tol 1e-8"}
    if ref is not None:
        rows = np.asarray(ref["rows"], dtype=np.int64)
        x_ref = np.asarray([float(v) for v in ref["x_ref"]])
        out["reference"] = (f"oracle PCG to {ref['reference']['tol']:g} (tests/golden/ref_{config}.json), "
                            f"{rows.size} sampled rows")
        out["oracle_1e-8_err_vs_reference"] = ref["oracle_1e-8"]["rel_err_vs_ref_sampled"]
    for label, (x, info) in answers.items():
        d = {"iters": info["iters"], "outer_iters": info["outer_iters"], "restarts": info["restarts"],
             "oracle_rel_res": oracle.true_relres(m, val64, b, x)}
        if ref is not None:
            d["err_vs_reference"] = float(np.linalg.norm(x[rows] - x_ref) / np.linalg.norm(x_ref))
        out[label] = d
    return out


def cpu_baseline(w, iters, full, gpu_ms, gpu_iters, gpu_iters_unperturbed):
    """The oracle (serial C, pinned to one host core) on the same system as
    the last timed step's FP64 solve.  Merge and update are timed in full.
    The PCG is either timed in full (full=True: to 1e-8 from x = 0), or as a
    sample: a run of 4 iterations (setup: diagonal scan, r = b - A x, first
    touch of the work vectors) and a run of 4 + iters; their difference is
    the steady per-iteration time, and the solve is rated as the 4-iteration
    run plus (GPU iterations - 4) such iterations."""
    import oracle
    cpu = sorted(os.sched_getaffinity(0))[0]
    old_aff = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {cpu})
    try:
        ranks = [w.part.rank(r) for r in range(w.n_ranks)]
        t0 = time.perf_counter()
        m = oracle.merge(w.part.n_cells, 0, w.n_ranks, ranks)
        merge_s = time.perf_counter() - t0
        vals = w.values(None)
        buf = oracle.receive_buffer([vals.rank(w.part, r) for r in range(w.n_ranks)])
        del vals
        t0 = time.perf_counter()
        val64, *_ = oracle.update(m, buf)
        update_s = time.perf_counter() - t0
        del buf
        b = w.rhs()
        if full:
            t0 = time.perf_counter()
            _, st, it, rs, rr = oracle.pcg(m, val64, b, tol=1e-8)
            solve_s = time.perf_counter() - t0
            value_ms = 1e3 * solve_s
            sample = (f"full serial FP64 PCG solve to 1e-8 from x = 0 on the {w.n_cells}-row system: "
                      f"{it} iterations, {rs} restarts, rel.res {rr:.2e}")
            per_iter_ms = value_ms / max(it, 1)
            extra = {"iters": it, "solve_s": round(solve_s, 1)}
        else:
            k0 = 4
            t0 = time.perf_counter()
            oracle.pcg(m, val64, b, tol=1e-8, max_iter=k0)
            t_k0 = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, _, it1, _, _ = oracle.pcg(m, val64, b, tol=1e-8, max_iter=k0 + iters)
            t_k1 = time.perf_counter() - t0
            per_iter_ms = 1e3 * (t_k1 - t_k0) / max(it1 - k0, 1)
            value_ms = 1e3 * t_k0 + per_iter_ms * max(gpu_iters_unperturbed - k0, 0)
            sample = (f"serial FP64 PCG on the same {w.n_cells}-row system: a {k0}-iteration run "
                      f"({1e3 * t_k0:.0f} ms, with setup) and a {it1}-iteration run; their difference gives "
                      f"{per_iter_ms:.1f} ms per steady iteration; rated at the GPU's "
                      f"{gpu_iters_unperturbed} iterations on this system")
            extra = {"setup_plus_4_iters_ms": round(1e3 * t_k0, 1), "timed_iters": it1 - k0}
    finally:
        os.sched_setaffinity(0, old_aff)
    return {"value": round(value_ms, 1), "unit": "ms/solve", "cores": 1, "kind": "oracle",
            "sample": sample + f"; merge {merge_s:.1f} s and update {1e3 * update_s:.0f} ms timed in full; "
                               f"pinned to host CPU {cpu}",
            "merge_s": round(merge_s, 2), "update_ms": round(1e3 * update_s, 1),
            "pcg_ms_per_iter": round(per_iter_ms, 2), "gpu_speedup": round(value_ms / gpu_ms, 1),
            "host_cpu": cpu_model(), "host_nproc": os.cpu_count(), **extra}


if __name__ == "__main__":
    main()
