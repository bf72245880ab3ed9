"""CPU ranks in processes of their own, handing their coefficients to the GPU
owner (the update procedure of Sec. 3; the GPU-aware vs host-buffer study of
Sec. 4).

RankPool starts worker processes (plain child processes of this program;
start them before it touches the GPU where it can).  Each worker owns a
contiguous run of the share's ranks and keeps their per-timestep values in
its own memory, as a CPU rank does.  For one update every worker, at once,
either
  - writes its ranks' slot blocks straight into the owner's device receive
    buffer through the IPC handle the owner exported (RecvWriter; the
    GPU-aware path), after which the owner reorders that buffer, or
  - copies them into a receive buffer in shared host memory, which the owner
    then hands to rp_update_values as host arrays (one host-to-device copy
    per rank array; the host-buffer path).
Workers talk to the owner over their stdin/stdout (one JSON object per line);
bulk values travel through POSIX shared memory.
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import time
from multiprocessing import shared_memory

import numpy as np


def _split(n_ranks: int, n_workers: int):
    """contiguous rank runs, as even as possible"""
    b = np.linspace(0, n_ranks, n_workers + 1).round().astype(int)
    return [(int(b[k]), int(b[k + 1])) for k in range(n_workers) if b[k + 1] > b[k]]


class RankPool:
    """n_workers rank processes for a share described by layout[r] =
    (slot_offset, n_cells, n_faces, n_iface) of every share rank."""

    def __init__(self, n_workers: int, layout):
        self.layout = [tuple(int(v) for v in r) for r in layout]
        self.runs = _split(len(self.layout), n_workers)
        env = dict(os.environ)
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        env["PYTHONPATH"] = root + os.pathsep + env.get("PYTHONPATH", "")
        self.procs = [subprocess.Popen([sys.executable, "-u", "-m", "paper_2510_08536_amd.ranks"],
                                       stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
                      for _ in self.runs]
        self._shm = []
        self._send_all(lambda k: {"cmd": "ranks", "ranks": self.layout[self.runs[k][0]:self.runs[k][1]]})

    # -- plumbing -------------------------------------------------------------
    def _send_all(self, msg_of):
        for k, p in enumerate(self.procs):
            p.stdin.write(json.dumps(msg_of(k)) + "\n")
            p.stdin.flush()
        out = []
        for p in self.procs:
            line = p.stdout.readline()
            if not line:
                raise RuntimeError(f"rank worker {p.pid} ended (exit code {p.poll()})")
            r = json.loads(line)
            if "error" in r:
                raise RuntimeError(f"rank worker {p.pid}: {r['error']}")
            out.append(r)
        return out

    def load(self, buffers):
        """buffers[t]: float64[n_slots], timestep t's values in slot order.
        Every worker copies its ranks' blocks into its own memory."""
        T, ns = len(buffers), len(buffers[0])
        shm = shared_memory.SharedMemory(create=True, size=max(8 * T * ns, 8))
        try:
            view = np.ndarray((T, ns), dtype=np.float64, buffer=shm.buf)
            for t, b in enumerate(buffers):
                view[t] = b
            self._send_all(lambda k: {"cmd": "load", "shm": shm.name, "T": T, "n_slots": ns})
        finally:
            del view
            shm.close()
            shm.unlink()

    def attach_device(self, handle: bytes):
        self._send_all(lambda k: {"cmd": "attach", "handle": handle.hex()})

    def write_device(self, t: int) -> float:
        """All workers write timestep t into the owner's device buffer; returns
        the longest worker time (s)."""
        return max(r["s"] for r in self._send_all(lambda k: {"cmd": "write_device", "t": t}))

    def host_buffer(self, n_slots: int) -> np.ndarray:
        """A receive buffer in shared host memory the workers write into."""
        shm = shared_memory.SharedMemory(create=True, size=max(8 * n_slots, 8))
        self._shm.append(shm)
        self._send_all(lambda k: {"cmd": "host_attach", "shm": shm.name, "n_slots": n_slots})
        return np.ndarray((n_slots,), dtype=np.float64, buffer=shm.buf)

    def write_host(self, t: int) -> float:
        return max(r["s"] for r in self._send_all(lambda k: {"cmd": "write_host", "t": t}))

    def close(self):
        for p in self.procs:
            try:
                p.stdin.write(json.dumps({"cmd": "quit"}) + "\n")
                p.stdin.flush()
            except (BrokenPipeError, ValueError):
                pass
        for p in self.procs:
            try:
                p.wait(timeout=60)
            except subprocess.TimeoutExpired:
                p.kill()
                p.wait()
        for shm in self._shm:
            shm.close()
            shm.unlink()
        self._shm = []
        self.procs = []


# ---------------------------------------------------------------------------
# worker side
# ---------------------------------------------------------------------------
def _attach_shm(name):
    """a segment the owner created and will unlink (not tracked here)"""
    shm = shared_memory.SharedMemory(name=name)
    try:
        from multiprocessing import resource_tracker
        resource_tracker.unregister(shm._name, "shared_memory")
    except Exception:
        pass
    return shm


def _worker():
    ranks, vals, writer, host = [], [], None, None
    host_shm = None
    for line in sys.stdin:
        msg = json.loads(line)
        cmd = msg["cmd"]
        try:
            if cmd == "quit":
                break
            if cmd == "ranks":
                ranks = [tuple(r) for r in msg["ranks"]]
                out = {}
            elif cmd == "load":
                shm = _attach_shm(msg["shm"])
                src = np.ndarray((msg["T"], msg["n_slots"]), dtype=np.float64, buffer=shm.buf)
                # each rank's [diag | upper | lower | iface] kept as arrays of its own
                vals = []
                for t in range(msg["T"]):
                    per = []
                    for off, nc, nf, ni in ranks:
                        blk = src[t, off:off + nc + 2 * nf + ni]
                        per.append((blk[:nc].copy(), blk[nc:nc + nf].copy(), blk[nc + nf:nc + 2 * nf].copy(),
                                    blk[nc + 2 * nf:].copy()))
                    vals.append(per)
                del src
                shm.close()
                out = {}
            elif cmd == "attach":
                from paper_2510_08536_amd.rp import RecvWriter
                writer = RecvWriter(bytes.fromhex(msg["handle"]))
                out = {}
            elif cmd == "write_device":
                t0 = time.perf_counter()
                for (off, nc, nf, ni), (d, u, lo, i) in zip(ranks, vals[msg["t"]]):
                    writer.write(off, d, u, i, lower=lo)
                out = {"s": time.perf_counter() - t0}
            elif cmd == "host_attach":
                host_shm = _attach_shm(msg["shm"])
                host = np.ndarray((msg["n_slots"],), dtype=np.float64, buffer=host_shm.buf)
                out = {}
            elif cmd == "write_host":
                t0 = time.perf_counter()
                for (off, nc, nf, ni), (d, u, lo, i) in zip(ranks, vals[msg["t"]]):
                    host[off:off + nc] = d
                    host[off + nc:off + nc + nf] = u
                    host[off + nc + nf:off + nc + 2 * nf] = lo
                    host[off + nc + 2 * nf:off + nc + 2 * nf + ni] = i
                out = {"s": time.perf_counter() - t0}
            else:
                out = {"error": f"unknown command {cmd}"}
        except Exception as e:  # reported to the owner, which raises
            out = {"error": f"{type(e).__name__}: {e}"}
        sys.stdout.write(json.dumps(out) + "\n")
        sys.stdout.flush()
    if writer is not None:
        writer.close()
    if host_shm is not None:
        del host
        host_shm.close()


if __name__ == "__main__":
    _worker()
