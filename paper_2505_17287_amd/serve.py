"""Continuous-batching server for ghost-cell projections on one GPU.

Each request is a whole projection (classification against its own body, ghost-cell
stencils and multigrid hierarchy, divergence right-hand side, pressure solve, velocity
correction) on its own grid.  The server keeps a few *slots*; a slot is a host worker
thread with its own HIP stream and a cache of grid handles (one per distinct grid, with
its workspace resident in HBM), so consecutive requests on the same grid reuse the bound
workspace and only re-run the geometry-dependent setup.

Admission by HBM footprint: the budget covers every resident workspace (the grid caches of
all slots) plus what the requests in flight hold (their velocity and pressure fields, and
the workspace of a grid a request is about to create).  A request is admitted in arrival
order when a slot is free and that total, with the request's own need added, stays within
the budget; to make room the least recently used cached grids of idle slots are released
first.  Concurrent slots overlap on the GPU: small grids leave most compute units idle and
are launch-latency bound, so running several at once raises throughput.

Latency of a request = host wall clock from its arrival to the moment its status and
statistics are visible on the host (its stream has completed); the corrected velocity and
the pressure stay in HBM.  Every slot runs the same deterministic kernels on a private
workspace, so a request's result does not depend on what runs beside it or before it on the
same handle.  A request that fails (a library error) is returned as a result carrying the
error; the other requests are served.

Threads rather than the library's non-blocking step API: the set-up calls of a request
(mesh upload and check, classification, stencils) synchronise their stream, and the
projection wraps the solve in the right-hand side and correction passes; a worker thread per
slot runs them as blocking calls, and ctypes releases the interpreter lock for the length
of each call, so the slots' GPU work overlaps just the same.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import ibm
from . import inputs as I


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the trace
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    verts: np.ndarray
    tris: np.ndarray
    vel_seed: int
    name: str = ""

    @property
    def shape(self):
        return (len(self.zf) - 1, len(self.yf) - 1, len(self.xf) - 1)

    @property
    def ncells(self):
        nz, ny, nx = self.shape
        return nx * ny * nz

    def grid_key(self):
        return (self.xf.tobytes(), self.yf.tobytes(), self.zf.tobytes())


@dataclass
class Result:
    rid: int
    name: str
    arrival: float
    admitted: float
    done: float
    slot: int
    status: int
    cycles: int
    rel_residual: float
    div_max: float
    counts: tuple
    p: object = None               # host copy of the pressure when the server keeps results
    u: object = None
    error: str = ""                # message of a failed request (status < 0)

    @property
    def latency(self):
        return self.done - self.arrival


def make_trace(n_requests: int, qps: float | None, trace_seed: int = 5, sizes=(64, 128, 192, 256),
               requests: list | None = None):
    """Requests ``0..n_requests-1`` of the seeded request stream (geometry and grid from
    ``inputs.serving_request``) with exponential inter-arrival times at rate ``qps``;
    ``qps=None`` puts every arrival at t = 0 (saturation).  Pass ``requests`` to re-time an
    already generated list."""
    if requests is None:
        requests = []
        for r in range(n_requests):
            wl = I.serving_request(r, trace_seed=trace_seed, sizes=sizes)
            requests.append(Request(r, 0.0, wl.xf, wl.yf, wl.zf, wl.verts, wl.tris, wl.seed, wl.name))
    rng = np.random.default_rng([trace_seed, 7919])
    gaps = rng.exponential(1.0 / qps, size=len(requests)) if qps else np.zeros(len(requests))
    t = np.cumsum(gaps) - (gaps[0] if len(gaps) else 0.0)
    return [Request(q.rid, float(t[i]), q.xf, q.yf, q.zf, q.verts, q.tris, q.vel_seed, q.name)
            for i, q in enumerate(requests)]


def field_bytes(req: Request) -> int:
    nz, ny, nx = req.shape
    return 8 * (nz * ny * (nx + 1) + nz * (ny + 1) * nx + (nz + 1) * ny * nx + nx * ny * nz)


def workspace_bound(req: Request, precision: str) -> int:
    """Upper bound of the workspace a handle for this request's grid, mesh and ghost
    capacity binds (ibm_workspace_bytes, no handle needed)."""
    nz, ny, nx = req.shape
    mg = ibm.estimate_max_ghosts(req.xf, req.yf, req.zf, req.verts, req.tris)
    prec = ibm.IBM_MIXED if precision == "mixed" else ibm.IBM_FP64
    return int(ibm.lib().ibm_workspace_bytes(nx, ny, nz, len(req.verts), len(req.tris), mg, prec))


def footprint(req: Request, precision: str) -> int:
    """Device bytes of a request on a slot without a cached grid for it: the workspace bound
    plus u, v, w and p."""
    return workspace_bound(req, precision) + field_bytes(req)


class _Slot:
    def __init__(self, index, device):
        import torch
        self.index = index
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.grids = {}                                  # grid key -> ibm.Grid (resident)
        self.last_use = {}                               # grid key -> admission counter

    @staticmethod
    def grid_bytes(g):
        return int(g.ws.numel()) if g.ws is not None else 0

    def resident_bytes(self):
        return sum(self.grid_bytes(g) for g in self.grids.values())

    def evict(self, key):
        g = self.grids.pop(key)
        self.last_use.pop(key, None)
        g.close()

    def close(self):
        for g in self.grids.values():
            g.close()
        self.grids.clear()
        self.last_use.clear()


class Server:
    """Serve a trace of projection requests with ``slots`` concurrent workers."""

    def __init__(self, slots: int = 4, budget_bytes: int = 64 << 30, precision: str = "mixed",
                 method: str = "bicgstab", rel_tol: float = 1e-10, dt: float = 1.0,
                 device: str = "cuda:0", keep_results: bool = False, poison: bool = False):
        import torch
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.method = method
        self.rel_tol = rel_tol
        self.dt = dt
        self.budget = int(budget_bytes)
        self.keep = keep_results
        self.poison = poison                             # debug: NaN-filled workspaces (ibm_debug_poison)
        ibm.lib()                                        # load once, before any worker starts
        self.slots = [_Slot(i, self.device) for i in range(slots)]

    def close(self):
        self.torch.cuda.synchronize(self.device)
        for s in self.slots:
            s.close()

    def resident_bytes(self):
        return sum(s.resident_bytes() for s in self.slots)

    # -- one request on one slot -------------------------------------------------------
    def _velocity(self, req: Request):
        """Synthetic face velocities generated on the device (seeded, on the slot's
        stream): i.i.d. U[-1, 1] on interior faces, zero on the walls."""
        torch = self.torch
        nz, ny, nx = req.shape
        gen = torch.Generator(device=self.device)
        gen.manual_seed(int(req.vel_seed))
        out = []
        for shp in ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)):
            a = torch.rand(shp, generator=gen, dtype=torch.float64, device=self.device)
            out.append(a.mul_(2.0).sub_(1.0))
        u, v, w = out
        u[:, :, 0] = 0.0
        u[:, :, -1] = 0.0
        v[:, 0, :] = 0.0
        v[:, -1, :] = 0.0
        w[0] = 0.0
        w[-1] = 0.0
        if nz == 1:
            w.zero_()
        return u, v, w

    def _run_one(self, slot: _Slot, req: Request, on_setup):
        """Set up and project one request on the slot's stream.  on_setup(ws_bytes) is called
        once the request's grid holds its workspace (before the projection)."""
        torch = self.torch
        with torch.cuda.device(self.device), torch.cuda.stream(slot.stream):
            key = req.grid_key()
            g = slot.grids.get(key)
            if g is None:
                g = ibm.Grid(req.xf, req.yf, req.zf, precision=self.precision, device=str(self.device),
                             stream=slot.stream, poison=self.poison)
                slot.grids[key] = g
            counts = g.setup(req.verts, req.tris)
            on_setup(_Slot.grid_bytes(g))
            u, v, w = self._velocity(req)
            p = torch.empty(req.shape, dtype=torch.float64, device=self.device)
            _, st = g.project(u, v, w, dt=self.dt, p=p, rel_tol=self.rel_tol, precision=self.precision,
                              method=self.method)
            slot.stream.synchronize()
            res = (counts, st, (p.cpu().numpy(), u.cpu().numpy()) if self.keep else None)
            del u, v, w, p
            return res

    # -- the serving loop ----------------------------------------------------------------
    def run(self, trace: list[Request], log_events: bool = False):
        """Serve ``trace`` (arrival times relative to the start) and return the results in
        request order, plus the makespan in seconds.  With log_events the server keeps, in
        ``self.events``, the accounted device bytes (resident workspaces + in flight) right
        after every admission and every workspace change, for the budget check."""
        cv = threading.Condition()
        pending: list[Request] = []
        queues = {s.index: [] for s in self.slots}
        free = [s.index for s in self.slots]
        # accounting (under cv): resident workspace bytes per (slot, grid) and the bytes each
        # request in flight holds beyond them
        resident = {(s.index, k): _Slot.grid_bytes(g) for s in self.slots for k, g in s.grids.items()}
        inflight: dict[int, int] = {}
        state = {"remaining": len(trace), "tick": 0}
        results: dict[int, Result] = {}
        self.events = []
        fields = {q.rid: field_bytes(q) for q in trace}
        bound = {q.rid: workspace_bound(q, self.precision) for q in trace}
        for q in trace:
            if fields[q.rid] + bound[q.rid] > self.budget:
                raise ValueError("request %d needs %d bytes, more than the budget %d"
                                 % (q.rid, fields[q.rid] + bound[q.rid], self.budget))
        t0 = time.perf_counter()

        def total_locked():
            return sum(resident.values()) + sum(inflight.values())

        def note_locked(what):
            if log_events:
                self.events.append((what, total_locked(), sum(resident.values()), sum(inflight.values())))

        def need_locked(q, si):
            key = q.grid_key()
            cached = resident.get((si, key))
            ws = bound[q.rid] if cached is None else max(0, bound[q.rid] - cached)
            return fields[q.rid], ws

        def admit_locked():
            while pending and free:
                q = pending[0]
                key = q.grid_key()
                # a free slot that already holds this grid, else the first free slot
                si = next((i for i in free if (i, key) in resident), free[0])
                f, ws = need_locked(q, si)
                # release least recently used grids of idle slots until the request fits
                while total_locked() + f + ws > self.budget:
                    cand = [(self.slots[i].last_use.get(k, -1), i, k) for (i, k) in resident
                            if i in free and not (i == si and k == key)]
                    if not cand:
                        break
                    _, i, k = min(cand, key=lambda c: c[0])
                    self.slots[i].evict(k)
                    del resident[(i, k)]
                    note_locked("evict")
                if total_locked() + f + ws > self.budget:
                    return  # wait for a request to finish
                pending.pop(0)
                free.remove(si)
                inflight[q.rid] = f + ws
                state["tick"] += 1
                self.slots[si].last_use[key] = state["tick"]
                queues[si].append((q, time.perf_counter() - t0))
                note_locked("admit")
                cv.notify_all()

        def worker(slot: _Slot):
            while True:
                with cv:
                    while not queues[slot.index] and state["remaining"] > 0:
                        cv.wait()
                    if not queues[slot.index] and state["remaining"] == 0:
                        return
                    q, t_adm = queues[slot.index].pop(0)
                key = q.grid_key()

                def on_setup(ws_bytes, q=q, key=key):
                    # the grid's workspace now counts as resident (its actual size, also after
                    # a rebind to a larger ghost capacity); the request keeps its fields
                    with cv:
                        resident[(slot.index, key)] = ws_bytes
                        inflight[q.rid] = fields[q.rid]
                        note_locked("setup")

                err, code = "", 0
                try:
                    counts, st, kept = self._run_one(slot, q, on_setup)
                except Exception as e:             # a failed request is isolated
                    code = getattr(e, "code", ibm.IBM_E_DEVICE)
                    err = "%s: %s" % (type(e).__name__, e)
                    counts, st, kept = (0, 0, 0), None, None
                    try:                               # nothing of the failed request left in flight
                        slot.stream.synchronize()
                    except Exception:
                        pass
                    with cv:
                        if key in slot.grids:    # its state is unknown: drop the handle
                            slot.evict(key)
                        resident.pop((slot.index, key), None)
                t_done = time.perf_counter() - t0
                if st is not None:
                    r = Result(q.rid, q.name, q.arrival, t_adm, t_done, slot.index, st.status, st.cycles,
                               st.rel_residual, st.div_max, tuple(int(c) for c in counts))
                else:
                    r = Result(q.rid, q.name, q.arrival, t_adm, t_done, slot.index, int(code), 0, float("nan"),
                               float("nan"), tuple(counts), error=err)
                if kept is not None:
                    r.p, r.u = kept
                with cv:
                    results[q.rid] = r
                    inflight.pop(q.rid, None)
                    state["remaining"] -= 1
                    free.append(slot.index)
                    note_locked("done")
                    admit_locked()
                    cv.notify_all()

        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in self.slots]
        for th in threads:
            th.start()
        order = sorted(trace, key=lambda q: (q.arrival, q.rid))
        for q in order:
            delay = q.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            with cv:
                pending.append(q)
                admit_locked()
        with cv:
            while state["remaining"] > 0:
                cv.wait(timeout=1.0)
            cv.notify_all()
        for th in threads:
            th.join()
        makespan = max(r.done for r in results.values()) if results else 0.0
        return [results[q.rid] for q in trace], makespan


def summarize(results: list[Result], makespan: float) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    out = {"requests": len(results), "solves_per_s": round(len(results) / makespan, 3) if makespan > 0 else None,
           "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3), "makespan_s": round(makespan, 3),
           "all_converged": all(r.status == 0 for r in results),
           "failed": sum(1 for r in results if r.status < 0)}
    errs = [r.error for r in results if r.error]
    if errs:
        out["errors"] = errs[:4]
    return out
