"""Serving form: a request loop with continuous batching of IPCS runs.

Requests (mesh size, viscosity, wave number, number of steps) arrive over
time. The loop keeps the runs it has admitted resident on the GPU (mesh, CSR
patterns, matrices and fields in the run's workspace) and advances all of them
together, one IPCS step per round, with `ipcs_batch_step`: the Krylov
iterations of all runs share kernel launches. Before each round it admits the
requests that have arrived, in arrival order, while the number of runs stays
within `max_slots` and their summed HBM footprint (each run's workspace, from
`ipcs_run_workspace_bytes`) within `hbm_budget`. A run leaves as soon as its
steps are done and its workspace is released, so that waiting requests take
its place in the next round.

Lanes. A round of one batch lasts as long as its slowest run, so a small
request batched with the largest meshes would wait for them at every step.
The loop therefore serves requests in lanes, by mesh size: each lane has its
own stream and host thread and batches only its own size class, so the rounds
of small runs are not paced by the large ones, and the lanes' launches
overlap on the GPU. Admission is shared: one slot cap and one HBM budget over
all lanes, each lane admitting its own requests in arrival order. A run's
result does not depend on what it is batched with, or on the stream, so it is
the same alone and in the mix.

Reserved CUs. Lanes still share the compute units, so a small lane's short
kernels can wait behind the grids of a large lane. A lane may therefore get a
set of CUs of its own (`lane_cus`): its stream is created with a CU mask
(HIP's CU-masked streams), and the lanes without a reservation share the
remaining CUs on streams masked to those. Masks change where kernels run, not
what they compute.

Per-step latency of a request is the time between two consecutive completions
of its steps (the first is counted from its admission); the report gives
their p50 and p99, overall and per mesh size, beside the aggregate
DOF-steps/s and the queueing delays.
"""
import threading
import time
from dataclasses import dataclass, field

import numpy as np


def _hip_runtime():
    """The HIP runtime this process already uses (the one torch loaded; the
    library links the same one), for the stream calls below."""
    import ctypes
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1] if line.strip() else ""
            if "libamdhip64.so" in path:
                return ctypes.CDLL(path)
    raise RuntimeError("the HIP runtime is not loaded")


def cu_masked_stream(torch, cus):
    """A stream whose kernels run only on the compute units listed (bit c of
    the device's CU mask for each c), wrapped for torch; returns (stream,
    handle) with handle for destroy_stream."""
    import ctypes
    hip = _hip_runtime()
    total = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    words = (total + 31) // 32
    mask = (ctypes.c_uint32 * words)()
    for c in cus:
        if not 0 <= c < total:
            raise ValueError(f"CU {c} out of range (the device has {total})")
        mask[c // 32] |= 1 << (c % 32)
    h = ctypes.c_void_p()
    rc = hip.hipExtStreamCreateWithCUMask(ctypes.byref(h), ctypes.c_uint32(words), mask)
    if rc != 0:
        raise RuntimeError(f"hipExtStreamCreateWithCUMask failed ({rc})")
    return torch.cuda.ExternalStream(h.value), h.value


def destroy_stream(handle):
    import ctypes
    _hip_runtime().hipStreamDestroy(ctypes.c_void_p(handle))


@dataclass
class Request:
    id: int
    t_arrive: float          # seconds after the start of the stream
    n: int                   # unit square with n x n squares
    k: float                 # Taylor-Green wave number
    nu: float
    steps: int
    dt: float


@dataclass
class Active:
    req: Request
    run: object
    footprint: int
    t_admit: float
    done: int = 0
    t_last: float = 0.0
    lat: list = field(default_factory=list)


def admit(queue, now, active_count, active_bytes, footprint_of, max_slots, hbm_budget):
    """Admission policy: the longest prefix of the arrival-ordered queue that
    has arrived by `now` and fits both limits (head-of-line order: a request
    that does not fit blocks the ones behind it, so none is starved). Returns
    the number of requests to admit."""
    k = 0
    slots, used = active_count, active_bytes
    for req in queue:
        if req.t_arrive > now or slots >= max_slots:
            break
        f = footprint_of(req)
        if used + f > hbm_budget and slots > 0:
            break
        if f > hbm_budget:
            raise ValueError(f"request {req.id} needs {f} bytes, more than the HBM budget")
        slots += 1
        used += f
        k += 1
    return k


class Server:
    def __init__(self, dim=2, precision=None, max_slots=64, hbm_budget=200 << 30, tol=1e-12,
                 tol_ir=1e-10, stream=None, poisson_part_rows=0, lanes=None, lane_cus=None):
        """lanes: tuple of tuples of mesh sizes, one lane per tuple (each with
        its own stream and host thread); None: one lane for every size (on
        `stream` if given). lane_cus: per lane, the number of CUs reserved
        for it (consecutive mask bits, from bit 0 in lane order) or None (the
        lane shares the CUs no lane reserved); None: no masks."""
        import torch
        from paper_2605_25403_amd import ipcs as I
        if dim != 2:
            raise ValueError("the request stream uses the 2D Taylor-Green problem")
        self.I, self.torch = I, torch
        self.precision = I.IPCS_MIXED if precision is None else precision
        self.max_slots, self.hbm_budget = max_slots, hbm_budget
        self.tol, self.tol_ir = tol, tol_ir
        self.part_rows = poisson_part_rows
        self.lanes = tuple(tuple(l) for l in lanes) if lanes else None
        self.lane_cus = tuple(lane_cus) if lane_cus else None
        if self.lane_cus is not None and (self.lanes is None or
                                          len(self.lane_cus) != len(self.lanes)):
            raise ValueError("lane_cus needs one entry per lane")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self._meshes = {}
        self._owned = []
        self._lock = threading.Lock()

    def mesh(self, n):
        with self._lock:
            if n not in self._meshes:
                self._meshes[n] = self.I.Mesh.unit_square(n)
            return self._meshes[n]

    def params(self, req):
        return self.I.ipcs_params_default(nu=req.nu, dt=req.dt, precision=self.precision,
                                          tol_mom=self.tol, tol_p=self.tol, tol_corr=self.tol,
                                          tol_ir=self.tol_ir, poisson_part_rows=self.part_rows)

    def footprint(self, req):
        return self.I.ipcs_run_workspace_bytes(self.mesh(req.n).h, self.params(req))

    def start_run(self, req, stream=None):
        r = self.I.Run(self.mesh(req.n), self.params(req),
                       stream=self.stream if stream is None else stream)
        r.set_builtin(self.I.IPCS_SOL_TAYLOR_GREEN_2D, (req.k,))
        return r

    def serve(self, requests, keep_fields=False, clock=time.perf_counter, keep_ids=None):
        """Runs the whole stream; returns a report dict and the results per
        request id (with the final fields when keep_fields, or for the ids in
        keep_ids)."""
        queue = sorted(requests, key=lambda q: (q.t_arrive, q.id))
        if self.lanes is None:
            lanes = [(None, queue, self.stream)]
        else:
            sizes = {q.n for q in queue}
            missing = sizes - {n for l in self.lanes for n in l}
            if missing:
                raise ValueError(f"no lane serves mesh sizes {sorted(missing)}")
            lanes = [(l, [q for q in queue if q.n in l], st)
                     for l, st in zip(self.lanes, self._lane_streams())]
        keep = (lambda q: True) if keep_fields else (
            (lambda q: q.id in keep_ids) if keep_ids else (lambda q: False))
        shared = {"slots": 0, "bytes": 0, "max_active": 0}
        results = {}
        counters = {"dof_steps": 0, "rounds": 0, "fails": 0}
        errors = []
        t0 = clock()
        threads = [threading.Thread(target=self._lane, args=(lq, st, t0, clock, shared, results,
                                                             counters, keep, errors))
                   for _, lq, st in lanes]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        self.torch.cuda.synchronize()
        for h in self._owned:
            destroy_stream(h)
        self._owned = []
        if errors:
            raise errors[0]
        wall = clock() - t0
        done = list(results.values())
        lat = np.concatenate([np.asarray(r["lat"]) for r in done if r["lat"]])
        qd = np.array([r["t_admit"] - r["t_arrive"] for r in done])
        e2e = np.array([r["t_done"] - r["t_arrive"] for r in done if "t_done" in r])
        first = min(q.t_arrive for q in requests)
        by_n = {}
        for n in sorted({r["n"] for r in done}):
            ln = np.concatenate([np.asarray(r["lat"]) for r in done if r["n"] == n and r["lat"]])
            by_n[str(n)] = {"p50_step_ms": 1000 * float(np.percentile(ln, 50)),
                            "p99_step_ms": 1000 * float(np.percentile(ln, 99))}
        report = {
            "requests": len(requests), "failed": counters["fails"],
            "rounds": counters["rounds"], "lanes": [list(l) for l, _, _ in lanes if l] or None,
            "lane_cus": list(self.lane_cus) if self.lane_cus else None,
            "max_active": shared["max_active"], "max_slots": self.max_slots,
            "hbm_budget_bytes": self.hbm_budget,
            "dof_steps": counters["dof_steps"], "wall_s": wall,
            "dof_steps_per_s": counters["dof_steps"] / max(wall - first, 1e-9),
            "p50_step_ms": 1000 * float(np.percentile(lat, 50)),
            "p99_step_ms": 1000 * float(np.percentile(lat, 99)),
            "step_ms_by_n": by_n,
            "queue_delay_p50_ms": 1000 * float(np.percentile(qd, 50)),
            "queue_delay_p99_ms": 1000 * float(np.percentile(qd, 99)),
            # arrival to the end of the last step, completed requests
            "end_to_end_p50_ms": 1000 * float(np.percentile(e2e, 50)) if e2e.size else None,
            "end_to_end_p99_ms": 1000 * float(np.percentile(e2e, 99)) if e2e.size else None,
        }
        return report, results

    def _lane(self, queue, stream, t0, clock, shared, results, counters, keep, errors):
        """One lane: admits its own requests (arrival order, shared limits),
        steps its resident runs together on its stream, one step per round."""
        I = self.I
        active = []
        try:
            while queue or active:
                now = clock() - t0
                with self._lock:
                    k = admit(queue, now, shared["slots"], shared["bytes"], self.footprint_nolock,
                              self.max_slots, self.hbm_budget)
                    adm = queue[:k]
                    for req in adm:
                        shared["slots"] += 1
                        shared["bytes"] += self.footprint_nolock(req)
                    shared["max_active"] = max(shared["max_active"], shared["slots"])
                for req in adm:
                    run = self.start_run(req, stream)
                    ta = clock() - t0
                    active.append(Active(req, run, self.footprint(req), ta, t_last=ta))
                del queue[:k]
                if not active:
                    # nothing to do until the next arrival (or until another
                    # lane frees room)
                    wait = queue[0].t_arrive - (clock() - t0)
                    time.sleep(max(0.0005, wait) if wait > 0 else 0.0005)
                    continue
                rc, stats = I.ipcs_batch_step([a.run.h for a in active], stream.cuda_stream)
                tdone = clock() - t0
                stay, freed = [], []
                for a, st in zip(active, stats):
                    if st["status"] != I.IPCS_OK:
                        results[a.req.id] = dict(status=st["status"], t_admit=a.t_admit,
                                                 t_arrive=a.req.t_arrive, lat=a.lat, n=a.req.n)
                        freed.append(a)
                        continue
                    a.lat.append(tdone - a.t_last)
                    a.t_last = tdone
                    a.done += 1
                    if a.done == a.req.steps:
                        res = dict(status=0, t_arrive=a.req.t_arrive, t_admit=a.t_admit,
                                   t_done=tdone, lat=a.lat, n=a.req.n)
                        if keep(a.req):
                            res["U"], res["P"] = a.run.velocity(), a.run.pressure()
                        results[a.req.id] = res
                        freed.append(a)
                    else:
                        stay.append(a)
                with self._lock:
                    counters["rounds"] += 1
                    counters["dof_steps"] += sum(2 * (2 * a.req.n + 1) ** 2 + (a.req.n + 1) ** 2
                                                 for a, st in zip(active, stats)
                                                 if st["status"] == I.IPCS_OK)
                    counters["fails"] += sum(st["status"] != I.IPCS_OK for st in stats)
                    for a in freed:
                        shared["slots"] -= 1
                        shared["bytes"] -= a.footprint
                for a in freed:
                    del a.run   # releases the workspace
                active = stay
        except Exception as e:   # reported by serve() after every lane has ended
            errors.append(e)

    def _lane_streams(self):
        """One stream per lane: plain, or masked to the lane's reserved CUs
        (or to the CUs no lane reserved)."""
        self._owned = []
        if self.lane_cus is None:
            return [self.torch.cuda.Stream() for _ in self.lanes]
        total = self.torch.cuda.get_device_properties(
            self.torch.cuda.current_device()).multi_processor_count
        first, ranges = 0, []
        for c in self.lane_cus:
            ranges.append(range(first, first + c) if c else None)
            first += c or 0
        if first >= total:
            raise ValueError("the reserved CUs leave none for the other lanes")
        rest = range(first, total)
        out = []
        for r in ranges:
            st, h = cu_masked_stream(self.torch, r if r is not None else rest)
            self._owned.append(h)
            out.append(st)
        return out

    def footprint_nolock(self, req):
        n = req.n
        if n not in self._meshes:
            self._meshes[n] = self.I.Mesh.unit_square(n)
        return self.I.ipcs_run_workspace_bytes(self._meshes[n].h, self.params(req))


def requests_from(stream_spec):
    """Request objects from workloads.serving_requests dicts."""
    return [Request(id=d["id"], t_arrive=d["t_arrive"], n=d["n"], k=d["k"], nu=d["nu"],
                    steps=d["steps"], dt=d["dt"]) for d in stream_spec]
