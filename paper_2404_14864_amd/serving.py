"""Serving loop: continuous batching of time-stepping jobs.

Each job is one heat, wave or Schroedinger stepper on its own domain, with
its state resident on the device from admission to completion.  Jobs arrive
over wall time (Poisson arrivals of `workloads.serving`) and are served by

  * the admission loop (the calling thread): arrivals join a FIFO queue;
    the head of the queue is admitted as soon as the admitted jobs' device
    footprints (domain with every table it allocates on first use, stepper
    state, output grid, as the library reports them) leave room for it in
    the budget; a job that cannot fit even alone is rejected;
  * lanes, threads that each own a HIP stream and step their jobs in
    rounds: every round advances each of the lane's admitted jobs by one
    step in one kfbi_batch_step call, whose launches run all of them
    together.  There is one lane per class of jobs with the same scalar
    type (real: heat and wave; complex: Schroedinger) and grid size, made
    when the first job of the class is admitted, so a round never waits for
    a larger grid's solves.  Between rounds a lane takes in the jobs
    admitted meanwhile and retires the ones whose last step has completed
    on the device, which frees their memory for the admission loop.

The lanes never wait for each other or for admission: a job that arrives
while lanes have work on the device is admitted at once if memory allows
and joins its lane's next round, and the lanes' streams run concurrently on
the device.  Every step is asynchronous (the host returns
once GMRES has finished on the device, the final grid solve still queued),
so a lane enqueues its next round while the previous one completes.  A
round is timed by HIP events on the lane's stream; the step latency of a
job is the device time of the round that advanced it, read once the run is
over.  Only control scalars cross to the host inside a round.

A job's data come from a fields provider (workloads.serving.job_fields):
initial arrays and boundary data that are fixed arrays times scalar time
factors, placed on the device once, on the job's lane stream.
"""

import itertools
import threading
import time

import numpy as np
import torch

from . import kfbi

DEV = "cuda:0"


def _dev(a):
    a = np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        return torch.from_numpy(a.astype(np.complex128)).to(DEV)
    return torch.from_numpy(a.astype(np.float64)).to(DEV)


class Job:
    """One admitted job: domain, stepper, device-resident data and output.
    The domain and every upload use the current torch stream of the
    creating thread (a lane's stream when the server creates it)."""

    _serial = itertools.count()

    def __init__(self, spec, fields_fn, precision=kfbi.KFBI_PREC_FP64):
        self.serial = next(Job._serial)  # unique for the process (id() is reused after a job is freed)
        self.spec = spec
        self.kind = spec["kind"]
        self.cplx = self.kind == "schrodinger"
        desc = spec["desc"]
        self.M, self.Nb, self.tau = desc["M"], desc["Nb"], spec["tau"]
        self.steps = spec["steps"]
        self.n = 0
        self.h = kfbi.kfbi_domain_create(desc, kfbi.KFBI_COMPLEX if self.cplx else kfbi.KFBI_REAL, precision)
        self.s = None
        try:
            zx, zy = kfbi.kfbi_domain_copy_boundary(self.h)
            f = fields_fn(spec, zx, zy)
            self.gfac, self.sfac = f["gfac"], f["sfac"]
            self.g0 = _dev(f["g0"].astype(np.complex128) if self.cplx else f["g0"])
            self.s0 = _dev(f["s0"]) if f["s0"] is not None else None
            self.s0g = _dev(f["s0g"]) if f["s0g"] is not None else None
            if self.kind == "heat":
                self.s = kfbi.kfbi_stepper_create(self.h, kfbi.KFBI_HEAT, self.tau)
            elif self.kind == "wave":
                self.s = kfbi.kfbi_stepper_create(self.h, kfbi.KFBI_WAVE, self.tau, theta=0.25)
            else:
                self.v, self.vg = _dev(f["v"]), _dev(f["vg"])
                self.s = kfbi.kfbi_stepper_create(self.h, kfbi.KFBI_SCHRODINGER, self.tau, v_grid=self.v,
                                                  v_gamma=self.vg)
            kfbi.kfbi_stepper_init(self.s, *[_dev(a) for a in f["init"]])
            dt = torch.complex128 if self.cplx else torch.float64
            self.u = torch.zeros((self.M + 1) ** 2, dtype=dt, device=DEV)
            self.footprint = (kfbi.kfbi_domain_get_info(self.h)["device_bytes_max"]
                              + kfbi.kfbi_stepper_state_bytes(self.s) + self.u.numel() * self.u.element_size())
        except Exception:
            self.close()
            raise

    def inputs(self):
        """g on Gamma at the next time and (heat) the step's sources."""
        t0, t1 = self.n * self.tau, (self.n + 1) * self.tau
        g = self.g0 * float(self.gfac(t1))
        if self.sfac is None:
            return g, None, None
        c = float(self.sfac(t0, t1))
        return g, self.s0 * c, self.s0g * c

    def step_alone(self, opts=None):
        g, sg, sgg = self.inputs()
        if self.kind == "heat":
            st = kfbi.kfbi_step_heat(self.s, g, sg, sgg, self.u, opts=opts)
        elif self.kind == "wave":
            st = kfbi.kfbi_step_wave(self.s, g, self.u, opts=opts)
        else:
            st = kfbi.kfbi_step_schrodinger(self.s, g, self.u, opts=opts)
        self.n += 1
        return st

    @property
    def done(self):
        return self.n >= self.steps

    def close(self):
        if self.s is not None:
            kfbi.kfbi_stepper_destroy(self.s)
            self.s = None
        if self.h is not None:
            kfbi.kfbi_domain_destroy(self.h)
            self.h = None


class _Lane(threading.Thread):
    """Steps its jobs in rounds on its own stream (see the module text)."""

    def __init__(self, server, key):
        super().__init__(daemon=True)
        self.srv = server
        self.key = key
        self.stream = torch.cuda.Stream(device=DEV)
        self.incoming = []          # admitted, not yet stepped (guarded by srv.cond)
        self.jobs = []              # stepping
        self.retiring = []          # (job, event of its last round)
        self.rounds = []            # (ev0, ev1, [(job kind, M, iters)])
        self.busy = False           # a round is on the device (guarded by srv.cond)
        self.batch, self.batch_ids = None, None
        self.error = None

    def _rebuild_batch(self):
        ids = [j.serial for j in self.jobs]
        if ids == self.batch_ids:
            return
        if self.batch is not None:
            kfbi.kfbi_batch_destroy(self.batch)
            self.batch = None
        self.batch_ids = ids
        if self.jobs:
            self.batch = kfbi.kfbi_batch_create([j.h for j in self.jobs])

    def _round(self):
        srv = self.srv
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        opts = dict(srv.opts or {}, **{"async": True})
        self._rebuild_batch()
        ins = [j.inputs() for j in self.jobs]
        st = kfbi.kfbi_batch_step(self.batch, [j.s for j in self.jobs], [x[0] for x in ins],
                                  [j.u for j in self.jobs], src_grid=[x[1] for x in ins],
                                  src_gamma=[x[2] for x in ins], opts=opts)
        for j in self.jobs:
            j.n += 1
        ev1.record(self.stream)
        self.rounds.append((ev0, ev1, [(j.kind, j.M, s["iters"], s["converged"]) for j, s in zip(self.jobs, st)]))
        for j in [j for j in self.jobs if j.done]:
            self.jobs.remove(j)
            self.retiring.append((j, ev1))

    def _retire(self, wait=False):
        srv = self.srv
        keep = []
        for j, ev in self.retiring:
            if wait:
                ev.synchronize()
            if not ev.query():
                keep.append((j, ev))
                continue
            if srv.keep_output is not None:
                srv.keep_output(j)
            j.close()
            with srv.cond:
                srv.used -= j.footprint
                srv.finished.append(j.spec["id"])
                srv.cond.notify_all()
        self.retiring = keep

    def run(self):
        srv = self.srv
        try:
            with torch.cuda.stream(self.stream):
                while True:
                    with srv.cond:
                        while not self.incoming and not self.jobs and not self.retiring and not srv.closing:
                            srv.cond.wait(0.05)
                        self.jobs += self.incoming
                        self.incoming = []
                        if not self.jobs and not self.retiring and srv.closing:
                            break
                        self.busy = bool(self.jobs)
                    if self.jobs:
                        self._round()
                    self._retire(wait=not self.jobs)
                    with srv.cond:
                        self.busy = False
                if self.batch is not None:
                    kfbi.kfbi_batch_destroy(self.batch)
                    self.batch = None
                self.stream.synchronize()
        except BaseException as e:  # reported by Server.run
            self.error = e
            with srv.cond:
                srv.closing = True
                srv.cond.notify_all()


class Server:
    """Continuous batching of time-stepping jobs (see the module text).

    budget_bytes: device memory the admitted jobs may hold together.
    fields_fn: the job data provider.  opts: solver options of every step
    (precision: the FP64 or mixed grid solve of every job).
    keep_output: called as keep_output(job) when a job's last step has
    completed, before its memory is freed (e.g. to copy its final grid; it
    runs on the job's lane, whose stream is then current).
    """

    def __init__(self, budget_bytes, fields_fn, opts=None, keep_output=None):
        self.budget = int(budget_bytes)
        self.fields_fn = fields_fn
        self.opts = opts
        self.keep_output = keep_output
        self.cond = threading.Condition()
        self.used = 0
        self.max_used = 0
        self.max_jobs = 0
        self.finished = []
        self.closing = False

    def run(self, specs, tick=1.0):
        """Serve the jobs of `specs`, whose arrival times are in units of
        `tick` seconds of wall time, to completion.  Returns a report: step
        latencies (ms, device time of the round that advanced the job)
        overall and per (kind, M), throughput in grid-pts*GMRES-iters/s over
        the wall time from the first arrival to the last completion, the
        peak footprint, job counts, and how many admissions happened while a
        lane had a round on the device."""
        pending = sorted(specs, key=lambda s: s["arrival"])
        queue, rejected = [], []
        cache = {}  # footprint of a job shape, once one has been created
        self.used, self.max_used, self.max_jobs = 0, 0, 0
        self.finished, self.closing = [], False
        lanes = {}  # (complex?, M) -> lane; read by the lanes under self.cond
        prec = (self.opts or {}).get("precision", kfbi.KFBI_PREC_FP64)
        admitted_busy = 0
        self.lanes = lanes
        t0 = time.perf_counter()
        try:
            while pending or queue:
                now = (time.perf_counter() - t0) / tick
                while pending and pending[0]["arrival"] <= now:
                    queue.append(pending.pop(0))
                admitted = False
                while queue:
                    spec = queue[0]
                    key = (spec["kind"], spec["desc"]["M"], spec["desc"]["Nb"])
                    need = cache.get(key)
                    with self.cond:
                        used = self.used
                    if need is not None and need <= self.budget and used + need > self.budget:
                        break
                    lkey = (spec["kind"] == "schrodinger", spec["desc"]["M"])
                    lane = lanes.get(lkey)
                    if lane is None:
                        lane = _Lane(self, lkey)
                        with self.cond:
                            lanes[lkey] = lane
                        lane.start()
                    with torch.cuda.stream(lane.stream):
                        job = Job(spec, self.fields_fn, prec)
                    cache[key] = job.footprint
                    if job.footprint > self.budget:
                        job.close()
                        rejected.append(queue.pop(0)["id"])
                        continue
                    with self.cond:
                        if self.used + job.footprint > self.budget:
                            fits = False
                        else:
                            fits = True
                            busy = any(ln.busy for ln in lanes.values() if ln is not lane) or lane.busy
                            admitted_busy += 1 if busy else 0
                            lane.incoming.append(job)
                            self.used += job.footprint
                            self.max_used = max(self.max_used, self.used)
                            n_act = sum(len(ln.jobs) + len(ln.incoming) + len(ln.retiring) for ln in lanes.values())
                            self.max_jobs = max(self.max_jobs, n_act)
                            self.cond.notify_all()
                    if not fits:
                        job.close()
                        break
                    queue.pop(0)
                    admitted = True
                if any(ln.error is not None for ln in lanes.values()):
                    break
                if not admitted:
                    # wait for the next arrival or for memory to free up
                    wait = 0.05 if not pending else max(0.0, pending[0]["arrival"] * tick - (time.perf_counter() - t0))
                    with self.cond:
                        self.cond.wait(min(wait, 0.05) if queue else min(wait, 0.5))
        finally:
            with self.cond:
                self.closing = True
                self.cond.notify_all()
            for ln in lanes.values():
                ln.join()
        wall = time.perf_counter() - t0
        for ln in lanes.values():
            if ln.error is not None:
                raise ln.error
        torch.cuda.synchronize()
        lat, lat_by, work, dev_ms, unconv = [], {}, 0.0, 0.0, 0
        for ln in lanes.values():
            for ev0, ev1, steps in ln.rounds:
                ms = ev0.elapsed_time(ev1)
                dev_ms += ms
                for kind, M, it, conv in steps:
                    unconv += 0 if conv else 1
                    lat.append(ms)
                    lat_by.setdefault("%s M=%d" % (kind, M), []).append(ms)
                    work += float((M - 1) ** 2) * it
        lat = np.asarray(lat)
        first = min((s["arrival"] for s in specs), default=0.0) * tick
        return {
            "lanes": len(lanes),
            "finished": list(self.finished),
            "rejected": rejected,
            "steps": int(lat.size),
            "unconverged_steps": unconv,
            "rounds": sum(len(ln.rounds) for ln in lanes.values()),
            "p50_step_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_step_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "p50_by_type_ms": {k: float(np.percentile(v, 50)) for k, v in sorted(lat_by.items())},
            "p99_by_type_ms": {k: float(np.percentile(v, 99)) for k, v in sorted(lat_by.items())},
            "throughput": work / max(wall - first, 1e-9),
            "unit": "grid-pts*GMRES-iters/s",
            "work": work,
            "wall_s": wall,
            "device_s_sum_of_lanes": dev_ms * 1e-3,
            "max_used_bytes": self.max_used,
            "budget_bytes": self.budget,
            "max_concurrent_jobs": self.max_jobs,
            "admitted_while_device_busy": admitted_busy,
        }


def serve_plain(specs, fields_fn, opts=None, keep_output=None):
    """The plain per-solve path on the same jobs: each job alone, in arrival
    order, one synchronous step after another.  Returns its per-step
    latencies (device time of the step), throughput over the wall time and
    the work done."""
    lat, lat_by, work = [], {}, 0.0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    for spec in sorted(specs, key=lambda s: s["arrival"]):
        j = Job(spec, fields_fn)
        try:
            for _ in range(j.steps):
                ev0.record()
                st = j.step_alone(opts)
                ev1.record()
                ev1.synchronize()
                ms = ev0.elapsed_time(ev1)
                lat.append(ms)
                lat_by.setdefault("%s M=%d" % (j.kind, j.M), []).append(ms)
                work += float((j.M - 1) ** 2) * st["iters"]
            if keep_output is not None:
                keep_output(j)
        finally:
            j.close()
    wall = time.perf_counter() - t0
    lat = np.asarray(lat)
    return {"steps": int(lat.size), "p50_step_ms": float(np.percentile(lat, 50)),
            "p99_step_ms": float(np.percentile(lat, 99)),
            "p50_by_type_ms": {k: float(np.percentile(v, 50)) for k, v in sorted(lat_by.items())},
            "throughput": work / wall, "unit": "grid-pts*GMRES-iters/s", "work": work, "wall_s": wall}
