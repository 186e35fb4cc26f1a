"""Serving loop: time-stepping jobs admitted by device footprint and advanced
together.

Each job is one heat, wave or Schroedinger stepper on its own domain, with
its state resident on the device from admission to completion.  Every tick
  1. jobs that have arrived join a FIFO queue;
  2. queued jobs are admitted in order while the sum of the admitted jobs'
     device footprints (domain, stepper state and output grid, as the
     library reports them) stays within the budget; a job that cannot fit
     even alone is rejected;
  3. every admitted job advances one step: the real (heat and wave) jobs in
     one kfbi_batch_step call, whose launches run all of them together, and
     the complex (Schroedinger) jobs one kfbi_step_schrodinger call each;
  4. finished jobs free their memory.
The device time of each tick's steps (HIP events on the stream) is the step
latency of every job that stepped in it.  Only control scalars cross to the
host inside a tick.

A job's data come from a fields provider (see workloads.serving.job_fields):
initial arrays and boundary data that are fixed arrays times scalar time
factors, placed on the device once.
"""

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
    """One admitted job: domain, stepper, device-resident data and output."""

    def __init__(self, spec, fields_fn):
        self.spec = spec
        self.kind = spec["kind"]
        self.cplx = self.kind == "schrodinger"
        desc = spec["desc"]
        self.M, self.Nb, self.tau = desc["M"], desc["Nb"], spec["tau"]
        self.steps = spec["steps"]
        self.n = 0
        self.h = kfbi.kfbi_domain_create(desc, kfbi.KFBI_COMPLEX if self.cplx else kfbi.KFBI_REAL)
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
            # the domain's peak (tables allocated on first use included), the
            # stepper's state and the output grid
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


class Server:
    """Admission by footprint and batched stepping of the admitted jobs.

    budget_bytes: device memory the admitted jobs may hold together.
    fields_fn: the job data provider.  opts: solver options of every step.
    keep_output: called as keep_output(job) when a job finishes (before its
    memory is freed), e.g. to copy its final grid.
    """

    def __init__(self, budget_bytes, fields_fn, opts=None, keep_output=None):
        self.budget = int(budget_bytes)
        self.fields_fn = fields_fn
        self.opts = opts
        self.keep_output = keep_output
        self.used = 0
        self.max_used = 0
        self.max_jobs = 0
        self.batch = None
        self.batch_members = None

    def _rebuild_batch(self, real):
        ids = [id(j) for j in real]
        if ids == self.batch_members:
            return
        if self.batch is not None:
            kfbi.kfbi_batch_destroy(self.batch)
            self.batch = None
        self.batch_members = ids
        if real:
            self.batch = kfbi.kfbi_batch_create([j.h for j in real])

    def run(self, specs, tick=1.0, max_ticks=100000):
        """Serve the jobs of `specs` (arrival times in units of `tick`) to
        completion.  Returns a report: step latencies (ms) overall and per
        (kind, M), throughput in grid-pts*GMRES-iters/s over the steps'
        device time, the peak footprint and job counts."""
        pending = sorted(specs, key=lambda s: s["arrival"])
        queue, active = [], []
        lat, lat_by, rejected, finished = [], {}, [], []
        work = 0.0
        dev_ms = 0.0
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cache = {}  # footprint of a job shape, once one has been created
        t_wall = time.perf_counter()
        k = 0
        try:
            while (pending or queue or active) and k < max_ticks:
                now = k * tick
                while pending and pending[0]["arrival"] <= now:
                    queue.append(pending.pop(0))
                # admission, in arrival order
                while queue:
                    spec = queue[0]
                    key = (spec["kind"], spec["desc"]["M"], spec["desc"]["Nb"])
                    need = cache.get(key)  # footprint of an earlier job of this shape
                    if need is not None and need <= self.budget and self.used + need > self.budget:
                        break
                    job = Job(spec, self.fields_fn)
                    cache[key] = job.footprint
                    if job.footprint > self.budget:
                        job.close()
                        rejected.append(queue.pop(0)["id"])
                        continue
                    if self.used + job.footprint > self.budget:
                        job.close()
                        break
                    queue.pop(0)
                    active.append(job)
                    self.used += job.footprint
                self.max_used = max(self.max_used, self.used)
                self.max_jobs = max(self.max_jobs, len(active))
                if not active:
                    k += 1
                    continue
                # one step of every admitted job
                real = [j for j in active if not j.cplx]
                self._rebuild_batch(real)
                ev0.record()
                stats = []
                if real:
                    ins = [j.inputs() for j in real]
                    st = kfbi.kfbi_batch_step(self.batch, [j.s for j in real], [x[0] for x in ins],
                                              [j.u for j in real], src_grid=[x[1] for x in ins],
                                              src_gamma=[x[2] for x in ins], opts=self.opts)
                    for j in real:
                        j.n += 1
                    stats += list(zip(real, st))
                for j in active:
                    if j.cplx:
                        stats.append((j, j.step_alone(self.opts)))
                ev1.record()
                ev1.synchronize()
                ms = ev0.elapsed_time(ev1)
                dev_ms += ms
                for j, st in stats:
                    lat.append(ms)
                    lat_by.setdefault("%s M=%d" % (j.kind, j.M), []).append(ms)
                    work += float((j.M - 1) ** 2) * st["iters"]
                # completions free their memory
                for j in [j for j in active if j.done]:
                    if self.keep_output is not None:
                        self.keep_output(j)
                    finished.append(j.spec["id"])
                    active.remove(j)
                    self.used -= j.footprint
                    j.close()
                k += 1
        finally:
            if self.batch is not None:
                kfbi.kfbi_batch_destroy(self.batch)
                self.batch = None
                self.batch_members = None
            for j in active:
                j.close()
        lat = np.asarray(lat)
        return {
            "ticks": k,
            "finished": finished,
            "rejected": rejected,
            "steps": int(lat.size),
            "p50_step_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_step_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "p50_by_type_ms": {key: float(np.percentile(v, 50)) for key, v in sorted(lat_by.items())},
            "throughput": work / (dev_ms * 1e-3) if dev_ms > 0 else 0.0,
            "unit": "grid-pts*GMRES-iters/s",
            "device_s": dev_ms * 1e-3,
            "wall_s": time.perf_counter() - t_wall,
            "max_used_bytes": self.max_used,
            "budget_bytes": self.budget,
            "max_concurrent_jobs": self.max_jobs,
        }
