"""Seeded job streams for the serving workload (problem data only).

Jobs arrive as a Poisson process; each is a heat, wave or Schroedinger
time-stepping problem (40/40/20) on a seeded star (heat, wave) or ellipse
(Schroedinger) domain, on a grid drawn uniformly from the given powers of
two, for a number of steps drawn uniformly from a range (heat: tau = h,
wave: tau = 4h, Schroedinger: tau = h/2).  The data of a job
are the manufactured solutions of `manufactured`: heat and wave use the exact
solutions of the heat and wave workloads, Schroedinger the Gaussian packet in
the harmonic potential with g = 0 on the boundary.  Every field here is a
fixed spatial array times a scalar function of time, so a job's per-step
boundary data and sources are produced by scaling arrays computed once.
"""

import numpy as np

from . import manufactured as mf
from .domains import ellipse, grid_coords, star

KINDS = ("heat", "wave", "schrodinger")


def job_stream(seed, n_jobs, rate, grids=(256, 512, 1024, 2048), steps=(50, 500), mix=(0.4, 0.4, 0.2)):
    """n_jobs job specs with Poisson arrivals of the given rate (jobs per
    unit time; arrival times in the same unit)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for i in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        kind = KINDS[int(rng.choice(3, p=np.asarray(mix, dtype=np.float64)))]
        M = int(grids[int(rng.integers(len(grids)))])
        n_steps = int(rng.integers(steps[0], steps[1] + 1))
        if kind == "schrodinger":
            a, b = rng.uniform(0.3, 0.7, 2)
            desc = ellipse(a, b, 1.0, M, M)
            tau = (2.0 / M) / 2.0
        else:
            r0 = rng.uniform(0.3, 0.6)
            lobes = int(rng.integers(3, 9))
            desc = star(r0, 0.2 * r0, lobes, 1.0, M, M)
            # heat: tau = h; wave: tau = 4h, where the theta = 1/4 steps stay
            # accurate over hundreds of steps (at tau = h they grow)
            tau = (2.0 / M) * (4.0 if kind == "wave" else 1.0)
        jobs.append({"id": i, "arrival": float(t), "kind": kind, "desc": desc, "steps": n_steps, "tau": tau})
    return jobs


def job_fields(spec, zx, zy):
    """Initial data and boundary data of a job at the grid nodes and at the
    collocation points (zx, zy) of its domain.

    Returns a dict with
      init: the arrays of the stepper's init call (u, lap u on the grid and on
            Gamma at t = 0; for wave also at t = -tau), flattened grids;
      g0, gfac: g on Gamma at time t is gfac(t) * g0;
      s0, s0g, sfac: heat sources s(t0) + s(t1) = sfac(t0, t1) * (s0, s0g),
            None for the other equations;
      v, vg: the potential on the grid and on Gamma (Schroedinger), else None.
    """
    M = spec["desc"]["M"]
    x = grid_coords(1.0, M)
    X, Y = np.meshgrid(x, x)
    kind, tau = spec["kind"], spec["tau"]
    out = {"s0": None, "s0g": None, "sfac": None, "v": None, "vg": None}
    if kind == "heat":
        out["init"] = [mf.heat_u(X, Y, 0).ravel(), mf.heat_lap(X, Y, 0).ravel(), mf.heat_u(zx, zy, 0),
                       mf.heat_lap(zx, zy, 0)]
        out["g0"], out["gfac"] = mf.heat_u(zx, zy, 0), lambda t: np.exp(-t)
        out["s0"], out["s0g"] = mf.heat_src(X, Y, 0).ravel(), mf.heat_src(zx, zy, 0)
        out["sfac"] = lambda t0, t1: np.exp(-t0) + np.exp(-t1)
    elif kind == "wave":
        out["init"] = [mf.wave_u(X, Y, 0).ravel(), mf.wave_lap(X, Y, 0).ravel(), mf.wave_u(zx, zy, 0),
                       mf.wave_lap(zx, zy, 0), mf.wave_u(X, Y, -tau).ravel(), mf.wave_lap(X, Y, -tau).ravel(),
                       mf.wave_u(zx, zy, -tau), mf.wave_lap(zx, zy, -tau)]
        out["g0"], out["gfac"] = mf.wave_u(zx, zy, 0), lambda t: np.cos(mf.SQRT2 * mf.PI * t)
    else:
        out["init"] = [mf.packet_u0(X, Y).ravel(), mf.packet_lap(X, Y).ravel(), mf.packet_u0(zx, zy),
                       mf.packet_lap(zx, zy)]
        out["g0"], out["gfac"] = np.zeros(len(zx), dtype=np.complex128), lambda t: 0.0
        out["v"], out["vg"] = mf.harmonic_potential(X, Y).ravel(), mf.harmonic_potential(zx, zy)
    return out
