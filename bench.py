#!/usr/bin/env python3
"""Benchmark of the KFBI time-stepping path on one MI355X.

Headline workload (the largest single-GPU time-stepping configuration):
the Schroedinger equation i u_t = lap u + v u with Strang splitting,
ellipse with semi-axes 0.6 / 0.4 in [-1,1]^2, 1024 x 1024 grid, 1024
collocation points (the paper's Nb = M of section 4; reading R4),
harmonic potential v = 50 (x^2 + y^2), Gaussian packet of width 0.1 and
momentum (20, 0), g = 0 on Gamma, tau = h/2, complex128.  One step = the
closed-form B-step and the right-hand side, the b-solve, GMRES on the
boundary integral equation (each iteration: corrections, sparse DST-x /
tridiagonal-y grid solve, stencil values and extraction, Arnoldi) and the
final grid solve.

Metric: grid-pts * GMRES-iters / s = sum over the timed steps of
(M-1)^2 * iterations, divided by their wall time (inputs resident in HBM).

Also reported: p50/p99 step latency (device time per step from HIP events
on the stepper's stream); the error of the GPU solution against the CPU
oracle after the same steps; the complex64 grid solve inside FP64
refinement on the same workload; the dominant kernel's algorithmic
bandwidth against the 8 TB/s HBM peak (launch duration from back-to-back
replay launches between two HIP events on the domain stream) and its
measured HBM traffic; the CPU oracle timed on a bounded sample of the same
workload on all host cores and on one; and, as secondary keys, the wave
workload (512 grid, FP64 and FP32 inner solves), the Richardson iteration
beside GMRES, the Neumann wave example, the batched Helmholtz workload and
the serving loop.

    python bench.py [--gpus 1] [--steps 100] [--warmup 3]
"""

import argparse
import json
import os
import platform
import sys
import time

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the kernel at its current version on the headline
# workload, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled
# by the same counters on a device copy of known size; the commands and
# counts are in profiles/*_hbm_traffic.md.  Kernels not listed (or changed
# since they were counted) report null.
TRAFFIC = {
    # Schroedinger 1024, complex128: 18.37 MB per sparse launch, 36.08 MB per
    # dense launch, weighted 80 / 20 like the algorithmic bytes of the profiled
    # steps (profiles/tridiag_schrodinger1024_c128_hbm_traffic.md)
    "k_tridiag / k_tridiag_rows": 21908926.0,
}
# the kernel each profile label belongs to: the two tridiagonal labels are
# the y-direction solves launched from one site (sparse or dense right-hand
# side); a sparse launch runs the LDS-tile or the register-row kernel, as the
# domain's launch-shape timing chose, a dense one the tile kernel
KTRI = "k_tridiag / k_tridiag_rows"
KERNEL_OF = {"tridiag_sparse": KTRI, "tridiag_dense": KTRI, "dst": "k_dst_rows",
             "idst": "k_dst_rows", "eval_nodes": "k_eval_extract / k_eval_nodes",
             "corrections": "k_corr_phi / k_corrections", "extract": "k_extract", "arnoldi": "k_gm_slot"}
REPLAYABLE = ("tridiag_sparse", "tridiag_dense", "eval_nodes", "corrections", "arnoldi")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--M", type=int, default=1024, help="grid of the headline Schroedinger workload")
    ap.add_argument("--wave-M", type=int, default=512, help="grid of the secondary wave workload")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle sample length, per core setting")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--replay", type=int, default=200)
    ap.add_argument("--no-secondary", action="store_true", help="headline workload only")
    ap.add_argument("--batch", type=int, default=256, help="instances of the batched Helmholtz run (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-jobs", type=int, default=16, help="jobs of the serving sample (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device three times (the reference transfer "
                         "for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": affinity}


# ---------------------------------------------------------------------------
# the headline workload's inputs (shared by the GPU legs and the oracle)
# ---------------------------------------------------------------------------
class Schr:
    def __init__(self, M):
        import numpy as np
        import workloads as W
        from workloads import manufactured as mf
        self.desc = W.domain_c3_schrodinger(M)
        self.M, self.Nb = M, self.desc["Nb"]
        self.h = 2.0 / M
        self.tau = self.h / 2.0
        x = W.grid_coords(1.0, M)
        self.X, self.Y = np.meshgrid(x, x)
        self.mf = mf

    def init_arrays(self, zx, zy):
        mf = self.mf
        return [mf.packet_u0(self.X, self.Y).ravel(), mf.packet_lap(self.X, self.Y).ravel(),
                mf.packet_u0(zx, zy), mf.packet_lap(zx, zy)]

    def potential(self, zx, zy):
        return self.mf.harmonic_potential(self.X, self.Y).ravel(), self.mf.harmonic_potential(zx, zy)


def oracle_schrodinger(M, seconds, max_steps, workers):
    """The oracle (numpy/scipy, unchanged) on the headline workload, timed on
    the host: as many time steps as fit in about `seconds` (at most
    max_steps), with scipy's FFTs on `workers` threads.  Returns the timing
    and the oracle's solution after its last step."""
    import numpy as np
    import scipy.fft
    from oracle.geometry import Domain
    from oracle.steppers import SchrodingerStepper
    S = Schr(M)
    od = Domain(S.desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    v, vg = S.potential(zx, zy)
    ini = S.init_arrays(zx, zy)
    st = SchrodingerStepper(od, S.tau, ini[0].reshape(M + 1, M + 1), ini[1].reshape(M + 1, M + 1), ini[2], ini[3],
                            v.reshape(M + 1, M + 1), vg)
    zero = np.zeros(od.Nb, dtype=np.complex128)
    iters, n, U, lat = 0, 0, None, []
    with scipy.fft.set_workers(workers):
        t0 = time.perf_counter()
        while n < max_steps:
            t1 = time.perf_counter()
            U = st.step(zero)
            lat.append(time.perf_counter() - t1)
            iters += st.last_stats["iters"]
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        el = time.perf_counter() - t0
    return {"value": (M - 1) ** 2 * iters / el, "steps": n, "iters": iters, "seconds": el,
            "ms_per_step": 1e3 * el / n, "p50_step_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
            "U": U, "inside": od.inside}


def cpu_baseline(M, seconds):
    """The oracle on the headline workload on all host cores and on one
    (the paper's single-CPU setting), each for about `seconds`."""
    info = cpu_info()
    # the host cores this process may use (a one-GPU share of the host: at most 16)
    cores = min(info["affinity"] or 1, 16)
    allc = oracle_schrodinger(M, seconds, 10 ** 6, cores)
    one = oracle_schrodinger(M, seconds, 10 ** 6, 1)
    sample = ("first %d time steps of the same Schroedinger workload (%d GMRES iterations) in %.1f s; "
              "numpy/scipy oracle, FFTs on %d threads" % (allc["steps"], allc["iters"], allc["seconds"], cores))
    out = {"value": allc["value"], "unit": "grid-pts*GMRES-iters/s", "cores": cores, "kind": "oracle",
           "sample": sample, "ms_per_step": allc["ms_per_step"],
           "single_core": {"value": one["value"], "cores": 1, "ms_per_step": one["ms_per_step"],
                           "sample": "first %d time steps (%d GMRES iterations) in %.1f s" % (
                               one["steps"], one["iters"], one["seconds"])}}
    out.update(info)
    return out, allc


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------
def schr_gpu(S, prec=None):
    """Domain and stepper of the headline workload on the GPU."""
    import torch
    from paper_2404_14864_amd import kfbi
    prec = kfbi.KFBI_PREC_FP64 if prec is None else prec
    dom = kfbi.kfbi_domain_create(S.desc, kfbi.KFBI_COMPLEX, prec)
    zx, zy = kfbi.kfbi_domain_copy_boundary(dom)
    c = lambda a: torch.from_numpy(a.astype("complex128")).to("cuda:0")  # noqa: E731
    r = lambda a: torch.from_numpy(a.astype("float64")).to("cuda:0")  # noqa: E731
    v, vg = S.potential(zx, zy)
    st = kfbi.kfbi_stepper_create(dom, kfbi.KFBI_SCHRODINGER, S.tau, v_grid=r(v), v_gamma=r(vg))
    init = [c(a) for a in S.init_arrays(zx, zy)]
    g0 = torch.zeros(S.Nb, dtype=torch.complex128, device="cuda:0")
    u = torch.zeros((S.M + 1) ** 2, dtype=torch.complex128, device="cuda:0")
    return dom, st, init, g0, u


def timed_steps(step, n, events):
    """n asynchronous steps; per-step device latency from events recorded on
    the current stream (the library's stream) between the calls."""
    import numpy as np
    import torch
    iters, refs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n):
        events[k].record()
        s = step(k)
        iters.append(s["iters"])
        refs.append(s["refinements"])
    events[n].record()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    lat = np.array([events[k].elapsed_time(events[k + 1]) for k in range(n)])
    return T, iters, refs, lat


def rel_inside(U, Ur, inside):
    import numpy as np
    return float(np.max(np.abs(U - Ur)[inside]) / max(np.max(np.abs(Ur[inside])), 1e-300))


def profile_dominant(dom, steps_fn, np_steps, replay):
    """Per-kernel HIP-event timing over np_steps profiled steps, replay
    durations, and the dominant kernel: the one with the largest launches x
    duration, the labels of one kernel taken together."""
    from paper_2404_14864_amd import kfbi
    import torch
    kfbi.kfbi_profile_enable(dom, True)
    steps_fn(np_steps)
    torch.cuda.synchronize()
    prof = kfbi.kfbi_profile_read(dom)
    kfbi.kfbi_profile_enable(dom, False)
    tot = sum(q["total_ms"] for q in prof.values())
    labels = {}
    for k, v in prof.items():
        if not v["launches"]:
            continue
        if k in REPLAYABLE:
            ms_k, by_k = kfbi.kfbi_profile_replay(dom, k, replay)
            how = "replay of %d back-to-back launches between two HIP events" % replay
        else:
            ms_k, by_k = v["total_ms"] / v["launches"], v["bytes"] / v["launches"]
            how = "HIP events around each launch"
        labels[k] = {"kernel": KERNEL_OF[k], "launches": v["launches"], "avg_us": 1e3 * ms_k,
                     "bytes_per_launch": by_k, "avg_us_events": 1e3 * v["total_ms"] / v["launches"],
                     "share_events": v["total_ms"] / max(tot, 1e-30), "timing": how}
    kern = {}
    for k, L in labels.items():
        g = kern.setdefault(L["kernel"], {"labels": [], "launches": 0, "time_us": 0.0, "bytes": 0.0})
        g["labels"].append(k)
        g["launches"] += L["launches"]
        g["time_us"] += L["launches"] * L["avg_us"]
        g["bytes"] += L["launches"] * L["bytes_per_launch"]
    kdom = max(kern, key=lambda q: kern[q]["time_us"])
    g = kern[kdom]
    avg_us = g["time_us"] / g["launches"]
    bytes_launch = g["bytes"] / g["launches"]
    return labels, kern, kdom, avg_us, bytes_launch


def headline(args, cpu_ref):
    import numpy as np
    import torch
    from paper_2404_14864_amd import kfbi
    S = Schr(args.M)
    dom, st, init, g0, u = schr_gpu(S)
    info = kfbi.kfbi_domain_get_info(dom)
    log("schrodinger M=%d Nb=%d inside=%d irregular=%d edges=%d" % (S.M, S.Nb, info["n_inside"],
                                                                    info["n_irregular"], info["n_edges"]))
    kfbi.kfbi_stepper_init(st, *init)
    for _ in range(args.warmup):
        kfbi.kfbi_step_schrodinger(st, g0, u)
    kfbi.kfbi_stepper_init(st, *init)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    aopts = {"async": True}
    T, iters, _, lat = timed_steps(lambda k: kfbi.kfbi_step_schrodinger(st, g0, u, opts=aopts), args.steps, ev)
    pts = (S.M - 1) ** 2
    value = pts * sum(iters) / T
    log("schrodinger fp64: %d steps in %.3f s, %d GMRES iterations, %.3g grid-pts*iters/s" % (
        args.steps, T, sum(iters), value))
    U_end = u.cpu().numpy().reshape(S.M + 1, S.M + 1)
    out = {"value": value, "T": T, "iters": iters, "lat": lat, "finite": bool(np.all(np.isfinite(U_end)))}

    # complex64 grid solves inside FP64 refinement, same steps
    mopts = {"precision": kfbi.KFBI_PREC_MIXED, "async": True}
    kfbi.kfbi_stepper_init(st, *init)
    for _ in range(args.warmup):
        kfbi.kfbi_step_schrodinger(st, g0, u, opts=mopts)
    kfbi.kfbi_stepper_init(st, *init)
    Tm, miters, mref, mlat = timed_steps(lambda k: kfbi.kfbi_step_schrodinger(st, g0, u, opts=mopts), args.steps, ev)
    Um = u.cpu().numpy().reshape(S.M + 1, S.M + 1)
    inside = (kfbi.kfbi_domain_copy_classification(dom) & 1).astype(bool)
    out["mixed"] = {"value": pts * sum(miters) / Tm, "ms_per_step": 1e3 * Tm / args.steps,
                    "p50_step_ms": float(np.percentile(mlat, 50)), "p99_step_ms": float(np.percentile(mlat, 99)),
                    "gmres_iters_per_step": float(np.mean(miters)), "refinements_per_step": float(np.mean(mref)),
                    "grid_solve": "complex64", "refinement": "fp64",
                    "rel_diff_vs_fp64_gpu_after_steps": rel_inside(Um, U_end, inside)}
    log("schrodinger mixed: %.3f ms/step, %.3g grid-pts*iters/s, %.1f refinements/step" % (
        out["mixed"]["ms_per_step"], out["mixed"]["value"], out["mixed"]["refinements_per_step"]))

    # accuracy against the oracle after the steps its timed sample ran
    if cpu_ref is not None:
        nacc = cpu_ref["steps"]
        acc = {"vs": "CPU FP64 oracle (same inputs, GMRES tol 1e-10 on both sides)", "steps": nacc}
        for label, o in (("fp64", {}), ("mixed", {"precision": kfbi.KFBI_PREC_MIXED})):
            kfbi.kfbi_stepper_init(st, *init)
            for _ in range(nacc):
                kfbi.kfbi_step_schrodinger(st, g0, u, opts=o)
            acc["rel_err_" + label] = rel_inside(u.cpu().numpy().reshape(S.M + 1, S.M + 1), cpu_ref["U"],
                                                 cpu_ref["inside"])
        out["accuracy"] = acc
        log("accuracy after %d steps vs the oracle: fp64 %.2e, mixed %.2e" % (nacc, acc["rel_err_fp64"],
                                                                               acc["rel_err_mixed"]))

    # profiled pass on the same steps, replay durations, dominant kernel
    def run_steps(n):
        kfbi.kfbi_stepper_init(st, *init)
        for _ in range(n):
            kfbi.kfbi_step_schrodinger(st, g0, u)
    labels, kern, kdom, avg_us, bytes_launch = profile_dominant(dom, run_steps, args.profile_steps, args.replay)
    out["profile"] = (labels, kern, kdom, avg_us, bytes_launch)
    log("dominant kernel %s: %d launches, avg %.2f us, %.3g bytes/launch" % (kdom, kern[kdom]["launches"],
                                                                            avg_us, bytes_launch))
    out["info"] = info
    out["S"] = S
    kfbi.kfbi_stepper_destroy(st)
    kfbi.kfbi_domain_destroy(dom)
    return out


def wave_leg(args):
    """The wave workload (theta = 1/4, five-lobed star, 512 grid, Nb = M,
    tau = h, manufactured cos(sqrt2 pi t) sin(pi x) sin(pi y)) in FP64 and
    with FP32 inner solves; the Richardson iteration beside GMRES on its
    first steps; the paper's Neumann wave example at the same grid."""
    import numpy as np
    import torch
    import workloads as W
    from workloads import manufactured as mf
    from paper_2404_14864_amd import kfbi
    dev = "cuda:0"
    M = args.wave_M
    desc = W.domain_c2_wave(M)
    theta, tau = 0.25, 2.0 / M
    dom = kfbi.kfbi_domain_create(desc)
    zx, zy = kfbi.kfbi_domain_copy_boundary(dom)
    x = W.grid_coords(1.0, M)
    X, Y = np.meshgrid(x, x)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    steps = args.steps
    total = args.warmup + steps
    g_all = d(np.stack([mf.wave_u(zx, zy, (n + 1) * tau) for n in range(total)]))
    init = [d(mf.wave_u(X, Y, 0).ravel()), d(mf.wave_lap(X, Y, 0).ravel()), d(mf.wave_u(zx, zy, 0)),
            d(mf.wave_lap(zx, zy, 0)), d(mf.wave_u(X, Y, -tau).ravel()), d(mf.wave_lap(X, Y, -tau).ravel()),
            d(mf.wave_u(zx, zy, -tau)), d(mf.wave_lap(zx, zy, -tau))]
    u = torch.zeros((M + 1) * (M + 1), dtype=torch.float64, device=dev)
    st = kfbi.kfbi_stepper_create(dom, kfbi.KFBI_WAVE, tau, theta=theta)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    pts = (M - 1) ** 2
    res = {"workload": "wave theta-scheme (theta=0.25), star r=0.5+0.1sin5t in [-1,1]^2, %dx%d grid, Nb=%d, "
                       "dt=h, manufactured cos(sqrt2 pi t) sin(pi x) sin(pi y)" % (M, M, desc["Nb"]),
           "unit": "grid-pts*GMRES-iters/s", "steps": steps}
    for label, o in (("fp64", {}), ("mixed", {"precision": kfbi.KFBI_PREC_MIXED})):
        kfbi.kfbi_stepper_init(st, *init)
        for n in range(args.warmup):
            kfbi.kfbi_step_wave(st, g_all[n], u, opts=o)
        kfbi.kfbi_stepper_init(st, *init)
        T, its, refs, lat = timed_steps(lambda k: kfbi.kfbi_step_wave(st, g_all[k], u, opts=dict(o, **{"async": True})),
                                        steps, ev)
        res[label] = {"value": pts * sum(its) / T, "ms_per_step": 1e3 * T / steps,
                      "p50_step_ms": float(np.percentile(lat, 50)), "p99_step_ms": float(np.percentile(lat, 99)),
                      "gmres_iters_per_step": float(np.mean(its))}
        if label == "mixed":
            res[label]["refinements_per_step"] = float(np.mean(refs))
        log("wave %s: %.3f ms/step, %.3g grid-pts*iters/s" % (label, res[label]["ms_per_step"], res[label]["value"]))
    # the paper's Richardson iteration (eq. 3.21) beside GMRES, first steps
    rich = {}
    rsteps = min(steps, 20)
    for label, ropts in (("gmres", {}), ("richardson_gamma1", {"solver": "richardson", "gamma": 1.0}),
                         ("richardson_gamma0.9", {"solver": "richardson", "gamma": 0.9})):
        kfbi.kfbi_stepper_init(st, *init)
        its = []
        torch.cuda.synchronize()
        ev[0].record()
        for k in range(rsteps):
            its.append(kfbi.kfbi_step_wave(st, g_all[k], u, opts=dict(ropts, tol=1e-10))["iters"])
        ev[1].record()
        torch.cuda.synchronize()
        rich[label] = {"products_per_step": float(np.mean(its)), "ms_per_step": ev[0].elapsed_time(ev[1]) / rsteps}
    rich["steps"], rich["tol"] = rsteps, 1e-10
    res["solvers"] = rich
    log("solvers: " + ", ".join("%s %.1f products %.3f ms" % (k, v["products_per_step"], v["ms_per_step"])
                                for k, v in rich.items() if isinstance(v, dict)))
    kfbi.kfbi_stepper_destroy(st)
    kfbi.kfbi_domain_destroy(dom)

    # the Neumann problem (eqs. 3.19-3.20): the paper's Neumann wave example
    # (eight-lobed star, u_n = 0, a logistic bump at rest), theta = 1/4,
    # tau = 4h, at the same grid size
    nsteps = min(steps, 50)
    ndesc = W.domain_neumann_wave(M)
    ndom = kfbi.kfbi_domain_create(ndesc)
    try:
        nzx, nzy = kfbi.kfbi_domain_copy_boundary(ndom)
        xn = W.grid_coords(ndesc["L"], M)
        Xn, Yn = np.meshgrid(xn, xn)
        ntau = 4.0 * 2.0 * ndesc["L"] / M
        u0g, l0g = mf.logistic_u0(Xn, Yn), mf.logistic_lap(Xn, Yn)
        u0b, l0b = mf.logistic_u0(nzx, nzy), mf.logistic_lap(nzx, nzy)
        ninit = [d(u0g.ravel()), d(l0g.ravel()), d(u0b), d(l0b), d((u0g + 0.5 * ntau ** 2 * l0g).ravel()),
                 d(l0g.ravel()), d(u0b + 0.5 * ntau ** 2 * l0b), d(l0b)]
        nst = kfbi.kfbi_stepper_create(ndom, kfbi.KFBI_WAVE, ntau, theta=theta, bc=kfbi.KFBI_BC_NEUMANN)
        try:
            gz = d(np.zeros(ndesc["Nb"]))
            kfbi.kfbi_stepper_init(nst, *ninit)
            for k in range(args.warmup):
                kfbi.kfbi_step_wave(nst, gz, u)
            kfbi.kfbi_stepper_init(nst, *ninit)
            T, its, _, lat = timed_steps(lambda k: kfbi.kfbi_step_wave(nst, gz, u, opts={"async": True}), nsteps, ev)
            finite = bool(torch.isfinite(u).all().item())
        finally:
            kfbi.kfbi_stepper_destroy(nst)
    finally:
        kfbi.kfbi_domain_destroy(ndom)
    res["neumann"] = {"workload": "Neumann wave, star r=0.8+0.2 sin 8t in [-1.5,1.5]^2, M=%d, Nb=%d, u_n=0, "
                                  "logistic bump at rest, theta=1/4, dt=4h" % (M, ndesc["Nb"]),
                      "steps": nsteps, "ms_per_step": 1e3 * T / nsteps, "iters_per_step": float(np.mean(its)),
                      "value": pts * sum(its) / T, "unit": "grid-pts*GMRES-iters/s", "finite": finite}
    log("neumann: %d steps %.3f ms/step, %.1f iterations/step" % (nsteps, res["neumann"]["ms_per_step"],
                                                                 res["neumann"]["iters_per_step"]))
    return res


def batched_helmholtz(n, reps):
    """Batched modified-Helmholtz solves: n seeded instances (star domains,
    grids drawn from {128, 256, 512, 1024}, kappa ~ U[1, 1e4], smooth random
    f and g), solved plain (one call per instance, in turn) and batched (one
    call for all), in FP64 and with FP32 inner solves.  Throughput in
    grid-pts * GMRES-iters / s over all instances."""
    import numpy as np
    import torch
    import workloads as W
    from workloads.fields import SmoothField
    from paper_2404_14864_amd import kfbi
    dev = "cuda:0"

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    t0 = time.perf_counter()
    mem = []
    for i in range(n):
        desc, kappa, rng = W.domain_c4_instance(i)
        f, g = SmoothField(rng), SmoothField(rng)
        h = kfbi.kfbi_domain_create(desc)
        zx, zy = kfbi.kfbi_domain_copy_boundary(h)
        x = W.grid_coords(1.0, desc["M"])
        M = desc["M"]
        mem.append({"h": h, "M": M, "Nb": desc["Nb"], "kappa": kappa, "f": d(f.grid(x, x).ravel()), "fg": d(f(zx, zy)),
                    "g": d(g(zx, zy)), "u": torch.zeros((M + 1) ** 2, dtype=torch.float64, device=dev)})
    torch.cuda.synchronize()
    log("batch: %d instances created in %.1f s (grids %s)" % (
        n, time.perf_counter() - t0, dict(zip(*np.unique([m["M"] for m in mem], return_counts=True)))))
    pts = np.array([(m["M"] - 1) ** 2 for m in mem], dtype=np.float64)
    out = {"workload": "%d batched Helmholtz instances, star r0~U[0.3,0.6] lobes 3..8 amp 0.2 r0, grids "
                       "U{128,256,512,1024}, Nb=M, kappa~U[1,1e4], smooth random f and g, tol 1e-10" % n}
    for label, prec in (("fp64", kfbi.KFBI_PREC_FP64), ("mixed", kfbi.KFBI_PREC_MIXED)):
        opts = {"tol": 1e-10, "precision": prec}
        # plain: one solve per instance in turn (first pass warms coefficients)
        for m in mem:
            kfbi.kfbi_helmholtz_solve(m["h"], m["kappa"], m["f"], m["fg"], m["g"], m["u"], opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for m in mem:
            s = kfbi.kfbi_helmholtz_solve(m["h"], m["kappa"], m["f"], m["fg"], m["g"], m["u"], opts=opts)
            its.append(s["iters"])
        torch.cuda.synchronize()
        Tp = time.perf_counter() - t0
        plain = float(np.dot(pts, its) / Tp)
        ref = [m["u"].clone() for m in mem]
        # batched
        b = kfbi.kfbi_batch_create([m["h"] for m in mem])
        args = ([m["kappa"] for m in mem], [m["f"] for m in mem], [m["fg"] for m in mem], [m["g"] for m in mem],
                [m["u"] for m in mem])
        kfbi.kfbi_batch_helmholtz(b, *args, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bits = None
        for _ in range(reps):
            st = kfbi.kfbi_batch_helmholtz(b, *args, opts=opts)
            bits = [x["iters"] for x in st]
        torch.cuda.synchronize()
        Tb = (time.perf_counter() - t0) / reps
        batched = float(np.dot(pts, bits) / Tb)
        diff = max(float((m["u"] - r).abs().max() / max(r.abs().max(), 1e-300)) for m, r in zip(mem, ref))
        tuning = [r for r in kfbi.kfbi_batch_tuning(b) if r["tuned"]]
        kfbi.kfbi_batch_destroy(b)
        # the same batch with the default tridiagonal launch shapes
        b = kfbi.kfbi_batch_create([m["h"] for m in mem])
        opts_nt = dict(opts, no_tune=True)
        kfbi.kfbi_batch_helmholtz(b, *args, opts=opts_nt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            kfbi.kfbi_batch_helmholtz(b, *args, opts=opts_nt)
        torch.cuda.synchronize()
        Tu = (time.perf_counter() - t0) / reps
        kfbi.kfbi_batch_destroy(b)
        out[label] = {"plain_value": plain, "plain_ms": 1e3 * Tp, "batched_value": batched, "batched_ms": 1e3 * Tb,
                      "batched_untuned_ms": 1e3 * Tu, "speedup": batched / plain, "gmres_iters_total": int(sum(bits)),
                      "max_rel_diff_batched_vs_plain": diff,
                      "tridiag_shapes": ["M%d %s: %s kernel, %d modes/wg%s, %.1f us" % (
                          r["M"], r["kind"], "register-row" if r["register_rows"] else "LDS-tile", r["modes_per_wg"],
                          " staged" if r["staged"] else "", r["us"])
                          for r in tuning]}
        log("batch %s: plain %.3g (%.1f ms), batched %.3g (%.1f ms; default shapes %.1f ms), x%.1f, %d iterations" % (
            label, plain, 1e3 * Tp, batched, 1e3 * Tb, 1e3 * Tu, batched / plain, sum(bits)))
        log("batch %s tridiagonal shapes: %s" % (label, "; ".join(out[label]["tridiag_shapes"])))
    out["unit"] = "grid-pts*GMRES-iters/s"
    for m in mem:
        kfbi.kfbi_domain_destroy(m["h"])
    return out


def serving(n_jobs, seed=20240423):
    """The serving workload on a bounded sample: n_jobs seeded jobs (heat,
    wave, Schroedinger 40/40/20; star or ellipse domains; grids uniform over
    {256, 512, 1024, 2048}; 50..500 steps each).  First the capacity: the
    jobs served with every arrival at t = 0 (jobs per second at
    saturation); then Poisson arrivals at 0.8 of that rate, in FP64 and with
    the FP32 / complex64 inner solves; then the plain per-solve path (each
    job alone, FP64, synchronous steps).  The budget is half of what the
    sample's jobs hold together, so admission waits for memory.  Every
    served job's final grid is compared with the plain path's."""
    import numpy as np
    import torch
    from workloads.serving import job_fields, job_stream
    from paper_2404_14864_amd import kfbi
    from paper_2404_14864_amd.serving import Job, Server, serve_plain
    specs = job_stream(seed, n_jobs, rate=1.0, grids=(256, 512, 1024, 2048), steps=(50, 500))
    # footprint of each job shape, for the budget
    fp = {}
    for s in specs:
        key = (s["kind"], s["desc"]["M"])
        if key not in fp:
            j = Job(s, job_fields)
            fp[key] = j.footprint
            j.close()
    total = sum(fp[(s["kind"], s["desc"]["M"])] for s in specs)
    budget = total // 2
    outs = {}

    def keeper(tag):
        d = outs.setdefault(tag, {})
        return lambda j: d.__setitem__(j.spec["id"], j.u.cpu().numpy())

    base = {"tol": 1e-10}
    sat = [dict(s, arrival=0.0) for s in specs]
    rep_sat = Server(budget, job_fields, base).run(sat, tick=1.0)
    capacity = len(specs) / rep_sat["wall_s"]
    rate = 0.8 * capacity
    # arrival times of the stream rescaled to the measured rate
    t = np.array([s["arrival"] for s in specs])
    poisson = [dict(s, arrival=float(a)) for s, a in zip(specs, t / rate)]
    rep = Server(budget, job_fields, base, keep_output=keeper("fp64")).run(poisson, tick=1.0)
    repm = Server(budget, job_fields, dict(base, precision=kfbi.KFBI_PREC_MIXED),
                  keep_output=keeper("mixed")).run(poisson, tick=1.0)
    plain = serve_plain(specs, job_fields, base, keep_output=keeper("plain"))
    # the wave jobs once more on the plain path at tol 1e-12: how far two
    # FP64 runs that both meet tol 1e-10 can drift apart over the steps
    tight = serve_plain([s for s in specs if s["kind"] == "wave"], job_fields, {"tol": 1e-12},
                        keep_output=keeper("plain_tol1e-12"))
    diff, diff_by = {}, {}
    kind_of = {s["id"]: "%s M=%d" % (s["kind"], s["desc"]["M"]) for s in specs}
    for tag in ("fp64", "mixed", "plain_tol1e-12"):
        by = diff_by.setdefault(tag, {})
        for i in outs[tag]:
            e = float(np.max(np.abs(outs[tag][i] - outs["plain"][i])) /
                      max(float(np.max(np.abs(outs["plain"][i]))), 1e-300))
            by[kind_of[i]] = max(by.get(kind_of[i], 0.0), e)
        diff[tag] = max(by.values()) if by else None
    for r in (rep_sat, rep, repm):
        r["n_finished"] = len(r.pop("finished"))
        r["n_rejected"] = len(r.pop("rejected"))
    out = {"workload": "%d jobs, heat/wave/Schroedinger 40/40/20, star (heat, wave) and ellipse (Schroedinger) "
                       "domains, grids U{256,512,1024,2048}, Nb=M, 50-500 steps, tol 1e-10; Poisson arrivals at 0.8 "
                       "of the measured capacity; budget half of the jobs' summed footprint" % len(specs),
           "capacity_jobs_per_s": capacity, "arrival_rate_jobs_per_s": rate, "budget_bytes": budget,
           "sum_of_footprints_bytes": total, "saturated": rep_sat, "served_fp64": rep, "served_mixed": repm,
           "plain_fp64": plain, "plain_fp64_tol1e-12_wave_jobs": {"steps": tight["steps"], "wall_s": tight["wall_s"]},
           "max_rel_diff_vs_plain": diff, "max_rel_diff_vs_plain_by_type": diff_by,
           "diff_note": "relative max-norm difference of each job's final grid from the plain FP64 path at tol "
                        "1e-10; plain_tol1e-12 is the same plain path solved to 1e-12 (wave jobs only)",
           "speedup_fp64_vs_plain": rep["throughput"] / plain["throughput"],
           "speedup_mixed_vs_plain": repm["throughput"] / plain["throughput"]}
    log("serving: capacity %.2f jobs/s; served fp64 %.3g (p50 %.2f p99 %.2f ms), mixed %.3g (p99 %.2f ms), plain %.3g "
        "(p50 %.2f p99 %.2f ms) grid-pts*iters/s; %d admitted while busy; diff vs plain fp64 %.1e mixed %.1e" % (
            capacity, rep["throughput"], rep["p50_step_ms"], rep["p99_step_ms"], repm["throughput"],
            repm["p99_step_ms"], plain["throughput"], plain["p50_step_ms"], plain["p99_step_ms"],
            rep["admitted_while_device_busy"], diff["fp64"], diff["mixed"]))
    return out


def graph_leg(grids=(256, 1024), n=50):
    """kfbi_grid_solve_noalloc (three dependent kernels, no allocation) n times
    back to back on a stream, and the same n calls captured once in a HIP
    graph and replayed: per-solve time of each, and whether every replay
    gives the stream's bits."""
    import torch
    import workloads as W
    from paper_2404_14864_amd import kfbi
    out = {}
    s = torch.cuda.Stream()
    for M in grids:
        h = kfbi.kfbi_domain_create(W.domain_c2_wave(M), kfbi.KFBI_REAL, stream=s.cuda_stream)
        try:
            g_rhs = torch.Generator(device="cuda:0")
            g_rhs.manual_seed(M)
            rhs = torch.randn((M + 1) ** 2, dtype=torch.float64, device="cuda:0", generator=g_rhs)
            u = torch.zeros_like(rhs)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(s):
                for _ in range(3):
                    kfbi.kfbi_grid_solve_noalloc(h, 7.0, rhs, u)
                e0.record(s)
                for _ in range(n):
                    kfbi.kfbi_grid_solve_noalloc(h, 7.0, rhs, u)
                e1.record(s)
            s.synchronize()
            t_stream = e0.elapsed_time(e1) / n
            ref = u.clone()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                for _ in range(n):
                    kfbi.kfbi_grid_solve_noalloc(h, 7.0, rhs, u)
            s.synchronize()
            times, same = [], True
            for _ in range(3):
                u.zero_()
                torch.cuda.synchronize()
                with torch.cuda.stream(s):
                    e0.record(s)
                    g.replay()
                    e1.record(s)
                s.synchronize()
                times.append(e0.elapsed_time(e1) / n)
                same = same and bool(torch.equal(u, ref))
            del g
        finally:
            kfbi.kfbi_domain_destroy(h)
        out["M=%d" % M] = {"stream_us_per_solve": 1e3 * t_stream, "graph_us_per_solve": 1e3 * min(times),
                           "graph_replays_bitwise_equal": same}
        log("graph capture, grid solve M=%d: stream %.2f us, graph replay %.2f us per solve (3 kernels)%s" % (
            M, 1e3 * t_stream, 1e3 * min(times), "" if same else "; REPLAY DIFFERS"))
    out["what"] = ("kfbi_grid_solve_noalloc x%d (x-DST, tridiagonal, inverse x-DST) on a stream vs captured in one "
                   "HIP graph and replayed (best of 3 replays)" % n)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the whole method on a single "
              "MI355X (no collectives or sharding); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    # the oracle's sample of the headline workload first: its solution after
    # the sampled steps is the reference of the accuracy figure
    cpu, cpu_ref = None, None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the headline workload (~%.0f s on all cores, ~%.0f s on one)" % (
            args.cpu_seconds, args.cpu_seconds))
        cpu, cpu_ref = cpu_baseline(args.M, args.cpu_seconds)
        log("oracle: %.3g grid-pts*iters/s on %d cores (%.0f ms/step), %.3g on one core" % (
            cpu["value"], cpu["cores"], cpu["ms_per_step"], cpu["single_core"]["value"]))

    H = headline(args, cpu_ref)
    labels, kern, kdom, avg_us, bytes_launch = H["profile"]
    S = H["S"]
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    lat = H["lat"]
    wave = None if args.no_secondary else wave_leg(args)

    if args.calibrate_copy > 0:
        nb = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nb, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB three times" % args.calibrate_copy)
        del src, dst

    batched = batched_helmholtz(args.batch, args.batch_reps) if (args.batch > 0 and not args.no_secondary) else None
    served = serving(args.serve_jobs) if (args.serve_jobs > 0 and not args.no_secondary) else None
    graph = None if args.no_secondary else graph_leg()

    pts = (S.M - 1) ** 2
    w = 16.0  # complex128 bytes per element
    out = {
        "metric": "grid-pts*GMRES-iters/s per KFBI step",
        "value": H["value"],
        "unit": "grid-pts*GMRES-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * H["T"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "Schroedinger, Strang splitting, ellipse 0.6/0.4 in [-1,1]^2, %dx%d grid, Nb=%d "
                               "(reading R4: the paper fixes Nb = M in section 4; the configuration lists 2M), "
                               "V=50(x^2+y^2), Gaussian packet width 0.1 k=(20,0), g=0, dt=h/2" % (S.M, S.M, S.Nb),
                   "equation": "schrodinger", "M": S.M, "Nb": S.Nb, "tau": S.tau, "precision": "fp64 (complex128)",
                   "parallelism": "single GPU"},
        "p50_step_ms": float(np.percentile(lat, 50)),
        "p99_step_ms": float(np.percentile(lat, 99)),
        "latency": "device time per step from HIP events on the library's stream",
        "gmres_iters_per_step": float(np.mean(H["iters"])),
        "solution_finite": H["finite"],
        "accuracy": H.get("accuracy"),
        "roofline": {"bound": "hbm", "kernel": kdom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC.get(kdom),
                     "avg_launch_us": avg_us, "bytes_per_launch": bytes_launch,
                     "labels": kern[kdom]["labels"],
                     "timing": "replay of %d back-to-back launches between two HIP events, averaged over the "
                               "kernel's launches in %d profiled steps" % (args.replay, args.profile_steps),
                     "per_unit": "the kernel's own algorithmic bytes: the write of U^ (w per grid point and "
                                 "iteration) plus its sparse input; a dense launch also reads R^"},
        "path_efficiency": {"model": "4w per grid point and iteration (the three-pass grid solve: write R^, "
                                     "read R^ and write U^, read U^), w = 16 B",
                            "achieved": 4 * w * H["value"] / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": 4 * w * H["value"] / 1e9 / HBM_PEAK_GBS},
        "kernels": labels,
        "kernels_merged": kern,
        "mixed_precision": H["mixed"],
        "wave": wave,
        "batched": batched,
        "serving": served,
        "graph_capture": graph,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
