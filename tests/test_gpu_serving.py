"""GPU tests of the serving loop (continuous batching: time-stepping jobs
admitted by device footprint as they arrive, heat and wave jobs advanced in
one batched step per round on one lane, Schroedinger jobs in one batched
step per round on another, the lanes running concurrently).

Bars:
  * each job served in the mix ends with the same grid, bit for bit, as the
    same job stepped alone, in FP64; with the FP32 / complex64 inner solves
    within 1e-8 of it;
  * jobs are admitted while earlier ones are on the device;
  * the admitted jobs never hold more than the budget, and a budget that
    binds still serves every job;
  * a job that cannot fit even alone is rejected, not queued forever.
Inputs: seeded job streams of `workloads.serving` on small grids; arrival
times in units of 1 ms of wall time.
"""

import numpy as np
import pytest

from workloads.serving import job_fields, job_stream

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2404_14864_amd import kfbi  # noqa: E402
from paper_2404_14864_amd.serving import Job, Server  # noqa: E402

OPTS = {"tol": 1e-10}
TICK = 1e-3


def _specs(n=7):
    return job_stream(11, n, rate=3.0, grids=(64, 128), steps=(2, 4))


def _alone(specs):
    ref = {}
    for s in specs:
        j = Job(s, job_fields)
        try:
            for _ in range(s["steps"]):
                st = j.step_alone(OPTS)
                assert st["converged"], s["id"]
            ref[s["id"]] = j.u.cpu().numpy()
        finally:
            j.close()
    return ref


def test_mix_equals_alone_bitwise():
    specs = _specs()
    assert {s["kind"] for s in specs} == {"heat", "wave", "schrodinger"}
    out = {}
    srv = Server(1 << 40, job_fields, OPTS, keep_output=lambda j: out.__setitem__(j.spec["id"], j.u.cpu().numpy()))
    rep = srv.run(specs, tick=TICK)
    assert sorted(rep["finished"]) == [s["id"] for s in specs] and not rep["rejected"]
    assert rep["max_concurrent_jobs"] >= 3
    assert rep["admitted_while_device_busy"] >= 1
    assert rep["steps"] == sum(s["steps"] for s in specs)
    assert rep["p50_step_ms"] > 0 and rep["p99_step_ms"] >= rep["p50_step_ms"] and rep["throughput"] > 0
    ref = _alone(specs)
    for s in specs:
        assert np.array_equal(ref[s["id"]], out[s["id"]]), s["id"]


def test_mixed_precision_mix_within_tolerance_of_alone():
    specs = _specs()
    out = {}
    srv = Server(1 << 40, job_fields, dict(OPTS, precision=kfbi.KFBI_PREC_MIXED),
                 keep_output=lambda j: out.__setitem__(j.spec["id"], j.u.cpu().numpy()))
    rep = srv.run(specs, tick=TICK)
    assert sorted(rep["finished"]) == [s["id"] for s in specs]
    ref = _alone(specs)
    for s in specs:
        a, b = out[s["id"]], ref[s["id"]]
        assert np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(b)), s["id"]


def test_budget_is_never_exceeded():
    specs = _specs()
    fps = []
    for s in specs:
        j = Job(s, job_fields)
        fps.append(j.footprint)
        j.close()
    budget = int(1.2 * max(fps))
    srv = Server(budget, job_fields, OPTS)
    rep = srv.run(specs, tick=TICK)
    assert sorted(rep["finished"]) == [s["id"] for s in specs] and not rep["rejected"]
    assert rep["max_used_bytes"] <= budget
    # the budget binds: all jobs together would not fit, and fewer run at once
    # than without a budget
    assert sum(fps) > budget and 1 <= rep["max_concurrent_jobs"] < len(specs)


def test_job_larger_than_budget_is_rejected():
    specs = _specs(3)
    srv = Server(4096, job_fields, OPTS)
    rep = srv.run(specs, tick=TICK)
    assert rep["finished"] == [] and sorted(rep["rejected"]) == [s["id"] for s in specs]
    assert rep["max_used_bytes"] == 0
