"""GPU tests of the serving loop (time-stepping jobs admitted by device
footprint and advanced together, heat and wave jobs in one batched step per
tick, Schroedinger jobs alone).

Bars:
  * each job served in the mix ends with the same grid, bit for bit, as the
    same job stepped alone;
  * the admitted jobs never hold more than the budget, and a budget that
    binds still serves every job;
  * a job that cannot fit even alone is rejected, not queued forever.
Inputs: seeded job streams of `workloads.serving` on small grids.
"""

import numpy as np
import pytest

from workloads.serving import job_fields, job_stream

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2404_14864_amd.serving import Job, Server  # noqa: E402

OPTS = {"tol": 1e-10}


def _specs(n=7):
    return job_stream(11, n, rate=3.0, grids=(64, 128), steps=(2, 4))


def test_mix_equals_alone_bitwise():
    specs = _specs()
    assert {s["kind"] for s in specs} == {"heat", "wave", "schrodinger"}
    out = {}
    srv = Server(1 << 40, job_fields, OPTS, keep_output=lambda j: out.__setitem__(j.spec["id"], j.u.cpu().numpy()))
    rep = srv.run(specs, tick=1.0)
    assert sorted(rep["finished"]) == [s["id"] for s in specs] and not rep["rejected"]
    assert rep["max_concurrent_jobs"] >= 3
    assert rep["steps"] == sum(s["steps"] for s in specs)
    assert rep["p50_step_ms"] > 0 and rep["p99_step_ms"] >= rep["p50_step_ms"] and rep["throughput"] > 0
    for s in specs:
        j = Job(s, job_fields)
        try:
            for _ in range(s["steps"]):
                st = j.step_alone(OPTS)
                assert st["converged"], s["id"]
            assert np.array_equal(j.u.cpu().numpy(), out[s["id"]]), s["id"]
        finally:
            j.close()


def test_budget_is_never_exceeded():
    specs = _specs()
    fps = []
    for s in specs:
        j = Job(s, job_fields)
        fps.append(j.footprint)
        j.close()
    budget = int(1.2 * max(fps))
    srv = Server(budget, job_fields, OPTS)
    rep = srv.run(specs, tick=1.0)
    assert sorted(rep["finished"]) == [s["id"] for s in specs] and not rep["rejected"]
    assert rep["max_used_bytes"] <= budget
    # the budget binds: all jobs together would not fit, and fewer run at once
    # than without a budget
    assert sum(fps) > budget and 1 <= rep["max_concurrent_jobs"] < len(specs)


def test_job_larger_than_budget_is_rejected():
    specs = _specs(3)
    srv = Server(4096, job_fields, OPTS)
    rep = srv.run(specs, tick=1.0)
    assert rep["finished"] == [] and sorted(rep["rejected"]) == [s["id"] for s in specs]
    assert rep["max_used_bytes"] == 0
