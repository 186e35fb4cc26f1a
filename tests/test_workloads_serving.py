"""The serving job stream: seeded, Poisson arrivals in increasing order, the
three equations in roughly the stated mix, grids and step counts within their
ranges, and fields that are fixed arrays times time factors."""

import numpy as np

from workloads import manufactured as mf
from workloads.serving import job_fields, job_stream


def test_stream_is_seeded_and_well_formed():
    a = job_stream(5, 400, rate=2.0)
    b = job_stream(5, 400, rate=2.0)
    assert [(x["arrival"], x["kind"], x["desc"]["M"], x["steps"]) for x in a] == \
        [(x["arrival"], x["kind"], x["desc"]["M"], x["steps"]) for x in b]
    t = np.array([x["arrival"] for x in a])
    assert np.all(np.diff(t) > 0)
    # mean inter-arrival 1/rate within sampling error
    assert abs(np.mean(np.diff(t)) - 0.5) < 0.1
    kinds = [x["kind"] for x in a]
    for k, p in (("heat", 0.4), ("wave", 0.4), ("schrodinger", 0.2)):
        assert abs(kinds.count(k) / len(kinds) - p) < 0.08
    assert {x["desc"]["M"] for x in a} == {256, 512, 1024, 2048}
    assert all(50 <= x["steps"] <= 500 for x in a)
    assert all(x["desc"]["Nb"] == x["desc"]["M"] for x in a)
    assert all(x["desc"]["kind"] == ("ellipse" if x["kind"] == "schrodinger" else "star") for x in a)


def test_fields_scale_with_time():
    for spec in job_stream(3, 12, rate=1.0, grids=(64,), steps=(2, 3)):
        zx = np.linspace(-0.4, 0.4, 64)
        zy = np.linspace(0.3, -0.3, 64)
        f = job_fields(spec, zx, zy)
        t = 0.37
        if spec["kind"] == "heat":
            assert np.allclose(f["gfac"](t) * f["g0"], mf.heat_u(zx, zy, t), rtol=1e-14, atol=1e-15)
            assert np.allclose(f["sfac"](0.1, t) * f["s0g"], mf.heat_src(zx, zy, 0.1) + mf.heat_src(zx, zy, t),
                               rtol=1e-13, atol=1e-14)
        elif spec["kind"] == "wave":
            assert np.allclose(f["gfac"](t) * f["g0"], mf.wave_u(zx, zy, t), rtol=1e-14, atol=1e-15)
            assert f["sfac"] is None
        else:
            assert not np.any(f["g0"]) and f["v"] is not None
