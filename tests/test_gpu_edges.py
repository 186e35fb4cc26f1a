"""GPU edge cases: the largest grid (2048, Nb = M as in the paper's
experiments) by a property that holds at any size (second-order convergence
to the exact solution e^{ax+by}, a^2 + b^2 = kappa, from 1024 to 2048), the
most collocation points a solve takes (8192, on the 2048 grid) by GMRES's own
invariants (the reported residual is the true one, and it does not grow with
the iteration count), kappa = 0 (Laplace), all-zero data
(u = 0 exactly, no GMRES iteration), a batched step with no active member,
and an empty batch (refused).
"""

import numpy as np
import pytest

import workloads as W
from workloads import manufactured as mf
from workloads.domains import star

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2404_14864_amd import kfbi  # noqa: E402
from tests.gpu_util import GpuDomain, dev, empty_gamma, empty_grid, host  # noqa: E402


def _exp_solve(M, kappa, a, b, Nb=None):
    desc = star(0.5, 0.1, 5, 1.0, M, Nb or M)
    x = W.grid_coords(1.0, M)
    X, Y = np.meshgrid(x, x)
    with GpuDomain(desc) as g:
        u = empty_grid(M)
        f = np.zeros((M + 1) ** 2)
        st = kfbi.kfbi_helmholtz_solve(g.h, kappa, dev(f), dev(np.zeros(g.Nb)), dev(mf.helm_exp_u(g.zx, g.zy, a, b)),
                                       u, opts={"tol": 1e-10})
        inside = (kfbi.kfbi_domain_copy_classification(g.h) & 1).astype(bool).ravel()
        U = host(u)
    ex = mf.helm_exp_u(X, Y, a, b).ravel()
    return st, np.max(np.abs(U - ex)[inside]) / np.max(np.abs(ex[inside]))


def test_largest_grid_second_order():
    kappa = 25.0
    a, b = 3.0, 4.0  # a^2 + b^2 = kappa
    st1, e1 = _exp_solve(1024, kappa, a, b)
    st2, e2 = _exp_solve(2048, kappa, a, b)
    assert st1["converged"] and st2["converged"], (st1, st2)
    assert e2 < 1e-5, e2
    assert e1 / e2 > 2.5, (e1, e2)


def test_most_collocation_points_gmres_invariants():
    """Nb = 8192 = 4M: 16 entries of each Krylov vector per thread.  With four
    collocation points per grid cell the discrete operator is far worse
    conditioned than at Nb = M (the oracle's K: condition number 2.5 at
    M = Nb = 64, 2.5e4 at M = 64, Nb = 256), so the test runs a fixed number
    of iterations from phi = 0 and checks GMRES's invariants: the reported
    relative residual equals ||g - K phi|| / ||g|| with K phi evaluated by a
    separate interface evaluation, and the minimal residual over a larger
    Krylov space is not larger."""
    M, Nb = 2048, 8192
    desc = star(0.5, 0.1, 5, 1.0, M, Nb)
    with GpuDomain(desc) as g:
        gg = dev(mf.helm_exp_u(g.zx, g.zy, 3.0, 4.0))
        gn = float(np.linalg.norm(host(gg)))
        res = []
        for it in (20, 40):
            u = empty_grid(M)
            phi = empty_gamma(Nb)
            st = kfbi.kfbi_helmholtz_solve(g.h, 25.0, None, None, gg, u, phi,
                                           opts={"fixed_iters": it, "restart": 50})
            assert st["iters"] == it
            up = empty_gamma(Nb)
            kfbi.kfbi_interface_apply(g.h, 25.0, None, None, phi, None, up)
            true = float(np.linalg.norm(host(gg) - host(up))) / gn
            assert abs(true - st["rel_resid"]) <= 1e-3 * true + 1e-10, (it, true, st)
            res.append(true)
        assert res[0] < 1.0 and res[1] <= res[0] * (1 + 1e-8), res


def test_laplace_kappa_zero():
    """u = e^x cos y is harmonic: the kappa = 0 solve reproduces it to second
    order."""
    errs = []
    for M in (128, 256):
        desc = star(0.5, 0.1, 5, 1.0, M, M)
        x = W.grid_coords(1.0, M)
        X, Y = np.meshgrid(x, x)
        ex = (np.exp(X) * np.cos(Y)).ravel()
        with GpuDomain(desc) as g:
            u = empty_grid(M)
            gg = np.exp(g.zx) * np.cos(g.zy)
            st = kfbi.kfbi_helmholtz_solve(g.h, 0.0, dev(np.zeros((M + 1) ** 2)), dev(np.zeros(g.Nb)), dev(gg), u,
                                           opts={"tol": 1e-12})
            inside = (kfbi.kfbi_domain_copy_classification(g.h) & 1).astype(bool).ravel()
            assert st["converged"]
            errs.append(np.max(np.abs(host(u) - ex)[inside]) / np.max(np.abs(ex[inside])))
    assert errs[1] < 1e-4 and errs[0] / errs[1] > 2.5, errs


def test_zero_data_zero_solution():
    desc = W.domain_c2_wave(128, Nb=128)
    with GpuDomain(desc) as g:
        u = empty_grid(g.M) + 7.0
        phi = empty_gamma(g.Nb)
        st = kfbi.kfbi_helmholtz_solve(g.h, 50.0, dev(np.zeros((g.M + 1) ** 2)), dev(np.zeros(g.Nb)),
                                       dev(np.zeros(g.Nb)), u, phi)
        inside = (kfbi.kfbi_domain_copy_classification(g.h) & 1).astype(bool).ravel()
        assert st["converged"] and st["iters"] == 0
        assert not np.any(host(u)[inside]) and not np.any(host(phi))


def test_batch_step_with_no_active_member():
    desc = W.domain_c2_wave(64, Nb=64)
    with GpuDomain(desc) as g:
        tau = 2.0 / 64
        s = kfbi.kfbi_stepper_create(g.h, kfbi.KFBI_WAVE, tau, theta=0.25)
        x = W.grid_coords(1.0, 64)
        X, Y = np.meshgrid(x, x)
        gx, gy = g.zx, g.zy
        kfbi.kfbi_stepper_init(s, dev(mf.wave_u(X, Y, 0).ravel()), dev(mf.wave_lap(X, Y, 0).ravel()),
                               dev(mf.wave_u(gx, gy, 0)), dev(mf.wave_lap(gx, gy, 0)),
                               dev(mf.wave_u(X, Y, -tau).ravel()), dev(mf.wave_lap(X, Y, -tau).ravel()),
                               dev(mf.wave_u(gx, gy, -tau)), dev(mf.wave_lap(gx, gy, -tau)))
        before = host(kfbi.kfbi_stepper_get_state(s)).copy()
        b = kfbi.kfbi_batch_create([g.h])
        try:
            st = kfbi.kfbi_batch_step(b, [s], [None], [None], active=[False])
            assert st[0]["iters"] == 0
            assert np.array_equal(host(kfbi.kfbi_stepper_get_state(s)), before)
        finally:
            kfbi.kfbi_batch_destroy(b)
            kfbi.kfbi_stepper_destroy(s)


def test_empty_batch_is_refused():
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.kfbi_batch_create([])
    assert e.value.code == kfbi.KFBI_EINVAL


def test_too_many_collocation_points_for_a_solve():
    """Domains take Nb up to 16384, solves up to 8192 (one workgroup holds a
    Krylov vector): beyond it the solve is refused before any launch."""
    desc = star(0.5, 0.1, 5, 1.0, 256, 8200)
    with GpuDomain(desc) as g:
        u = empty_grid(256)
        with pytest.raises(kfbi.KfbiError) as e:
            kfbi.kfbi_helmholtz_solve(g.h, 10.0, None, None, dev(np.zeros(g.Nb)), u)
        assert e.value.code == kfbi.KFBI_ENOTSUP


def test_batch_refuses_small_grids_at_creation():
    """Members below M = 64 are refused by kfbi_batch_create (the batched
    row-wise stencil evaluation needs a 64-mode row), not half-way through a
    solve."""
    from workloads.domains import disk
    with GpuDomain(disk(0.3, 1.0, 32, 32)) as g:
        with pytest.raises(kfbi.KfbiError) as e:
            kfbi.kfbi_batch_create([g.h])
        assert e.value.code == kfbi.KFBI_ENOTSUP and "M >= 64" in str(e.value)


def test_refused_domains_free_their_setup_buffers():
    """A disk too small to cross a grid line is refused after the set-up has
    allocated its temporaries; repeated refusals leave the device's free
    memory where it was."""
    from workloads.domains import disk
    M = 256
    h = 2.0 / M
    desc = disk(0.1 * h, 1.0, M, 16, cx=0.5 * h, cy=0.5 * h)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(200):
        with pytest.raises(kfbi.KfbiError) as e:
            kfbi.kfbi_domain_create(desc)
        assert e.value.code == kfbi.KFBI_EDOMAIN
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (1 << 20)
