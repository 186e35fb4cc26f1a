"""GPU parity of the Neumann problem (eqs. 3.19, 3.20, 3.22, the interface
problem 3.29) against the oracle: fixed-iteration and converged solves
(density, grid solution, trace U+), real and complex kappa, FP64, mixed
precision and the Richardson form; Neumann steppers of the three equations;
second-order convergence on the 512 grid; refused cases.

Each side evaluates boundary data at its own collocation points and with
its own outward normals.
"""

import numpy as np
import pytest

import workloads as W
from workloads import manufactured as mf
from oracle import bie
from oracle.geometry import Domain
from oracle.steppers import HeatStepper, SchrodingerStepper, WaveStepper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2404_14864_amd import kfbi  # noqa: E402
from tests.gpu_util import GpuDomain, dev, empty_gamma, empty_grid, host, rel_err  # noqa: E402

TOL = 1e-10

DOMAINS = {
    "c1_disk64": W.domain_c1_heat(64),
    "c2_star128": W.domain_c2_wave(128),
    "c2_star256_nb2M": W.domain_c2_wave(256, Nb=512),
    "c3_ellipse128": W.domain_c3_schrodinger(128),
    "star_even_lobes": W.domains.star(0.45, 0.09, 4, 1.0, 128, 256),
}


def _dn_oracle(grad, od):
    gx, gy = grad
    return gx * od.colloc["nx"] + gy * od.colloc["ny"]


def _dn_gpu(grad, g):
    nx, ny = kfbi.kfbi_domain_copy_normals(g.h)
    gx, gy = grad
    return gx * nx + gy * ny


def test_normals_match_oracle():
    for name in ("c1_disk64", "c2_star128", "c3_ellipse128"):
        od = Domain(DOMAINS[name])
        with GpuDomain(DOMAINS[name]) as g:
            nx, ny = kfbi.kfbi_domain_copy_normals(g.h)
        assert np.max(np.abs(nx - od.colloc["nx"])) < 1e-13
        assert np.max(np.abs(ny - od.colloc["ny"])) < 1e-13


@pytest.mark.parametrize("name,kappa", [("c1_disk64", 64.0), ("c2_star128", 4.0 * 64 * 64),
                                         ("c2_star256_nb2M", 300.0), ("c3_ellipse128", 2j * 256),
                                         ("star_even_lobes", 50.0)])
def test_neumann_solve_fixed_iterations(name, kappa):
    """Same number of GMRES iterations on both sides: same density, grid
    solution and trace to rounding (f and du/dn of sin(pi x) cos(pi y))."""
    desc = DOMAINS[name]
    cplx = isinstance(kappa, complex)
    od = Domain(desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    U_ref, psi_ref, tr_ref, st_ref = bie.neumann_solve(
        od, kappa, mf.helm_trig_f(od.X, od.Y, kappa), mf.helm_trig_f(zx, zy, kappa),
        _dn_oracle(mf.helm_trig_grad(zx, zy), od) + 0j * cplx, fixed_iters=12)
    with GpuDomain(desc, cplx) as g:
        M, Nb = g.M, g.Nb
        u, psi, tr = empty_grid(M, cplx), empty_gamma(Nb, cplx), empty_gamma(Nb, cplx)
        st = kfbi.kfbi_neumann_solve(
            g.h, kappa, dev(mf.helm_trig_f(od.X, od.Y, kappa).ravel(), cplx),
            dev(mf.helm_trig_f(g.zx, g.zy, kappa), cplx), dev(_dn_gpu(mf.helm_trig_grad(g.zx, g.zy), g), cplx),
            u, psi, tr, opts={"fixed_iters": 12})
        U = host(u).reshape(M + 1, M + 1)
        PSI, TR = host(psi), host(tr)
    assert st["iters"] == st_ref["iters"] == 12
    assert abs(st["rel_resid"] - st_ref["rel_resid"]) <= 1e-3 * st_ref["rel_resid"] + 1e-14
    assert rel_err(PSI, psi_ref) < TOL
    assert rel_err(U, U_ref, od.inside) < TOL
    assert rel_err(TR, tr_ref) < TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_neumann_solve_to_tolerance(precision):
    """exp(3x + 4y), kappa = 25, no source, warm start from zero."""
    desc = DOMAINS["c2_star128"]
    od = Domain(desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    U_ref, psi_ref, tr_ref, st_ref = bie.neumann_solve(od, 25.0, None, None,
                                                       _dn_oracle(mf.helm_exp_grad(zx, zy, 3.0, 4.0), od), tol=1e-12)
    opts = {"tol": 1e-12 if precision == "fp64" else 1e-11,
            "precision": kfbi.KFBI_PREC_FP64 if precision == "fp64" else kfbi.KFBI_PREC_MIXED}
    with GpuDomain(desc) as g:
        u, psi, tr = empty_grid(g.M), empty_gamma(g.Nb), empty_gamma(g.Nb)
        st = kfbi.kfbi_neumann_solve(g.h, 25.0, None, None, dev(_dn_gpu(mf.helm_exp_grad(g.zx, g.zy, 3.0, 4.0), g)),
                                     u, psi, tr, opts=opts)
        U = host(u).reshape(g.M + 1, g.M + 1)
        TR = host(tr)
    assert st["converged"]
    tol = 1e-10 if precision == "fp64" else 1e-8
    assert rel_err(U, U_ref, od.inside) < tol
    assert rel_err(TR, tr_ref) < tol


def test_neumann_richardson_matches_oracle():
    """Eq. 3.22 with gamma = 0.9, fixed updates on both sides."""
    desc = DOMAINS["c1_disk64"]
    od = Domain(desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    U_ref, psi_ref, _, _ = bie.neumann_solve(od, 64.0, None, None, _dn_oracle(mf.helm_exp_grad(zx, zy, 3.0, 4.0), od),
                                             fixed_iters=15, solver="richardson", gamma=0.9)
    with GpuDomain(desc) as g:
        u, psi = empty_grid(g.M), empty_gamma(g.Nb)
        st = kfbi.kfbi_neumann_solve(g.h, 64.0, None, None, dev(_dn_gpu(mf.helm_exp_grad(g.zx, g.zy, 3.0, 4.0), g)),
                                     u, psi, opts={"fixed_iters": 15, "solver": "richardson", "gamma": 0.9})
        U = host(u).reshape(g.M + 1, g.M + 1)
        PSI = host(psi)
    assert st["iters"] == 15
    assert rel_err(PSI, psi_ref) < TOL
    assert rel_err(U, U_ref, od.inside) < TOL


def test_neumann_second_order_on_512_grid():
    """A property at a size the oracle is not run at: the error against
    exp(3x + 4y) falls by more than 3 from the 256 to the 512 grid."""
    errs = []
    for M in (256, 512):
        desc = W.domains.star(0.5, 0.1, 5, 1.0, M, M)
        x = W.grid_coords(1.0, M)
        X, Y = np.meshgrid(x, x)
        with GpuDomain(desc) as g:
            u = empty_grid(M)
            st = kfbi.kfbi_neumann_solve(g.h, 25.0, None, None,
                                         dev(_dn_gpu(mf.helm_exp_grad(g.zx, g.zy, 3.0, 4.0), g)), u)
            inside = (kfbi.kfbi_domain_copy_classification(g.h) & 1).astype(bool)
            assert st["converged"]
            ex = mf.helm_exp_u(X, Y, 3.0, 4.0)
            errs.append(np.max(np.abs(host(u).reshape(M + 1, M + 1) - ex)[inside]) / np.max(np.abs(ex[inside])))
    assert errs[1] < errs[0] / 3.0 and errs[1] < 2e-4, errs


def test_neumann_heat_steps_match_oracle():
    desc = DOMAINS["c1_disk64"]
    od = Domain(desc)
    X, Y, zx, zy = od.X, od.Y, od.colloc["x"], od.colloc["y"]
    tau = od.h
    ref = HeatStepper(od, tau, mf.heat_u(X, Y, 0), mf.heat_lap(X, Y, 0), mf.heat_u(zx, zy, 0), mf.heat_lap(zx, zy, 0),
                      tol=1e-12, bc="neumann")
    with GpuDomain(desc) as g:
        gx, gy = g.zx, g.zy
        s = kfbi.kfbi_stepper_create(g.h, kfbi.KFBI_HEAT, tau, bc=kfbi.KFBI_BC_NEUMANN)
        kfbi.kfbi_stepper_init(s, dev(mf.heat_u(X, Y, 0).ravel()), dev(mf.heat_lap(X, Y, 0).ravel()),
                               dev(mf.heat_u(gx, gy, 0)), dev(mf.heat_lap(gx, gy, 0)))
        u = empty_grid(g.M)
        for n in range(5):
            t0, t1 = n * tau, (n + 1) * tau
            Ur = ref.step(_dn_oracle(mf.heat_grad(zx, zy, t1), od), mf.heat_src(X, Y, t0) + mf.heat_src(X, Y, t1),
                          mf.heat_src(zx, zy, t0) + mf.heat_src(zx, zy, t1))
            st = kfbi.kfbi_step_heat(s, dev(_dn_gpu(mf.heat_grad(gx, gy, t1), g)),
                                     dev((mf.heat_src(X, Y, t0) + mf.heat_src(X, Y, t1)).ravel()),
                                     dev(mf.heat_src(gx, gy, t0) + mf.heat_src(gx, gy, t1)), u, opts={"tol": 1e-12})
            assert st["converged"]
            assert rel_err(host(u).reshape(g.M + 1, g.M + 1), Ur, od.inside) < TOL, n
        kfbi.kfbi_stepper_destroy(s)


def test_neumann_wave_steps_match_oracle():
    desc = DOMAINS["c2_star128"]
    od = Domain(desc)
    X, Y, zx, zy = od.X, od.Y, od.colloc["x"], od.colloc["y"]
    tau = 4.0 * od.h
    ref = WaveStepper(od, tau, mf.wave_u(X, Y, 0), mf.wave_lap(X, Y, 0), mf.wave_u(zx, zy, 0), mf.wave_lap(zx, zy, 0),
                      mf.wave_u(X, Y, -tau), mf.wave_lap(X, Y, -tau), mf.wave_u(zx, zy, -tau),
                      mf.wave_lap(zx, zy, -tau), tol=1e-12, bc="neumann")
    with GpuDomain(desc) as g:
        gx, gy = g.zx, g.zy
        s = kfbi.kfbi_stepper_create(g.h, kfbi.KFBI_WAVE, tau, theta=0.25, bc=kfbi.KFBI_BC_NEUMANN)
        kfbi.kfbi_stepper_init(s, dev(mf.wave_u(X, Y, 0).ravel()), dev(mf.wave_lap(X, Y, 0).ravel()),
                               dev(mf.wave_u(gx, gy, 0)), dev(mf.wave_lap(gx, gy, 0)),
                               dev(mf.wave_u(X, Y, -tau).ravel()), dev(mf.wave_lap(X, Y, -tau).ravel()),
                               dev(mf.wave_u(gx, gy, -tau)), dev(mf.wave_lap(gx, gy, -tau)))
        u = empty_grid(g.M)
        for n in range(5):
            t1 = (n + 1) * tau
            Ur = ref.step(_dn_oracle(mf.wave_grad(zx, zy, t1), od))
            st = kfbi.kfbi_step_wave(s, dev(_dn_gpu(mf.wave_grad(gx, gy, t1), g)), u, opts={"tol": 1e-12})
            assert st["converged"]
            assert rel_err(host(u).reshape(g.M + 1, g.M + 1), Ur, od.inside) < TOL, n
        kfbi.kfbi_stepper_destroy(s)


def test_neumann_schrodinger_steps_match_oracle():
    """Free Schroedinger solution with its du/dn on the ellipse."""
    desc = DOMAINS["c3_ellipse128"]
    od = Domain(desc)
    X, Y, zx, zy = od.X, od.Y, od.colloc["x"], od.colloc["y"]
    tau = od.h / 2
    zg, zgam = np.zeros(X.shape), np.zeros(od.Nb)
    ref = SchrodingerStepper(od, tau, mf.schr_free_u(X, Y, 0), mf.schr_free_lap(X, Y, 0), mf.schr_free_u(zx, zy, 0),
                             mf.schr_free_lap(zx, zy, 0), zg, zgam, tol=1e-12, bc="neumann")
    with GpuDomain(desc, cplx=True) as g:
        gx, gy = g.zx, g.zy
        s = kfbi.kfbi_stepper_create(g.h, kfbi.KFBI_SCHRODINGER, tau, bc=kfbi.KFBI_BC_NEUMANN)
        kfbi.kfbi_stepper_init(s, dev(mf.schr_free_u(X, Y, 0).ravel()), dev(mf.schr_free_lap(X, Y, 0).ravel()),
                               dev(mf.schr_free_u(gx, gy, 0)), dev(mf.schr_free_lap(gx, gy, 0)))
        u = empty_grid(g.M, cplx=True)
        for n in range(5):
            t1 = (n + 1) * tau
            Ur = ref.step(_dn_oracle(mf.schr_free_grad(zx, zy, t1), od))
            st = kfbi.kfbi_step_schrodinger(s, dev(_dn_gpu(mf.schr_free_grad(gx, gy, t1), g)), u,
                                            opts={"tol": 1e-12})
            assert st["converged"]
            assert rel_err(host(u).reshape(g.M + 1, g.M + 1), Ur, od.inside) < TOL, n
        kfbi.kfbi_stepper_destroy(s)


def test_neumann_refusals():
    desc = DOMAINS["c1_disk64"]
    with GpuDomain(desc) as g:
        u = empty_grid(g.M)
        with pytest.raises(kfbi.KfbiError) as e:
            kfbi.kfbi_neumann_solve(g.h, 0.0, None, None, dev(np.zeros(g.Nb)), u)
        assert e.value.code == kfbi.KFBI_EINVAL
        tau = g.info["h"]
        sn = kfbi.kfbi_stepper_create(g.h, kfbi.KFBI_HEAT, tau, bc=kfbi.KFBI_BC_NEUMANN)
        sd = kfbi.kfbi_stepper_create(g.h, kfbi.KFBI_HEAT, tau)
        x = W.grid_coords(1.0, g.M)
        X, Y = np.meshgrid(x, x)
        for s in (sn, sd):
            kfbi.kfbi_stepper_init(s, dev(mf.heat_u(X, Y, 0).ravel()), dev(mf.heat_lap(X, Y, 0).ravel()),
                                   dev(mf.heat_u(g.zx, g.zy, 0)), dev(mf.heat_lap(g.zx, g.zy, 0)))
        # a Dirichlet checkpoint does not restart a Neumann stepper
        with pytest.raises(kfbi.KfbiError):
            kfbi.kfbi_stepper_set_state(sn, kfbi.kfbi_stepper_get_state(sd))
        b = kfbi.kfbi_batch_create([g.h])
        try:
            with pytest.raises(kfbi.KfbiError) as e:
                kfbi.kfbi_batch_step(b, [sn], [dev(np.zeros(g.Nb))], [u])
            assert e.value.code == kfbi.KFBI_ENOTSUP
        finally:
            kfbi.kfbi_batch_destroy(b)
        with pytest.raises(kfbi.KfbiError) as e:
            p = kfbi.StepParams(tau=tau, bc=7)
            h = kfbi._P()
            import ctypes
            kfbi._check(kfbi.lib().kfbi_stepper_create(g.h, kfbi.KFBI_HEAT, ctypes.byref(p), ctypes.byref(h)))
        assert e.value.code == kfbi.KFBI_EINVAL
        kfbi.kfbi_stepper_destroy(sn)
        kfbi.kfbi_stepper_destroy(sd)
