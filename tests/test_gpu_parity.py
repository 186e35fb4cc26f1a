"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded synthetic inputs.

Bars: node classification and irregular-node lists bit-exact; crossings and
collocation geometry to 1e-13; every floating-point result of the FP64 path
within 1e-10 relative (the FP64 tolerance of the path; most land near 1e-13), with GMRES
run for the same fixed number of iterations on both sides where the
iteration itself is compared (reading R20).
"""

import numpy as np
import pytest

import workloads as W
from workloads import manufactured as mf
from oracle import bie, boxsolve, interface
from oracle.geometry import Domain

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
    "c2_star512": W.domain_c2_wave(512),
    "c2_star256_nb2M": W.domain_c2_wave(256, Nb=512),
    "c3_ellipse256": W.domain_c3_schrodinger(256),
    "c4_inst0": W.domain_c4_instance(0)[0],
    "c4_inst1": W.domain_c4_instance(1)[0],
    "c4_inst5": W.domain_c4_instance(5)[0],
    "star_even_lobes": W.domains.star(0.45, 0.09, 4, 1.0, 128, 256),
    "offcentre_disk": W.domains.disk(0.4, 1.0, 64, 100, cx=0.1, cy=-0.05),
}


@pytest.mark.parametrize("name", sorted(DOMAINS))
def test_classification_bit_exact(name):
    desc = DOMAINS[name]
    od = Domain(desc)
    with GpuDomain(desc) as g:
        fl = kfbi.kfbi_domain_copy_classification(g.h)
        assert np.array_equal((fl & 1).astype(bool), od.inside)
        assert np.array_equal((fl & 2).astype(bool), od.irregular)
        assert g.info["n_inside"] == int(od.inside.sum())
        assert g.info["n_irregular"] == int(od.irregular.sum())
        assert g.info["n_edges"] == len(od.edge_p)


@pytest.mark.parametrize("name", ["c1_disk64", "c2_star512", "c3_ellipse256", "c4_inst1"])
def test_crossings_and_collocation_points(name):
    desc = DOMAINS[name]
    od = Domain(desc)
    with GpuDomain(desc) as g:
        pq, xyt = kfbi.kfbi_domain_copy_edges(g.h)
        ins = od.inside.ravel()
        opin = np.where(ins[od.edge_p], od.edge_p, od.edge_q)
        opout = np.where(ins[od.edge_p], od.edge_q, od.edge_p)
        ref = {(int(a), int(b)): e for e, (a, b) in enumerate(zip(opin, opout))}
        assert len(ref) == len(pq)
        for e in range(len(pq)):
            k = ref[(int(pq[e, 0]), int(pq[e, 1]))]
            assert abs(xyt[e, 0] - od.edge_X[k]) < 1e-13
            assert abs(xyt[e, 1] - od.edge_Y[k]) < 1e-13
            dth = abs(xyt[e, 2] - od.edge_theta[k])
            assert min(dth, 2 * np.pi - dth) < 1e-12
        assert np.max(np.abs(g.zx - od.colloc["x"])) < 1e-14
        assert np.max(np.abs(g.zy - od.colloc["y"])) < 1e-14


@pytest.mark.parametrize("M,kappa", [(16, 0.0), (64, 64.0), (256, 4.0 * 256 * 256 / 4), (128, 2j * 1024)])
def test_grid_solve_matches_oracle(M, kappa):
    cplx = isinstance(kappa, complex)
    rng = np.random.default_rng(M)
    desc = W.domains.disk(0.3, 1.0, M, 64)
    R = rng.standard_normal((M + 1, M + 1))
    if cplx:
        R = R + 1j * rng.standard_normal((M + 1, M + 1))
    h = 2.0 / M
    ref = np.zeros_like(R)
    ref[1:-1, 1:-1] = boxsolve.solve(R[1:-1, 1:-1], h, kappa)
    if M <= 16:
        assert rel_err(ref[1:-1, 1:-1], boxsolve.solve_dense(R[1:-1, 1:-1], h, kappa)) < 1e-12
    with GpuDomain(desc, cplx) as g:
        out = empty_grid(M, cplx)
        kfbi.kfbi_grid_solve(g.h, kappa, dev(R.ravel(), cplx), out)
        U = host(out).reshape(M + 1, M + 1)
    assert rel_err(U, ref) < 1e-12


def _phi(theta):
    return np.cos(3 * theta) + 0.3 * np.sin(7 * theta) + 0.1


@pytest.mark.parametrize("name,kappa", [("c1_disk64", 64.0), ("c2_star128", 4.0 * 64 * 64),
                                         ("c2_star512", 1000.0), ("c3_ellipse256", 2j * 512),
                                         ("c2_star256_nb2M", 300.0)])
@pytest.mark.parametrize("with_f", [False, True])
def test_interface_apply_matches_oracle(name, kappa, with_f):
    desc = DOMAINS[name]
    cplx = isinstance(kappa, complex)
    od = Domain(desc)
    phi = _phi(od.theta) * (1.0 + 0.5j if cplx else 1.0)
    f = mf.helm_trig_f(od.X, od.Y, kappa) if with_f else None
    fg_o = mf.helm_trig_f(od.colloc["x"], od.colloc["y"], kappa) if with_f else None
    U_ref, P_ref = interface.interface_solve(od, kappa, f, fg_o, phi)
    with GpuDomain(desc, cplx) as g:
        M, Nb = g.M, g.Nb
        u = empty_grid(M, cplx)
        up = empty_gamma(Nb, cplx)
        fgrid = dev(f.ravel(), cplx) if with_f else None
        fgam = dev(mf.helm_trig_f(g.zx, g.zy, kappa), cplx) if with_f else None
        kfbi.kfbi_interface_apply(g.h, kappa, fgrid, fgam, dev(phi, cplx), u, up)
        U = host(u).reshape(M + 1, M + 1)
        P = host(up)
    assert rel_err(U, U_ref) < 1e-12
    assert rel_err(P, P_ref) < 1e-12


@pytest.mark.parametrize("name,kappa", [("c1_disk64", 64.0), ("c2_star128", 500.0),
                                         ("c3_ellipse256", 2j * 512)])
def test_helmholtz_solve_fixed_iterations(name, kappa):
    """Same number of GMRES iterations on both sides: same density and
    solution to rounding."""
    desc = DOMAINS[name]
    cplx = isinstance(kappa, complex)
    od = Domain(desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    U_ref, phi_ref, st_ref = bie.helmholtz_solve(
        od, kappa, mf.helm_trig_f(od.X, od.Y, kappa), mf.helm_trig_f(zx, zy, kappa),
        mf.helm_trig_u(zx, zy) + 0j * cplx, fixed_iters=12)
    with GpuDomain(desc, cplx) as g:
        M, Nb = g.M, g.Nb
        u = empty_grid(M, cplx)
        phi = empty_gamma(Nb, cplx)
        st = kfbi.kfbi_helmholtz_solve(
            g.h, kappa, dev(mf.helm_trig_f(od.X, od.Y, kappa).ravel(), cplx),
            dev(mf.helm_trig_f(g.zx, g.zy, kappa), cplx), dev(mf.helm_trig_u(g.zx, g.zy), cplx), u, phi,
            opts={"fixed_iters": 12})
        U = host(u).reshape(M + 1, M + 1)
        PHI = host(phi)
    assert st["iters"] == st_ref["iters"] == 12
    assert abs(st["rel_resid"] - st_ref["rel_resid"]) <= 1e-3 * st_ref["rel_resid"] + 1e-14
    assert rel_err(PHI, phi_ref) < TOL
    assert rel_err(U, U_ref, od.inside) < TOL


@pytest.mark.parametrize("name,kappa", [("c2_star128", 64.0), ("c4_inst1", None)])
def test_helmholtz_solve_to_tolerance(name, kappa):
    desc = DOMAINS[name]
    if kappa is None:
        desc, kappa, _ = W.domain_c4_instance(1)
    od = Domain(desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    U_ref, phi_ref, st_ref = bie.helmholtz_solve(
        od, kappa, mf.helm_trig_f(od.X, od.Y, kappa), mf.helm_trig_f(zx, zy, kappa),
        mf.helm_trig_u(zx, zy), tol=1e-12)
    with GpuDomain(desc) as g:
        M, Nb = g.M, g.Nb
        u = empty_grid(M)
        st = kfbi.kfbi_helmholtz_solve(
            g.h, kappa, dev(mf.helm_trig_f(od.X, od.Y, kappa).ravel()),
            dev(mf.helm_trig_f(g.zx, g.zy, kappa)), dev(mf.helm_trig_u(g.zx, g.zy)), u,
            opts={"tol": 1e-12})
        U = host(u).reshape(M + 1, M + 1)
    assert st["converged"] and st["rel_resid"] <= 1e-12
    assert abs(st["iters"] - st_ref["iters"]) <= 1
    assert rel_err(U, U_ref, od.inside) < 1e-10


def test_helmholtz_warm_start_and_restart():
    desc = DOMAINS["c2_star128"]
    kappa = 200.0
    od = Domain(desc)
    g_o = mf.helm_trig_u(od.colloc["x"], od.colloc["y"])
    U_ref, phi_ref, _ = bie.helmholtz_solve(od, kappa, None, None, g_o, tol=1e-13, restart=5)
    with GpuDomain(desc) as g:
        u = empty_grid(g.M)
        phi = empty_gamma(g.Nb)
        st = kfbi.kfbi_helmholtz_solve(g.h, kappa, None, None, dev(mf.helm_trig_u(g.zx, g.zy)), u, phi,
                                       opts={"tol": 1e-13, "restart": 5})
        assert st["converged"] and st["iters"] > 5
        assert rel_err(host(phi), phi_ref) < 1e-10
        # warm start from the converged density: converged at once
        st2 = kfbi.kfbi_helmholtz_solve(g.h, kappa, None, None, dev(mf.helm_trig_u(g.zx, g.zy)), u, phi,
                                        opts={"tol": 1e-10})
        assert st2["iters"] == 0 and st2["converged"]
        assert rel_err(host(u).reshape(g.M + 1, g.M + 1), U_ref, od.inside) < 1e-10


def test_noconvergence_is_reported():
    desc = DOMAINS["c2_star128"]
    with GpuDomain(desc) as g:
        u = empty_grid(g.M)
        st = kfbi.kfbi_helmholtz_solve(g.h, 100.0, None, None, dev(mf.helm_trig_u(g.zx, g.zy)), u,
                                       opts={"max_iter": 2, "tol": 1e-14})
        assert not st["converged"] and st["iters"] == 2
        assert np.all(np.isfinite(host(u)))


def test_domain_errors():
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.kfbi_domain_create(W.domains.disk(0.97, 1.0, 64, 128))
    assert e.value.code == kfbi.KFBI_EDOMAIN
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.kfbi_domain_create(W.domains.disk(0.5, 1.0, 100, 128))
    assert e.value.code == kfbi.KFBI_EINVAL
    with pytest.raises(kfbi.KfbiError) as e:
        kfbi.kfbi_domain_create(W.domains.disk(0.5, 1.0, 64, 4))
    assert e.value.code == kfbi.KFBI_EDOMAIN
