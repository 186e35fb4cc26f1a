"""GPU tests of the two tridiagonal kernels of the grid solve (eq. 3.31's
y-direction solves with a sparse right-hand side, section 3.4): the LDS-tile
kernel and the register-row kernel form every value by the same operations
in the same order, so a solve gives the same bits whichever the launch-shape
timing keeps.  The environment variable KFBI_TRIDIAG_KERNEL limits that
timing to one kernel; each case solves the same problem on two domains, one
timed with each.

Bar: bit-for-bit equality of U and phi (FP64, complex128, and the mixed
solves' FP32 / complex64 inner kernels), single domains and batches (whose
dense-input launches also have a register-row form), and the register-row
kernel kept by the batch timing when it is the only one allowed.  Inputs: the heat, wave, Schroedinger and batched workloads'
domains (ellipse and star), seeded smooth random f and g.
"""

import os

import numpy as np
import pytest

import workloads as W
from workloads.fields import SmoothField

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2404_14864_amd import kfbi  # noqa: E402
from tests.gpu_util import dev, empty_gamma, empty_grid, host  # noqa: E402


class _Kernel:
    """Limits the launch-shape timing to one tridiagonal kernel."""

    def __init__(self, which):
        self.which = which

    def __enter__(self):
        self.old = os.environ.get("KFBI_TRIDIAG_KERNEL")
        os.environ["KFBI_TRIDIAG_KERNEL"] = self.which

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("KFBI_TRIDIAG_KERNEL", None)
        else:
            os.environ["KFBI_TRIDIAG_KERNEL"] = self.old


def _data(desc, cplx, seed):
    rng = np.random.default_rng(seed)
    fr, fi, gr, gi = (SmoothField(rng) for _ in range(4))
    M = desc["M"]
    x = W.grid_coords(1.0, M)
    X, Y = np.meshgrid(x, x)

    def f(a, b):
        return fr(a, b) + 1j * fi(a, b) if cplx else fr(a, b)

    def g(a, b):
        return gr(a, b) + 1j * gi(a, b) if cplx else gr(a, b)

    return f, g, X, Y


def _solve(desc, cplx, kappa, which, seed, **opts):
    with _Kernel(which):
        h = kfbi.kfbi_domain_create(desc, kfbi.KFBI_COMPLEX if cplx else kfbi.KFBI_REAL)
        try:
            zx, zy = kfbi.kfbi_domain_copy_boundary(h)
            f, g, X, Y = _data(desc, cplx, seed)
            u, phi = empty_grid(desc["M"], cplx), empty_gamma(desc["Nb"], cplx)
            st = kfbi.kfbi_helmholtz_solve(h, kappa, dev(f(X, Y).ravel()), dev(f(zx, zy)), dev(g(zx, zy)), u, phi,
                                           opts=opts)
            return host(u), host(phi), st["iters"]
        finally:
            kfbi.kfbi_domain_destroy(h)


CASES = [
    ("wave 512 real", W.domain_c2_wave(512), False, 40.0),
    ("heat 256 real", W.domain_c1_heat(256), False, 12.0),
    ("batched-workload instance 1024 real", W.domain_c4_instance(3, grids=(1024,))[0], False, 25.0),
    ("Schroedinger 1024 complex", W.domain_c3_schrodinger(1024), True, 2j * 1024.0),
    ("Schroedinger 256 complex", W.domain_c3_schrodinger(256), True, 300.0 + 900.0j),
]


@pytest.mark.parametrize("name,desc,cplx,kappa", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [kfbi.KFBI_PREC_FP64, kfbi.KFBI_PREC_MIXED], ids=["fp64", "mixed"])
def test_single_solve_same_bits_with_either_kernel(name, desc, cplx, kappa, precision):
    print("case", name, "precision", precision, flush=True)
    opts = {"fixed_iters": 12, "precision": precision} if precision == kfbi.KFBI_PREC_FP64 else \
        {"tol": 1e-10, "precision": precision}
    ut, pt, it_t = _solve(desc, cplx, kappa, "tile", 11, **opts)
    ur, pr, it_r = _solve(desc, cplx, kappa, "rows", 11, **opts)
    assert it_t == it_r
    assert np.all(np.isfinite(ut))
    assert np.array_equal(ut, ur)
    assert np.array_equal(pt, pr)


def test_eight_mode_row_choice_leaves_dense_launches_valid():
    """The register-row kernel timed at 8 modes per workgroup (512 lanes) on
    a 2048 grid: the dense-input launches of the b-solve and the final solve
    run the tile kernel at its own default shape, and the solve gives the
    tile kernel's bits."""
    desc = W.domain_c2_wave(2048)
    opts = {"fixed_iters": 6}
    ut, pt, _ = _solve(desc, False, 40.0, "tile", 5, **opts)
    ur, pr, _ = _solve(desc, False, 40.0, "rows:8", 5, **opts)
    assert np.all(np.isfinite(ut))
    assert np.array_equal(ut, ur)
    assert np.array_equal(pt, pr)


def test_batch_same_bits_with_either_kernel():
    descs = [W.domain_c4_instance(q, grids=(256, 512, 1024))[0] for q in range(6)]
    runs = {}
    for which in ("tile", "rows"):
        with _Kernel(which):
            hs = [kfbi.kfbi_domain_create(d, kfbi.KFBI_REAL) for d in descs]
            b = None
            try:
                b = kfbi.kfbi_batch_create(hs)
                fs, fgs, ggs, us = [], [], [], []
                for q, (d, h) in enumerate(zip(descs, hs)):
                    zx, zy = kfbi.kfbi_domain_copy_boundary(h)
                    f, g, X, Y = _data(d, False, 100 + q)
                    fs.append(dev(f(X, Y).ravel()))
                    fgs.append(dev(f(zx, zy)))
                    ggs.append(dev(g(zx, zy)))
                    us.append(empty_grid(d["M"]))
                kap = [10.0 + 5.0 * q for q in range(len(descs))]
                kfbi.kfbi_batch_helmholtz(b, kap, fs, fgs, ggs, us, opts={"fixed_iters": 10})
                tuning = kfbi.kfbi_batch_tuning(b)
                runs[which] = ([host(u) for u in us], tuning)
            finally:
                if b is not None:
                    kfbi.kfbi_batch_destroy(b)
                for h in hs:
                    kfbi.kfbi_domain_destroy(h)
    for a, c in zip(runs["tile"][0], runs["rows"][0]):
        assert np.array_equal(a, c)
    # the register-row kernel served the sparse launches and, in its dense-input
    # form, the b-solve's and final solve's launches of every class it fits
    for kind in ("sparse64", "dense64"):
        rows = [r["register_rows"] for r in runs["rows"][1] if r["tuned"] and r["kind"] == kind]
        assert rows and all(rows), kind
    assert not any(r["register_rows"] for r in runs["tile"][1])
