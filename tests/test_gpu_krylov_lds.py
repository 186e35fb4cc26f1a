"""GPU parity of the GMRES control kernel when the Krylov basis no longer
fits in LDS: past nvl staged vectors (nvl = (128 KiB - m^2 w - Nb w) /
(Nb w), w the element size) its Gram-Schmidt passes read the remaining
basis vectors from global memory.  Fixed iteration counts on both sides
below and beyond nvl, real and complex, against the oracle.
"""

import numpy as np
import pytest

import workloads as W
from workloads import manufactured as mf
from oracle import bie
from oracle.geometry import Domain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2404_14864_amd import kfbi  # noqa: E402
from tests.gpu_util import GpuDomain, dev, empty_gamma, empty_grid, host, rel_err  # noqa: E402

TOL = 1e-10


def _nvl(Nb, es, m=50):
    hb, vb = m * m * es, Nb * es
    return min((131072 - hb - vb) // vb, m + 1)


@pytest.mark.parametrize("case", ["cplx512_staged", "cplx512_beyond", "cplx1024_beyond", "real2048_beyond"])
def test_fixed_iterations_across_lds_staging(case):
    if case.startswith("cplx512"):
        desc, kappa = W.domain_nls_example(512), 128j
        iters = 8 if case.endswith("staged") else 14
    elif case == "cplx1024_beyond":
        desc, kappa, iters = W.domain_c3_schrodinger(1024), 2j * 1024, 8
    else:
        desc, kappa, iters = W.domain_c2_wave(2048), 1000.0, 6
    cplx = isinstance(kappa, complex)
    nvl = _nvl(desc["Nb"], 16 if cplx else 8)
    assert (iters <= nvl) == case.endswith("staged"), (iters, nvl)
    od = Domain(desc)
    zx, zy = od.colloc["x"], od.colloc["y"]
    g_ref = mf.helm_trig_u(zx, zy) + 0j * cplx
    U_ref, phi_ref, st_ref = bie.helmholtz_solve(od, kappa, mf.helm_trig_f(od.X, od.Y, kappa),
                                                 mf.helm_trig_f(zx, zy, kappa), g_ref, fixed_iters=iters)
    with GpuDomain(desc, cplx) as g:
        u, phi = empty_grid(g.M, cplx), empty_gamma(g.Nb, cplx)
        st = kfbi.kfbi_helmholtz_solve(g.h, kappa, dev(mf.helm_trig_f(od.X, od.Y, kappa).ravel(), cplx),
                                       dev(mf.helm_trig_f(g.zx, g.zy, kappa), cplx),
                                       dev(mf.helm_trig_u(g.zx, g.zy), cplx), u, phi, opts={"fixed_iters": iters})
        U = host(u).reshape(g.M + 1, g.M + 1)
        PHI = host(phi)
    assert st["iters"] == iters
    assert abs(st["rel_resid"] - st_ref["rel_resid"]) <= 1e-3 * st_ref["rel_resid"] + 1e-14, (st, st_ref)
    assert rel_err(PHI, phi_ref) < TOL
    assert rel_err(U, U_ref, od.inside) < TOL
