"""Helpers for the GPU parity tests: device tensors from numpy arrays and
relative errors.  Inputs for both sides come from `workloads`; each side
evaluates boundary fields at its own collocation points."""

import numpy as np
import torch

from paper_2404_14864_amd import kfbi

DEV = "cuda:0"


def dev(a, cplx=False):
    a = np.ascontiguousarray(a)
    dt = torch.complex128 if (cplx or np.iscomplexobj(a)) else torch.float64
    return torch.from_numpy(a.astype(np.complex128 if dt == torch.complex128 else np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty_grid(M, cplx=False):
    return torch.zeros((M + 1) * (M + 1), dtype=torch.complex128 if cplx else torch.float64, device=DEV)


def empty_gamma(Nb, cplx=False):
    return torch.zeros(Nb, dtype=torch.complex128 if cplx else torch.float64, device=DEV)


def rel_err(a, b, mask=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a, b = a[mask], b[mask]
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


class GpuDomain:
    """Owns one library domain for a test."""

    def __init__(self, desc, cplx=False):
        self.desc = desc
        self.cplx = cplx
        self.h = kfbi.kfbi_domain_create(desc, kfbi.KFBI_COMPLEX if cplx else kfbi.KFBI_REAL)
        self.info = kfbi.kfbi_domain_get_info(self.h)
        self.M, self.Nb = desc["M"], desc["Nb"]
        self.zx, self.zy = kfbi.kfbi_domain_copy_boundary(self.h)

    def close(self):
        if self.h is not None:
            kfbi.kfbi_domain_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
