"""Error norms of the numerical examples (section 4; TEST INFRASTRUCTURE ONLY).

The paper's scaled 2-norm divides by N with N defined twice differently
(reading R18); the oracle reports the max norm and the root-mean-square
over inside nodes.
"""

import numpy as np


def max_norm(err, inside):
    return float(np.max(np.abs(err[inside]))) if np.any(inside) else 0.0


def rms_norm(err, inside):
    return float(np.sqrt(np.mean(np.abs(err[inside]) ** 2))) if np.any(inside) else 0.0
