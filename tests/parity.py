"""Error measures of the GPU parity tests (a helper module, not a test file).

rel:    relative L2 over all particles, ||x - x_ref|| / ||x_ref|| (rows of a
        field count as 3-vectors);
maxrel: the worst single particle against the typical size of the
        reference, max_i |x_i - x_ref,i| / rms_i |x_ref,i|.  A global L2 norm
        can hide an error confined to a few leaves; this cannot.

Bounds of maxrel next to the relative-L2 bounds of the same comparisons:
FP64 path vs the oracle FMM 1e-9 (next to 1e-11); mixed path vs the oracle
FMM 2e-4 (next to 1e-5): an error of 3e-4 of the rms in a single leaf fails.
"""
import numpy as np

MAX_FP64 = 1e-9
MAX_MIXED = 2e-4


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    d = a - b
    if d.ndim == 2:
        dn, bn = np.linalg.norm(d, axis=1), np.linalg.norm(b, axis=1)
    else:
        dn, bn = np.abs(d), np.abs(b)
    rms = np.sqrt(np.mean(bn * bn))
    return float(np.max(dn) / rms) if len(dn) else 0.0
