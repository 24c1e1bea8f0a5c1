"""Seeded synthetic particle sets (positions and charges), FP64, host numpy.

This module only draws random inputs; it holds none of the method's
arithmetic and imports nothing else from the package, so the tests, the
benchmark and the CPU reference can all share it.

Distributions:
  * uniform  -- points uniform in the unit cube, the paper's benchmark
                workload (Sec. 5: random particles in a unit cube);
  * plummer  -- Plummer sphere with scale radius a = 1 truncated at r = 20
                (inverse-CDF radius, isotropic direction, no recentring);
  * batch    -- instance sizes N_k = round(2^(10 + 6 u_k)), u_k ~ U[0, 1),
                i.e. log-uniform in [1024, 65536];
  * velocities -- straight-line motion for time stepping: displacement
                directions uniform in [-1, 1]^3, scaled per particle.
Charges are uniform in [-1, 1] unless stated.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cube(n, seed):
    rng = _rng(seed)
    pos = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return pos, q


def plummer(n, seed, a=1.0, rmax=20.0, equal_charges=False):
    rng = _rng(seed)
    mmax = rmax ** 3 / (1.0 + rmax ** 2) ** 1.5   # enclosed mass fraction at rmax (a = 1)
    u = rng.uniform(0.0, mmax, n)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(1.0 - cz * cz)
    pos = np.stack([r * sz * np.cos(ph), r * sz * np.sin(ph), r * cz], axis=1)
    if equal_charges:
        q = np.full(n, 1.0 / n)
    else:
        q = rng.uniform(-1.0, 1.0, n)
    return pos, q


def velocities(n, seed, amplitude=1.0):
    """Per-particle displacement directions for synthetic time stepping:
    amplitude (a scalar or one value per particle) times a vector uniform in
    [-1, 1]^3.  Step k of a run moves particle i to pos_i + k dt v_i."""
    a = np.asarray(amplitude, dtype=np.float64)
    v = _rng(seed).uniform(-1.0, 1.0, (n, 3))
    return v * (a[:, None] if a.ndim == 1 else a)


def error_sample(n, seed, k=4096):
    """Indices of the k targets used for error estimates (without replacement)."""
    if n <= k:
        return np.arange(n, dtype=np.int64)
    return np.sort(_rng(seed + 100).choice(n, k, replace=False)).astype(np.int64)


def batch_sizes(n_inst=256, seed=5, lo_log2=10, hi_log2=16):
    u = _rng(seed).random(n_inst)
    return np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def batch(n_inst=256, seed=5):
    """Concatenated instances: even k uniform cube, odd k Plummer, charges U[-1,1].

    Returns (pos (sum N, 3), q (sum N), offsets (n_inst + 1))."""
    sizes = batch_sizes(n_inst, seed)
    ps, qs = [], []
    for k, nk in enumerate(sizes):
        if k % 2 == 0:
            p, q = uniform_cube(int(nk), 5000 + k)
        else:
            p, q = plummer(int(nk), 5000 + k)
        ps.append(p)
        qs.append(q)
    offsets = np.zeros(n_inst + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return np.concatenate(ps), np.concatenate(qs), offsets


# Named workloads (sizes, distribution, expansion order, leaf size, MAC).
WORKLOADS = {
    "uniform4k_p4": dict(n=4096, dist="uniform", seed=1, p=4, ncrit=64, theta=(1, 2)),
    "uniform1m_p8": dict(n=1048576, dist="uniform", seed=2, p=8, ncrit=64, theta=(1, 2)),
    "plummer4m_p10": dict(n=4194304, dist="plummer_equal", seed=3, p=10, ncrit=32, theta=(2, 5)),
    "plummer1m_p8": dict(n=1048576, dist="plummer", seed=4, p=8, ncrit=64, theta=(1, 2)),
}


def make(name):
    w = WORKLOADS[name]
    if w["dist"] == "uniform":
        pos, q = uniform_cube(w["n"], w["seed"])
    elif w["dist"] == "plummer":
        pos, q = plummer(w["n"], w["seed"])
    else:
        pos, q = plummer(w["n"], w["seed"], equal_charges=True)
    return pos, q, w
