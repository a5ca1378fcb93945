"""Oracle noise statistics for large maps, spread over worker processes.

Test helper (not a test module).  The realisations 0 .. R-1 are cut into
consecutive runs; each run's (count, mean, m2) comes from
``oracle.noise_moments`` in its own process, and the runs are combined in
order with ``oracle.merge_moments``.  Nothing here does arithmetic of its
own: the result equals ``oracle.noise_sigma`` up to the rounding of the
pairwise merge (pinned in tests/test_oracle_noise.py).

Workers are started with the "spawn" method, so they never share the GPU
state of the test process; they import only numpy and the oracle.  The pool
size is min(16, os.cpu_count(), runs), or AMAP_ORACLE_WORKERS if set.
"""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import oracle as O


def _run(args):
    g1, g2, J, seed, a, b = args
    return O.noise_moments(g1, g2, J, seed, a, b)


def _workers(runs):
    env = os.environ.get("AMAP_ORACLE_WORKERS")
    w = int(env) if env else min(16, os.cpu_count() or 1)
    return max(1, min(w, runs))


def noise_moments_pool(g1, g2, J, n_real, seed, workers=None):
    """(count, mean, m2) of realisations 0 .. n_real-1, runs computed in parallel."""
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    w = workers or _workers(n_real)
    per = -(-n_real // w)
    bounds = [(a, min(a + per, n_real)) for a in range(0, n_real, per)]
    if len(bounds) == 1:
        return O.noise_moments(g1, g2, J, seed, 0, n_real)
    jobs = [(g1, g2, J, seed, a, b) for a, b in bounds]
    acc = (0, 0.0, 0.0)
    with ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        for part in ex.map(_run, jobs):  # in run order
            acc = O.merge_moments(acc, part)
    return acc


def noise_sigma_pool(g1, g2, J, n_real, seed, workers=None):
    """oracle.noise_sigma, with its realisations spread over worker processes."""
    count, _, m2 = noise_moments_pool(g1, g2, J, n_real, seed, workers)
    return O.sigma_from_moments(count, m2)
