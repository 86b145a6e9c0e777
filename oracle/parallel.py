"""Oracle TSQR over several worker processes (test infrastructure: timing the
oracle on all host cores, and full-size oracle runs in tests).

The binary tree of oracle.tsqr pairs factors (0, 1), (2, 3), ... at every
level.  A run of 2^L consecutive leaves that starts at a multiple of 2^L is
therefore reduced, within the first L levels, exactly as reduce_tree reduces
that run on its own, and becomes one node of level L; a shorter run at the end
of the list does the same (its odd factors move up unchanged).  So each worker
factors one aligned run of leaves with oracle.tsqr.leaf_factors and
reduce_tree, and the parent applies reduce_tree to the run results: the
same operations in the same order as oracle.tsqr.tsqr_r, hence the same R,
bit for bit.  Workers read X from shared memory; nothing here changes the
oracle's arithmetic.
"""

import multiprocessing
import os
from multiprocessing import shared_memory

import numpy as np

from . import tsqr


def host_cores():
    """CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _run(args):
    name, shape, dtype, r0, r1, leaf_rows = args
    import threadpoolctl
    shm = shared_memory.SharedMemory(name=name)
    X = None
    try:
        X = np.ndarray(shape, dtype=dtype, buffer=shm.buf)
        with threadpoolctl.threadpool_limits(1):      # one thread per worker
            return tsqr.reduce_tree(tsqr.leaf_factors(X[r0:r1], leaf_rows))
    finally:
        del X
        shm.close()


class OraclePool:
    """A pool of `workers` spawned processes (none of them touches a GPU) that
    runs the oracle TSQR on a matrix placed in shared memory.  Create it before
    the parent initialises a GPU; close() releases the processes and memory."""

    def __init__(self, workers):
        self.workers = int(workers)
        self._pool = multiprocessing.get_context("spawn").Pool(self.workers)
        self._shm = None

    def load(self, X):
        """Copy X (rows x n, any float dtype) into shared memory."""
        X = np.ascontiguousarray(X)
        self._free()
        self._shm = shared_memory.SharedMemory(create=True, size=max(1, X.nbytes))
        buf = np.ndarray(X.shape, dtype=X.dtype, buffer=self._shm.buf)
        buf[...] = X
        self._shape, self._dtype = X.shape, X.dtype
        del buf

    def tsqr_r(self, leaf_rows=1000, run_leaves=None):
        """oracle.tsqr.tsqr_r of the loaded matrix (same R bit for bit)."""
        m = self._shape[0]
        leaves = (m + leaf_rows - 1) // leaf_rows
        if run_leaves is None:            # a power of two giving a few runs per worker
            run_leaves = 1
            while run_leaves * 4 * self.workers < leaves:
                run_leaves *= 2
        if run_leaves & (run_leaves - 1):
            raise ValueError("run_leaves must be a power of two")
        span = run_leaves * leaf_rows
        tasks = [(self._shm.name, self._shape, self._dtype, r0, min(m, r0 + span), leaf_rows)
                 for r0 in range(0, m, span)]
        return tsqr.reduce_tree(self._pool.map(_run, tasks, chunksize=1))

    def _free(self):
        if self._shm is not None:
            self._shm.close()
            self._shm.unlink()
            self._shm = None

    def close(self):
        self._free()
        self._pool.close()
        self._pool.join()
