"""The oracle's lattice step with its per-node collisions spread over worker processes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

``lbm.step`` collides every fluid node (``collision.collide`` on the batch of
nodes) and then streams.  The collision of one node depends on that node
alone, so the batch can be cut into chunks and collided in separate
processes; the chunks are joined and streamed by ``lbm.stream`` exactly as in
``lbm.step``.  No arithmetic of the method is added or changed here: the
workers run ``collision.collide`` as it stands, one chunk each.  Workers are
fresh interpreters (spawn) with one BLAS thread each, so that they neither
inherit a parent's device state nor oversubscribe the cores; a worker that
dies raises (BrokenProcessPool) instead of being replaced.
"""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import collision, lbm
from .lattice import LATTICES


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:       # the environment variables set by the parent still apply
        pass


def _collide_chunk(args):
    q, f, F, omega, per_mass = args
    return collision.collide(LATTICES[q], f, F, omega, per_mass)


class Pool:
    """A pool of `workers` processes (default: every host CPU, at most 16)."""

    def __init__(self, workers=None):
        self.workers = int(workers or min(os.cpu_count() or 1, 16))
        saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
        for k in saved:
            os.environ[k] = "1"
        try:
            self._pool = ProcessPoolExecutor(self.workers, mp_context=mp.get_context("spawn"),
                                             initializer=_init_worker)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v

    def close(self):
        self._pool.shutdown(wait=True)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def collide_field(self, lat, f, F, omega, solid=None, per_mass=False):
        """lbm.collide_field with the fluid nodes collided in chunks."""
        shape = f.shape[1:]
        fluid = lbm.fluid_mask(solid, shape)
        fn = np.moveaxis(f, 0, -1)[fluid]
        Fn = np.broadcast_to(np.asarray(F), tuple(shape) + (3,))[fluid] if np.asarray(F).ndim == 1 \
            else np.moveaxis(np.asarray(F), 0, -1)[fluid]
        omega = list(omega)
        cuts = np.array_split(np.arange(len(fn)), max(1, min(len(fn), 4 * self.workers)))
        jobs = [(lat.Q, fn[c], np.ascontiguousarray(Fn[c]), omega, per_mass) for c in cuts if len(c)]
        parts = list(self._pool.map(_collide_chunk, jobs))
        dtype = np.result_type(fn, Fn, np.asarray(omega))
        post = np.zeros(tuple(shape) + (lat.Q,), dtype=dtype)
        post[fluid] = np.concatenate(parts, axis=0) if parts else np.zeros((0, lat.Q), dtype=dtype)
        return np.moveaxis(post, -1, 0)

    def step(self, lat, f, F, omega, solid=None, per_mass=False):
        """lbm.step, collisions in the workers."""
        return lbm.stream(lat, self.collide_field(lat, f, F, omega, solid, per_mass), solid)

    def run(self, lat, f, F, omega, nsteps, solid=None, callback=None, per_mass=False):
        for n in range(nsteps):
            f = self.step(lat, f, F, omega, solid, per_mass)
            if callback is not None:
                callback(n + 1, f)
        return f
