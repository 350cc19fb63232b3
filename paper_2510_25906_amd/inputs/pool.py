"""Fork-based process pool for the input generators (mesh-sized numpy work that
splits into independent cell ranges).

The shared read-only state is published in a module global before the fork,
so the workers inherit it instead of receiving pickled copies.  Forking is
only safe in a process that has not initialised a GPU: generate inputs before
any device call.
"""
from __future__ import annotations

SHARED = None


def pool_map(fn, items, workers=1, shared=None):
    """[fn(item) for item in items], in ``workers`` forked processes when
    workers > 1; ``fn`` reads ``shared`` from ``pool.SHARED``."""
    global SHARED
    SHARED = shared
    try:
        if workers > 1 and len(items) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(min(workers, len(items))) as p:
                return p.map(fn, items)
        return [fn(it) for it in items]
    finally:
        SHARED = None
