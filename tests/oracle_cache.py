"""Disk cache of oracle results for the large test graphs.

A result is computed by the oracle alone and stored as an .npz (no pickles) under the
directory named by HYTM_ORACLE_CACHE, keyed by a caller's tag plus hashes of the oracle's
and the generator's sources, so a change to either recomputes it.  Without the variable
nothing is cached and every call computes.
"""
import hashlib
import os

import numpy as np

import gen
import oracle


def _oracle_tag() -> str:
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(oracle.__file__))
    for f in ("oracle.c", "__init__.py"):
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cached(tag: str, compute):
    """compute() -> an array or a tuple of arrays / ints, through the cache when enabled."""
    root = os.environ.get("HYTM_ORACLE_CACHE")
    if not root:
        return compute()
    path = os.path.join(root, f"{tag}-{_oracle_tag()}-{gen.source_tag()}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            items = [z[f"a{i}"] for i in range(len(z.files) - 1)]
            return items[0] if int(z["single"]) else tuple(
                int(x) if x.shape == () and x.dtype.kind in "iu" else x for x in items)
    res = compute()
    single = not isinstance(res, tuple)
    items = [res] if single else list(res)
    os.makedirs(root, exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}.npz"
    np.savez(tmp, single=np.array(int(single)), **{f"a{i}": np.asarray(x) for i, x in enumerate(items)})
    os.replace(tmp, path)
    return res
