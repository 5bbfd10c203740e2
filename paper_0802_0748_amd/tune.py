"""Autotuner for the launch shape of the shifted-COCG solver.

Two parameters set the shape of the dominant kernel (the deferred per-shift update):
the block length T (iterations whose updates are applied in one pass) and the number
of shifts one workgroup walks through.  The tuner times short fixed-iteration solves
of the caller's problem for each candidate on the device (HIP events inside the
library) and keeps the fastest per iteration.  Results are cached in a JSON file keyed
by the device kind and the problem signature (n, stored entries, right-hand sides, shifts,
precision).
"""

import json
import os
import tempfile
import time

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "scocg", "tune.json")
BLOCKS = (16, 24, 32, 40, 48)
SHIFTS_PER_WG = (32, 64)


def _key(H, n_rhs, n_shift, precision, device):
    """The problem signature, prefixed by the device's architecture and compute-unit count (a
    cache in a shared home directory may be read on another kind of GPU)."""
    prop = torch.cuda.get_device_properties(device)
    arch = getattr(prop, "gcnArchName", prop.name).split(":")[0]
    return f"{arch}_cu{prop.multi_processor_count}_n{H.n}_nnz{H.nnz}_K{n_rhs}_M{n_shift}_{precision}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(H: "api.Hamiltonian", z, B: torch.Tensor, precision="fp64", iters=64, cache=DEFAULT_CACHE,
         blocks=BLOCKS, shifts_per_wg=SHIFTS_PER_WG, force=False, verbose=False):
    """Return {'block': T, 'shifts_per_wg': G, 'ms_per_iter': t} for this problem shape."""
    K, M = B.shape[0], len(z)
    key = _key(H, K, M, precision, B.device)
    table = _load(cache) if cache else {}
    if not force and key in table:
        return table[key]
    out = torch.empty((K, M, H.n), dtype=torch.complex128, device=B.device)
    best = None
    results = []
    for tb in blocks:
        for g in shifts_per_wg:
            if g > M and g != shifts_per_wg[0]:
                continue
            n_it = max(iters, 2 * tb)
            n_it -= n_it % tb
            api.shifted_cocg_solve(H, z, B, out=out, fixed_iter=n_it, seed_index=0, block=tb, shifts_per_wg=g,
                                   precision=precision)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.shifted_cocg_solve(H, z, B, out=out, fixed_iter=n_it, seed_index=0, block=tb, shifts_per_wg=g,
                                   precision=precision)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / n_it
            results.append((tb, g, ms))
            if verbose:
                print(f"[tune] block {tb:2d} shifts/wg {g:3d}: {ms:.4f} ms/iteration", flush=True)
            if best is None or ms < best["ms_per_iter"]:
                best = {"block": tb, "shifts_per_wg": g, "ms_per_iter": ms}
    del out
    best["candidates"] = [list(r) for r in results]
    if cache:
        _store(cache, key, best)
    return best


def _store(path, key, entry):
    """Add one entry to the cache file.  Each writer fills a temporary file of its own and
    renames it over the cache, so concurrent tuners never leave a torn file (the last rename
    wins; a lost entry is only re-tuned)."""
    d = os.path.dirname(path) or "."
    os.makedirs(d, exist_ok=True)
    table = _load(path)
    table[key] = entry
    fd, tmp = tempfile.mkstemp(prefix=".tune-", suffix=".json", dir=d)
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(table, f, indent=1)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise
