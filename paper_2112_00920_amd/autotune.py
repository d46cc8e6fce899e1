"""Autotuner for the propagation kernel's tiling.

Candidates: the z-segment length per thread (through the block size
N1 N2 N3 / ZL), the occupancy target (waves per SIMD, i.e. the register
budget), bands per workgroup and k-points per workgroup.  Each candidate is
timed with HIP events on a sample of the workload (instances of the most common
grid shape with at least `min_items` k-points in all, so that the sample fills the
GPU as the workload does) for a few steps; the fastest per update wins.  Results
are cached in a JSON file keyed by the grid shapes, band counts and precision.
tune_classes does this per shape class of an uneven batch (grid, lattice kind, band
count) and returns per-class tiling rules for the library.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "tdks_autotune.json")
_ZLS = (2, 3, 4, 6, 8, 10, 12, 16)


def _key(instances, precision) -> str:
    shapes = sorted({(tuple(i.grid), i.n_bands, i.cell) for i in instances})
    return json.dumps({"precision": precision, "shapes": shapes})


def candidates(inst, precision) -> List[Dict]:
    """Tilings the library has kernels for, for one grid shape."""
    N1, N2, N3 = inst.grid
    out = []
    blocks = []
    for z in _ZLS:
        nseg = -(-N3 // z)  # the last segment of a column may be shorter
        b = (N1 * N2 * nseg + 63) // 64 * 64
        if 64 <= b <= 1024:
            blocks.append(b)
    for b in sorted(set(blocks)):
        waves = (4,) if b > 512 else (2, 4)
        for w in waves:
            for bpg in sorted({0, max(1, inst.n_bands // 2)}):
                for kpg in ((1, 4) if inst.n_k >= 4 else (1,)):
                    out.append({"block_size": b, "waves_per_simd": w, "bands_per_group": bpg, "k_per_group": kpg})
    return out


def tune(instances: Sequence, precision: str = "fp32", steps: int = 3, min_items: int = 2048,
         cache: Optional[str] = DEFAULT_CACHE, verbose: bool = False, max_candidates: int = 32) -> Dict:
    """Returns the Propagator tiling options with the best measured updates/s.

    The sample is the instances of the most common grid shape, as many as it takes to
    reach `min_items` k-points (so that the sample fills the GPU the way the workload
    does), with their full k-sets."""
    import torch
    import workloads as W
    from . import Propagator

    key = _key(instances, precision)
    if cache and os.path.exists(cache):
        try:
            with open(cache) as fh:
                stored = json.load(fh)
            if key in stored:
                return stored[key]["options"]
        except (OSError, ValueError):
            pass
    shapes = {}
    for inst in instances:
        shapes.setdefault(tuple(inst.grid), []).append(inst)
    group = max(shapes.values(), key=len)
    sample, nk = [], 0
    for inst in group:
        sample.append(inst)
        nk += inst.n_k
        if nk >= min_items:
            break
    us = [W.random_orbitals_torch(7 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega)
          for i, inst in enumerate(sample)]
    A = W.Field("kick", 1e-3).table(steps + 2, 0.02)
    upd = sum(inst.n_k * inst.n_bands * inst.ng for inst in sample)
    results, seen = [], set()
    for opts in candidates(sample[0], precision)[:max_candidates]:
        try:
            with Propagator(sample, precision=precision, **opts) as p:
                til = p.tiling()
                sig = (til["block"], til["zl"], til["waves_per_simd"], til["bands_per_group"], til["k_per_group"])
                if sig in seen:  # the library maps this request onto a tiling already measured
                    continue
                seen.add(sig)
                for i, u in enumerate(us):
                    p.load_orbitals(i, u)
                p.step(A[:2])
                t = p.time_kernels(A[2:2 + steps])["propagate_ms"]
        except Exception as exc:  # a tiling the library rejects for this shape
            if verbose:
                print(f"autotune: {opts} rejected ({exc})")
            continue
        rate = upd / (t * 1e-3)
        results.append((rate, opts))
        if verbose:
            print(f"autotune: {opts} (tiling {til}) -> {rate:.3e} updates/s")
    del us
    torch.cuda.empty_cache()
    if not results:
        return {}
    best = max(results, key=lambda x: x[0])[1]
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            stored = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    stored = json.load(fh)
            stored[key] = {"options": best, "updates_per_s": max(r for r, _ in results)}
            with open(cache, "w") as fh:
                json.dump(stored, fh, indent=1)
        except (OSError, ValueError):
            pass
    return best


def _nonorth(inst) -> int:
    """1 when the lattice rows are not mutually orthogonal (mixed derivatives in the stencil)."""
    L = np.asarray(inst.lattice, float)
    G = L @ L.T
    return int(np.any(np.abs(G - np.diag(np.diag(G))) > 1e-12 * np.max(np.abs(G))))


def _class_key(inst):
    return (tuple(int(g) for g in inst.grid), _nonorth(inst), int(inst.n_bands))


def tune_classes(instances: Sequence, precision: str = "fp32", steps: int = 3, min_items: int = 2048,
                 cache: Optional[str] = DEFAULT_CACHE, verbose: bool = False,
                 max_candidates: int = 32) -> List[Dict]:
    """Tunes every shape class of a batch on its own (grid, lattice kind, band count): the
    instances of the class, as many as it takes to reach `min_items` k-points, are timed
    under each candidate tiling, and the fastest becomes a tiling rule for that class.
    Returns the rules for Propagator(..., tiling_rules=...); each class is cached under its
    own key, so batches that share a class share its result."""
    groups: Dict = {}
    for inst in instances:
        groups.setdefault(_class_key(inst), []).append(inst)
    rules = []
    for (grid, nonorth, nb), members in groups.items():
        opts = tune(members, precision, steps=steps, min_items=min_items, cache=cache, verbose=verbose,
                    max_candidates=max_candidates)
        rule = {"grid": list(grid), "nonorth": nonorth, "n_bands": nb}
        rule.update({k: int(v) for k, v in opts.items()})
        if verbose:
            print(f"autotune class grid {grid} nonorth {nonorth} bands {nb}: {rule}")
        rules.append(rule)
    return rules
