"""Autotuner for the propagation kernel's tiling.

Candidates: the z-segment length per thread (through the block size
N1 N2 N3 / ZL), the occupancy target (waves per SIMD, i.e. the register
budget), bands per workgroup and k-points per workgroup.  Each candidate is
timed with HIP events on a sample of the workload (the first instance of each
grid shape, a slice of its k-points) for a few steps; the fastest per update
wins.  Results are cached in a JSON file keyed by the grid shapes, band counts
and precision.
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
        if N3 % z:
            continue
        b = (N1 * N2 * (N3 // z) + 63) // 64 * 64
        if 64 <= b <= 1024:
            blocks.append(b)
    for b in sorted(set(blocks)):
        waves = (4,) if b > 512 else (2, 4)
        for w in waves:
            for bpg in sorted({0, max(1, inst.n_bands // 2)}):
                out.append({"block_size": b, "waves_per_simd": w, "bands_per_group": bpg, "k_per_group": 1})
    return out


def tune(instances: Sequence, precision: str = "fp32", steps: int = 3, k_sample: int = 64,
         cache: Optional[str] = DEFAULT_CACHE, verbose: bool = False, max_candidates: int = 12) -> Dict:
    """Returns the Propagator tiling options with the best measured updates/s."""
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
    # sample: the first instance of the most common grid shape, with a slice of its k-points
    shapes = {}
    for inst in instances:
        shapes.setdefault(tuple(inst.grid), []).append(inst)
    main = max(shapes.values(), key=len)[0]
    from .kpoints import from_spec
    kf = from_spec(main.kspec)[:k_sample]
    u = W.random_orbitals_torch(7, len(kf), main.n_bands, main.grid, main.omega)
    A = W.Field("kick", 1e-3).table(steps + 2, 0.02)
    upd = len(kf) * main.n_bands * main.ng
    results = []
    for opts in candidates(main, precision)[:max_candidates]:
        try:
            with Propagator([main], k_fracs=[kf], precision=precision, **opts) as p:
                p.load_orbitals(0, u)
                p.step(A[:2])
                t = p.time_kernels(A[2:2 + steps])["propagate_ms"]
        except Exception as exc:  # a tiling the library rejects for this shape
            if verbose:
                print(f"autotune: {opts} rejected ({exc})")
            continue
        rate = upd / (t * 1e-3)
        results.append((rate, opts))
        if verbose:
            print(f"autotune: {opts} -> {rate:.3e} updates/s")
    del u
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
