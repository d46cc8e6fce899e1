"""Writes the golden induced currents of tests/golden/*.txt with the CPU FP64 oracle.

Each file holds delta J(t) = J(t) - J_pre (Eq. (5) with the kinetic momentum of Eq. (6),
Sec. III.A's induced current) of one instance of a workload at its full k-set, over at
least 50 explicit Taylor-4 steps (Eq. (1)) with the Hxc potential updated every step,
computed by the oracle (plain NumPy FP64, ``oracle.pool`` spreading the k-points over the
host cores).  The header's recipe line names the seeded inputs (workload, instance,
orbital seed, field window) so that a test regenerates the same inputs with ``workloads``
and compares the GPU path with these values.

    python tests/golden/make_golden.py [case ...]

Imports only ``oracle`` and ``workloads``.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.hamiltonian import System  # noqa: E402
from oracle.pool import PoolRun  # noqa: E402

STEPS = 50


def _uneven_first(kind):
    wl = W.config("uneven40")
    for i, inst in enumerate(wl.instances):
        if kind == "fcc2" and inst.cell == "fcc2":
            return i
        if kind == "super16" and inst.cell == "super16":
            return i
        if kind == "cubic16" and inst.cell == "diamond8" and inst.grid == (16, 16, 16):
            return i
        if kind == "cubic20" and inst.cell == "diamond8" and inst.grid == (20, 20, 20):
            return i
    raise KeyError(kind)


def cases():
    hhg = W.config("hhg_twostep_g20_mp4_s4")
    return {
        # plain method, 512 k, 16^3, kick
        "c2_plain_g16_mp8": dict(workload="diamond8_g16_mp8", instance=0, seed=2100, start=0),
        # one sub-simulation of the two-step batch (shift (3, 2, 1) of the 4^3 shifts), 512 k
        "c3_twostep_sub27": dict(workload="twostep_g16_mp8_s4", instance=27, seed=2300, start=0),
        # one HHG sub-simulation (20^3, 64 k) at the peak of the sin^2 pulse
        "c4_hhg_sub21_peak": dict(workload="hhg_twostep_g20_mp4_s4", instance=21, seed=2400,
                                  start=hhg.steps // 2),
        # one instance of each kind of the uneven batch
        "c5_uneven_fcc2": dict(workload="uneven40", instance=_uneven_first("fcc2"), seed=2500, start=0),
        "c5_uneven_cubic16": dict(workload="uneven40", instance=_uneven_first("cubic16"), seed=2501, start=0),
        "c5_uneven_cubic20": dict(workload="uneven40", instance=_uneven_first("cubic20"), seed=2502, start=0),
        "c5_uneven_super16": dict(workload="uneven40", instance=_uneven_first("super16"), seed=2503, start=0),
    }


def inputs(recipe):
    """(instance, initial orbitals, A table, dt) of a recipe -- the same call the tests make."""
    wl = W.config(recipe["workload"])
    inst = wl.instances[recipe["instance"]]
    u0 = W.random_orbitals(recipe["seed"], inst.n_k, inst.n_bands, inst.grid, inst.omega)
    A = wl.field.table(recipe["steps"], wl.dt, start=recipe["start"])
    return inst, u0, A, wl.dt


def write(name, recipe):
    recipe = dict(recipe, steps=STEPS)
    inst, u0, A, dt = inputs(recipe)
    t0 = time.time()
    with PoolRun(System(inst), u0, dt, "scf") as run:
        J = run.run(A)
        jpre = run.J_pre
        workers = len(run.blocks)
    dj = J - jpre
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as f:
        f.write(f"# golden induced current delta J^n = J^n - J_pre (Eqs. 5-6), n = 1..{STEPS}, of one\n")
        f.write("# instance at its full k-set, explicit Taylor-4 steps (Eq. 1) with SCF Hxc, by the CPU FP64\n")
        f.write("# oracle; written by tests/golden/make_golden.py\n")
        f.write(f"# {inst.cell} {inst.grid[0]}x{inst.grid[1]}x{inst.grid[2]}, {inst.n_k} k, {inst.n_bands} bands\n")
        f.write("# recipe: " + json.dumps(recipe) + "\n")
        f.write("# J_pre: " + " ".join(f"{x:.17e}" for x in jpre) + "\n")
        for n in range(STEPS):
            f.write(f"{n + 1} " + " ".join(f"{x:.17e}" for x in dj[n]) + "\n")
    print(f"{name}: {inst.n_k} k x {inst.n_bands} bands x {inst.ng} points, {STEPS} steps on {workers} "
          f"processes in {time.time() - t0:.1f} s; peak |dJ| {np.max(np.abs(dj)):.3e}", flush=True)


def read(name):
    """(recipe, J_pre, delta J [n][3]) of a golden file."""
    path = os.path.join(HERE, name + ".txt")
    recipe, jpre, rows = None, None, []
    with open(path) as f:
        for line in f:
            if line.startswith("# recipe: "):
                recipe = json.loads(line[len("# recipe: "):])
            elif line.startswith("# J_pre: "):
                jpre = np.array([float(x) for x in line.split()[2:]])
            elif not line.startswith("#") and line.strip():
                rows.append([float(x) for x in line.split()[1:]])
    return recipe, jpre, np.array(rows)


if __name__ == "__main__":
    todo = cases()
    names = sys.argv[1:] or list(todo)
    for nm in names:
        write(nm, todo[nm])
