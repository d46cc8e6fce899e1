"""N_H convergence harness of the two-step scheme (Sec. II.B procedure, Sec. III.A).

Runs the N_H sub-simulations of a two-step workload together on the GPU (one
batched Propagator), records every sub-simulation's delta J_m(t), and tabulates
how the dielectric function of the average converges with the number of shifts:
for N_H = 1, 2, 4, ... the largest deviation from the full average and the mean
standard error of Im eps over the frequency window (the error bars of the
paper's Fig. 6; with random shifts they are a true standard error).

    python -m paper_2112_00920_amd.harness --workload twostep_g16_mp8_halton64 --steps 1000

Starting orbitals are the seeded smooth random orbitals of the workloads module;
with --ground-state N the library first relaxes them towards the Kohn-Sham ground
state (imaginary-time iterations), without it the table exercises the machinery
only (random orbitals are not stationary).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import Propagator, spectra


def run_two_step(instances, A, dt, precision="fp32", orbitals=None, log=None, ground_state=None):
    """Propagate all sub-simulations over the rows of A ([n][2][3]); returns
    (delta J per sub-simulation [N_H, n, 3], wall seconds of the propagation, ground-state
    residuals or None).  orbitals(i, inst) returns the starting orbitals of sub-simulation i;
    ground_state = (n_iter, tau, mix) first prepares the ground state from them."""
    import torch

    with Propagator(instances, precision=precision, dt=dt) as prop:
        for i, inst in enumerate(instances):
            u = orbitals(i, inst)
            prop.load_orbitals(i, u)
            del u
            if log and (i + 1) % 16 == 0:
                log(f"loaded {i + 1}/{len(instances)} sub-simulations")
        res = None
        if ground_state is not None and ground_state[0] > 0:
            n_it, tau, mix = ground_state
            done = 0
            while done < n_it:
                m = min(100, n_it - done)
                res = prop.ground_state(m, tau, mix)
                done += m
                if log:
                    log(f"ground state: {done}/{n_it} iterations, max residual {np.max(res):.3e}")
        t0 = time.perf_counter()
        chunk = 500
        for s in range(0, len(A), chunk):
            prop.step(A[s:s + chunk])
            if log:
                torch.cuda.synchronize()  # the library's stream is one of the device's
                log(f"step {min(s + chunk, len(A))}/{len(A)}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return prop.current(), wall, res


def table(t, dj, k0, omega, gamma=0.005, axis=0):
    rows = spectra.nh_convergence(t, dj, k0, omega, gamma=gamma, axis=axis)
    return [{"n_h": r["n_h"], "max_dev_eps": r["dev"],
             "mean_sem_im_eps": float(np.mean(r["eps_sem"].imag)),
             "max_sem_im_eps": float(np.max(r["eps_sem"].imag))} for r in rows]


def main(argv=None):
    import workloads as W

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="twostep_g16_mp8_halton64")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--n-sub", type=int, default=0, help="use only the first N sub-simulations")
    ap.add_argument("--omega", default="0.05:1.0:40", help="lo:hi:count in Ha")
    ap.add_argument("--ground-state", type=int, default=0, metavar="N",
                    help="first run N imaginary-time ground-state iterations")
    ap.add_argument("--tau", type=float, default=0.1, help="imaginary time step (Ha^-1)")
    ap.add_argument("--mix", type=float, default=0.5, help="linear density mixing")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    wl = W.config(a.workload)
    insts = wl.instances[: a.n_sub] if a.n_sub > 0 else wl.instances
    A = wl.field.table(a.steps, wl.dt)
    dj, wall, gres = run_two_step(insts, A, wl.dt, a.precision,
                                  lambda i, inst: W.random_orbitals_torch(2000 + i, inst.n_k, inst.n_bands,
                                                                          inst.grid, inst.omega), log,
                                  (a.ground_state, a.tau, a.mix))
    lo, hi, n = a.omega.split(":")
    om = np.linspace(float(lo), float(hi), int(n))
    t = wl.dt * np.arange(1, a.steps + 1)
    res = {"workload": wl.name, "sub_simulations": len(insts), "steps": a.steps, "precision": a.precision,
           "propagation_s": wall, "k0": wl.field.k0,
           "ground_state": None if gres is None else {"iterations": a.ground_state, "tau": a.tau, "mix": a.mix,
                                                      "max_residual": float(np.max(gres))}, "omega_Ha": [float(lo), float(hi), int(n)],
           "table": table(t, dj, wl.field.k0, om)}
    print(json.dumps(res))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
