#!/usr/bin/env python3
"""Throughput benchmark of the TDKS propagation path on one MI355X.

Headline: batched two-step propagation, 64 independent sub-simulations
(8^3 coarse Monkhorst-Pack grid x 4^3 uniform shifts, each with its own density
and Hxc), 8-atom Si-like cell on a 16^3 grid, 16 bands, complex-FP32 propagation
with FP64 density/current/Hxc, delta kick 1e-3, dt = 0.02.  One step = one
Taylor-4 step of every orbital of every sub-simulation, plus density, current,
Poisson + LDA of every sub-simulation.  Metric: k*band*gridpoint*step updates/s.

Also measured: the plain method in FP64 (one instance, direct 8^3 MP grid,
16^3, 16 bands), the FP32-vs-FP64 deviation of the two-step current over the
timed steps, the propagation kernel's device time (HIP events on the library
stream) for the roofline, and the CPU FP64 oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TF = 157.3    # MI355X published FP32 vector peak
FP64_VECTOR_PEAK_TF = 78.6
# Algorithmic work per update (one grid point of one orbital advanced one Taylor-4 step):
BYTES_PER_UPDATE = {"fp32": 16.0, "fp64": 32.0}   # read u once, write u once
FLOPS_PER_UPDATE = 700.0  # 4 x (stencil 75 + projectors 65 + Taylor 4) + density 5 + current 122


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of every source that sets the profiled launch: the kernel, its instantiations and
    dispatch, and the runtime that picks the tiling and k grouping."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2112_00920_amd", "csrc")
    names = sorted(f for f in os.listdir(csrc)
                   if f.startswith("tdks_prop") or f in ("tdks_internal.h", "tdks_runtime.cpp"))
    for f in names:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_hash and m_bytes) or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def make_two_step(n_inst):
    import workloads as W
    wl = W.config("twostep_g16_mp8_s4")
    return wl, wl.instances[:n_inst]


def load_all(prop, insts, seed0, torch):
    import workloads as W
    for i, inst in enumerate(insts):
        u = W.random_orbitals_torch(seed0 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega, device="cuda")
        prop.load_orbitals(i, u)
        del u
        if len(insts) > 16 and (i + 1) % 16 == 0:
            torch.cuda.synchronize()
            log(f"  loaded {i + 1}/{len(insts)} sub-simulations")
    torch.cuda.synchronize()


def timed_steps(prop, A, steps, warmup, torch):
    if warmup:
        prop.step(A[:warmup])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prop.step(A[warmup:warmup + steps])
    torch.cuda.synchronize()
    return time.perf_counter() - t0


CPU_POOL_MAX = 16  # worker processes of the oracle pool (the host share of one GPU)


def cpu_baseline(pool_budget_s=15.0, single_budget_s=6.0):
    """The oracle as it stands on the host cores, before anything touches the GPU (its
    workers are forked without exec).  Pool: one sub-simulation of the two-step workload at
    its full 512 k (16 bands, 16^3, SCF), k-points spread over min(affinity, 16) processes,
    density and current reduced in the parent every step (oracle.pool), timed over whole
    steps for about pool_budget_s.  Single core: the same sub-simulation restricted to 2 of
    its k-points, one process, BLAS limited to 1 thread."""
    import workloads as W
    from oracle import kpoints as okp
    from oracle import propagate as OP
    from oracle.hamiltonian import System
    from oracle.pool import PoolRun
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except Exception:
        pass
    wl = W.config("twostep_g16_mp8_s4")
    inst = wl.instances[0]
    A = wl.field.table(1000, wl.dt)
    affinity = sorted(os.sched_getaffinity(0))
    workers = max(1, min(len(affinity), CPU_POOL_MAX))
    # single core, 2 k-points
    kf = okp.kset(inst.kspec)[:2]
    run = OP.Run(System(inst, k_frac=kf), W.random_orbitals(99, 2, inst.n_bands, inst.grid, inst.omega),
                 wl.dt, "scf")
    t0 = time.perf_counter()
    n1 = 0
    while n1 < 2 or time.perf_counter() - t0 < single_budget_s:
        run.step(A[n1, 0], A[n1, 1])
        n1 += 1
    el1 = time.perf_counter() - t0
    single = 2 * inst.n_bands * inst.ng * n1 / el1
    # pool over the host cores, full k-set
    sysm = System(inst)
    u0 = W.random_orbitals(98, sysm.nk, inst.n_bands, inst.grid, inst.omega)
    with PoolRun(sysm, u0, wl.dt, "scf", workers=workers) as pr:
        t0 = time.perf_counter()
        n = 0
        while n < 1 or time.perf_counter() - t0 < pool_budget_s:
            pr.step(A[n, 0], A[n, 1])
            n += 1
        el = time.perf_counter() - t0
    upd = sysm.nk * inst.n_bands * inst.ng * n
    return {"value": upd / el, "unit": "k*band*gridpt*step updates/s", "cores": workers, "kind": "oracle",
            "sample": f"one two-step sub-simulation (16^3, 16 bands, all 512 k, SCF) as a k-parallel pool of "
                      f"{workers} forked processes, density/current reduced in the parent each step: {n} steps "
                      f"in {el:.1f} s; NumPy FP64, BLAS 1 thread per process",
            "host_cpu_count": os.cpu_count(), "affinity_cores": len(affinity),
            "single_core_value": single,
            "single_core_sample": f"same sub-simulation restricted to 2 of its 512 k-points, one process, "
                                  f"{n1} steps in {el1:.1f} s",
            "ms_per_step_full_subsim": 1e3 * el / n}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--instances", type=int, default=64, help="two-step sub-simulations (64 = full workload)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-others", action="store_true", help="leave out the HHG and uneven workloads")
    ap.add_argument("--skip-ground-state", action="store_true",
                    help="leave out the ground-state iteration measurement (keeps a profile of the "
                         "step kernel free of its launches)")
    ap.add_argument("--uneven-classes", action="store_true",
                    help="also time each shape class of the uneven batch alone (one context per class)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB -> 1 GiB device copy kernel (torch neg), so that a counter "
                         "profile of this command holds a kernel of known HBM traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the two-step sub-simulations "
              "are independent and would shard across GPUs without communication, but this build runs on one.",
              file=sys.stderr)
        sys.exit(2)

    # the oracle's host baseline first: its pool forks, which must happen before any GPU use
    cpu = None if args.skip_cpu else cpu_baseline()
    if cpu:
        log(f"  oracle: {cpu['value']:.3e} updates/s on {cpu['cores']} processes "
            f"(single core {cpu['single_core_value']:.3e})")

    import torch
    import paper_2112_00920_amd as tdks

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    K, Wm = args.steps, args.warmup
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x neg over 2^28 floats (1 GiB read + 1 GiB written per launch)")
    wl, insts = make_two_step(args.instances)
    A = wl.field.table(K + Wm + 8, wl.dt)
    n_inst = len(insts)
    upd_step = sum(i.n_k * i.n_bands * i.ng for i in insts)

    # ---- headline: batched two-step, FP32 propagation
    log(f"two-step FP32: {n_inst} sub-simulations x 512 k x 16 bands x 16^3 ({upd_step:.3e} updates/step)")
    with tdks.Propagator(insts, precision="fp32", dt=wl.dt) as prop:
        load_all(prop, insts, 1000, torch)
        til = prop.tiling()
        el = timed_steps(prop, A, K, Wm, torch)
        kt = prop.time_kernels(A[K + Wm:K + Wm + 4])
        dj32 = prop.current(per="instance")
        # ground-state preparation on the same batch (outside the timed region): a few
        # imaginary-time iterations (Taylor-4 filter, orthonormalisation, density, mixing, Hxc)
        n_gs, tau_gs = 3, 0.1
        ground = None
        if not args.skip_ground_state:
            prop.ground_state(1, tau_gs, 0.5)  # first call allocates its buffers
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res_gs = prop.ground_state(n_gs, tau_gs, 0.5)
            torch.cuda.synchronize()
            ground = {"ms_per_iteration": 1e3 * (time.perf_counter() - t0) / n_gs, "iterations": n_gs,
                      "tau": tau_gs, "mix": 0.5, "residual_max": float(np.max(res_gs)),
                      "note": "imaginary-time Taylor-4 + Cholesky orthonormalisation + density + mixing + "
                              "Hxc, all 64 sub-simulations, FP32 orbitals"}
            log(f"  ground-state iteration: {ground['ms_per_iteration']:.2f} ms")
    value = upd_step * K / el
    ms_step = 1e3 * el / K
    log(f"  {value:.3e} updates/s, {ms_step:.2f} ms/step, kernels {kt}, tiling {til}")

    # ---- roofline of the propagation kernel (one launch per step for this workload)
    upd_launch = upd_step
    t_launch = kt["propagate_ms"] * 1e-3
    flops_achieved = FLOPS_PER_UPDATE * upd_launch / t_launch / 1e12
    bytes_achieved = BYTES_PER_UPDATE["fp32"] * upd_launch / t_launch / 1e9
    traffic = profiled_traffic("propagate_twostep_g16_fp32_counters.txt")
    roofline = {"bound": "alu", "achieved": round(flops_achieved, 2), "peak": FP32_VECTOR_PEAK_TF,
                "unit": "TFLOP/s", "frac": round(flops_achieved / FP32_VECTOR_PEAK_TF, 4),
                "traffic": traffic,
                "hbm_algorithmic_GBs": round(bytes_achieved, 1),
                "hbm_algorithmic_frac": round(bytes_achieved / HBM_PEAK_GBS, 4),
                "kernel": "k_propagate (Taylor-4 step + density/current partials)",
                "flops_per_update": FLOPS_PER_UPDATE,
                "projector_mfma_frac": 0.0,
                "projector_note": "the KB projector contraction runs on the VALU (no MFMA instructions in the "
                                  "kernel), so its MFMA fraction is 0",
                "kernel_ms": round(kt["propagate_ms"], 3), "step_ms_eager": round(kt["step_ms"], 3)}

    # ---- predictor-corrector propagator (v_Hxc at the mid-step): two propagations per step
    pc = None
    if not args.skip_fp64:
        with tdks.Propagator(insts, precision="fp32", dt=wl.dt, propagator="pc") as p:
            load_all(p, insts, 1000, torch)
            Kp = max(2, K // 4)
            elp = timed_steps(p, A, Kp, 1, torch)
            ktp = p.time_kernels(A[Kp + 1:Kp + 3])
        pc = {"value": upd_step * Kp / elp, "ms_per_step": 1e3 * elp / Kp, "steps": Kp,
              "propagate_ms": ktp["propagate_ms"],
              "note": "FP32, predictor + corrector propagation, density, 2 x Hxc per step"}
        log(f"  two-step FP32 predictor-corrector: {pc['value']:.3e} updates/s")

    # ---- FP32 vs FP64 on the same inputs (first 4 sub-simulations, timed steps)
    acc = None
    fp64_twostep = None
    plain = None
    if not args.skip_fp64:
        sub = insts[:4]
        res = {}
        for prec in ("fp32", "fp64"):
            with tdks.Propagator(sub, precision=prec, dt=wl.dt) as p:
                load_all(p, sub, 1000, torch)
                p.step(A[:K + Wm])
                res[prec] = p.current(per="instance").mean(axis=0)
        ref = res["fp64"]
        acc = float(np.max(np.abs(res["fp32"] - ref)) / np.max(np.abs(ref)))
        log(f"  FP32 vs FP64 over {K + Wm} steps (mean of 4 sub-simulations): {acc:.2e} of peak |dJ|")
        # FP64 batched two-step (same workload, FP64 propagation)
        with tdks.Propagator(insts, precision="fp64", dt=wl.dt) as p:
            load_all(p, insts, 1000, torch)
            el64 = timed_steps(p, A, K, Wm, torch)
            kt64 = p.time_kernels(A[K + Wm:K + Wm + 2])
        fp64_twostep = {"value": upd_step * K / el64, "ms_per_step": 1e3 * el64 / K,
                        "kernel_ms": kt64["propagate_ms"]}
        log(f"  two-step FP64: {fp64_twostep['value']:.3e} updates/s")
        # plain method FP64: one instance, direct 8^3 MP grid
        wl2 = __import__("workloads").config("diamond8_g16_mp8")
        inst2 = wl2.instances[0]
        with tdks.Propagator([inst2], precision="fp64", dt=wl2.dt) as p:
            load_all(p, [inst2], 2000, torch)
            A2 = wl2.field.table(K + Wm, wl2.dt)
            el2 = timed_steps(p, A2, K, Wm, torch)
            kt2 = p.time_kernels(A2[:2])
        upd2 = inst2.n_k * inst2.n_bands * inst2.ng
        plain = {"workload": "diamond8_g16_mp8 (plain method, 512 k, 16 bands, 16^3, FP64)",
                 "value": upd2 * K / el2, "ms_per_step": 1e3 * el2 / K, "kernel_ms": kt2["propagate_ms"],
                 "hbm_algorithmic_frac": BYTES_PER_UPDATE["fp64"] * upd2 / (kt2["propagate_ms"] * 1e-3) / 1e9
                 / HBM_PEAK_GBS}
        log(f"  plain FP64: {plain['value']:.3e} updates/s")

    # ---- the other batched FP32 workloads: HHG two-step (64 x 64 k x 16 bands on 20^3, at the
    # pulse peak) and the uneven 40-instance batch (four shape classes launched concurrently)
    others = {}
    if not args.skip_others:
        import workloads as W
        for key, name, start in (("hhg_two_step", "hhg_twostep_g20_mp4_s4", None), ("uneven", "uneven40", 0)):
            wlo = W.config(name)
            ins = wlo.instances
            st = wlo.steps // 2 if start is None else start
            Ao = wlo.field.table(K + Wm + 4, wlo.dt, start=st)
            upd_o = sum(i.n_k * i.n_bands * i.ng for i in ins)
            with tdks.Propagator(ins, precision="fp32", dt=wlo.dt) as p:
                load_all(p, ins, 3000, torch)
                elo = timed_steps(p, Ao, K, Wm, torch)
                kto = p.time_kernels(Ao[K + Wm:K + Wm + 2])
                tilo = p.tiling()
            others[key] = {"workload": name, "value": upd_o * K / elo, "ms_per_step": 1e3 * elo / K,
                           "propagate_ms_eager": kto["propagate_ms"], "updates_per_step": upd_o,
                           "instances": len(ins), "tiling_first_class": tilo}
            log(f"  {name} FP32: {others[key]['value']:.3e} updates/s, {others[key]['ms_per_step']:.2f} ms/step")
            if key == "uneven" and args.uneven_classes:
                # each shape class (cell kind and grid) in a context of its own: its step alone
                classes = {}
                for idx, inst in enumerate(ins):
                    classes.setdefault((inst.cell, tuple(inst.grid)), []).append(idx)
                alone = {}
                for (cell, grid), idxs in classes.items():
                    sub = [ins[i] for i in idxs]
                    upd_c = sum(i.n_k * i.n_bands * i.ng for i in sub)
                    with tdks.Propagator(sub, precision="fp32", dt=wlo.dt) as p:
                        load_all(p, sub, 3000, torch)
                        elc = timed_steps(p, Ao, K, Wm, torch)
                        ktc = p.time_kernels(Ao[K + Wm:K + Wm + 2])
                        tilc = p.tiling()
                    label = f"{cell} {grid[0]}x{grid[1]}x{grid[2]}"
                    alone[label] = {"instances": len(sub), "updates_per_step": upd_c,
                                    "ms_per_step": 1e3 * elc / K, "propagate_ms_eager": ktc["propagate_ms"],
                                    "value": upd_c * K / elc, "tiling": tilc}
                    log(f"    class {label} alone ({len(sub)} instances): {1e3 * elc / K:.3f} ms/step, "
                        f"{upd_c * K / elc:.3e} updates/s, tiling {tilc}")
                others[key]["classes_alone"] = alone

    out = {
        "metric": "k*band*gridpt*step updates/s (batched FP32 two-step)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 reductions)",
        "data": "synthetic (seeded Gaussian pseudopotential, smooth random orthonormal orbitals)",
        "config": {"workload": "twostep_g16_mp8_s4", "sub_simulations": n_inst, "coarse_k": "8^3",
                   "shifts": "4^3 uniform", "bands": 16, "grid": [16, 16, 16], "atoms": 8,
                   "dt": wl.dt, "field": "kick 1e-3", "hxc": "SCF every step",
                   "updates_per_step": upd_step, "tiling": til},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_GBs_algorithmic": round(bytes_achieved, 1),
        "fp64_two_step": fp64_twostep,
        "fp64_plain": plain,
        "speedup_fp32_batched_vs_fp64_plain": (value / plain["value"]) if plain else None,
        "fp32_vs_fp64_dJ_rel_err": acc,
        "ground_state": ground,
        "predictor_corrector": pc,
        "other_workloads_fp32": others or None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
