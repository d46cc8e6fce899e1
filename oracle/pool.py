"""Oracle (test infrastructure only): the explicit Taylor-4 run of ``oracle.propagate.Run``
spread over host processes by k-point.

The arithmetic is that of ``oracle.propagate`` unchanged -- per k the Taylor step
(Eq. (1)), the band sums of the density (Eq. (3)) and of <u|pi|u> (Eqs. (5)-(6)) --
and of ``oracle.hxc`` for v_Hxc.  Eqs. (3) and (5) are sums over the k-set with the
weights of Eq. (7), so the k-set is cut into contiguous blocks, one per worker, each
worker returns its block's partial sums, and the parent adds them in block order and
applies the Hxc update.  Only the order of the k-sum differs from ``Run`` (rounding).

Workers are forked from the parent (no exec) and inherit the System and the initial
orbitals; they never import anything beyond NumPy and this package.  A process that
has initialised a GPU must not fork them.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from .hxc import v_hxc as hxc_potential
from .propagate import current_k, taylor_step


def _block_sums(sys, kappa_shift, u, ks):
    """Partial density and current of the k-points ks (weights w_k, occupations f_b)."""
    rho = np.zeros(sys.cell.shape)
    j = np.zeros(3)
    for i, k in enumerate(ks):
        rho += sys.wk[k] * np.einsum("b,bijl->ijl", sys.occ, np.abs(u[i]) ** 2)
        j += sys.wk[k] * current_k(sys, sys.k_cart[k] + kappa_shift, u[i])
    return rho, j


def _worker(conn, sys, u_all, ks, dt):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except Exception:
        pass
    u = np.array(u_all[ks[0]:ks[-1] + 1], dtype=complex)
    while True:
        msg = conn.recv()
        if msg[0] == "stop":
            conn.close()
            return
        if msg[0] == "observe":  # partial sums at kappa = k + A
            conn.send(_block_sums(sys, np.asarray(msg[1], float), u, ks))
        elif msg[0] == "step":   # Taylor step of the block with v_Hxc, then partial sums at A_end
            _, a_mid, a_end, v = msg
            for i, k in enumerate(ks):
                u[i] = taylor_step(sys, sys.k_cart[k] + np.asarray(a_mid, float), v, u[i], dt)
            conn.send(_block_sums(sys, np.asarray(a_end, float), u, ks))
        elif msg[0] == "get":
            conn.send(u)


class PoolRun:
    """A single TDDFT simulation (as ``oracle.propagate.Run`` with the explicit Taylor step)
    whose k-points are spread over `workers` forked processes."""

    def __init__(self, sys, u0, dt, hxc_mode="scf", v_hxc_frozen=None, workers=None):
        self.sys = sys
        self.dt = float(dt)
        self.mode = hxc_mode
        n = workers or len(os.sched_getaffinity(0))
        n = max(1, min(n, sys.nk))
        bounds = np.linspace(0, sys.nk, n + 1).round().astype(int)
        self.blocks = [list(range(bounds[i], bounds[i + 1])) for i in range(n) if bounds[i + 1] > bounds[i]]
        ctx = mp.get_context("fork")
        self.conns, self.procs = [], []
        for ks in self.blocks:
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(b, sys, u0, ks, self.dt), daemon=True)
            p.start()
            b.close()
            self.conns.append(a)
            self.procs.append(p)
        rho, jsum = self._gather(("observe", np.zeros(3)))
        if hxc_mode == "scf":
            self.v_hxc = hxc_potential(sys.cell, rho)
        elif hxc_mode == "frozen":
            self.v_hxc = np.asarray(v_hxc_frozen, float).reshape(sys.cell.shape)
        elif hxc_mode == "none":
            self.v_hxc = np.zeros(sys.cell.shape)
        else:
            raise ValueError(hxc_mode)
        self.J_pre = -jsum / sys.cell.omega

    def _gather(self, msg):
        for c in self.conns:
            c.send(msg)
        rho = np.zeros(self.sys.cell.shape)
        j = np.zeros(3)
        for c in self.conns:  # block order
            r, jj = c.recv()
            rho += r
            j += jj
        return rho, j

    def step(self, A_mid, A_end):
        rho, jsum = self._gather(("step", A_mid, A_end, self.v_hxc))
        if self.mode == "scf":
            self.v_hxc = hxc_potential(self.sys.cell, rho)
        return -jsum / self.sys.cell.omega

    def run(self, A_tab):
        out = np.empty((len(A_tab), 3))
        for n in range(len(A_tab)):
            out[n] = self.step(A_tab[n, 0], A_tab[n, 1])
        return out

    def orbitals(self):
        for c in self.conns:
            c.send(("get",))
        return np.concatenate([c.recv() for c in self.conns], axis=0)

    def close(self):
        for c, p in zip(self.conns, self.procs):
            try:
                c.send(("stop",))
            except (BrokenPipeError, OSError):
                pass
            p.join(timeout=10)
            if p.is_alive():
                p.kill()
        self.conns, self.procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
