"""MI355X (gfx950) real-time TDKS propagation with two-step Brillouin-zone
sampling (Sato, arXiv:2112.00920) -- thin Python binding of libtdks.so.

Every step of the method runs in the library's HIP kernels; this module only
marshals arguments, hands PyTorch's device allocator and current stream to the
library, and builds k-point sets and spectra on the host.  It raises
ImportError when libtdks.so is missing; there is no CPU fallback.

    import paper_2112_00920_amd as tdks
    prop = tdks.Propagator(instances, precision="fp32", dt=0.02)
    prop.load_orbitals(i, u)            # complex128 [k][band][N3][N2][N1]
    prop.step(A_tab)                    # [n][2][3]: A(t_n + dt/2), A(t_{n+1})
    dj = prop.current(per="group")      # delta J, averaged per two-step group
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from . import kpoints, spectra
from ._lib import TdksError

__all__ = ["Propagator", "TdksError", "kpoints", "spectra", "instance_arrays"]


def instance_arrays(inst, k_frac=None):
    """Host arrays describing one instance (from a workloads.Instance)."""
    kf = kpoints.from_spec(inst.kspec) if k_frac is None else np.asarray(k_frac, float)
    return {
        "lattice": np.ascontiguousarray(inst.lattice, dtype=np.float64),
        "grid": tuple(int(g) for g in inst.grid),
        "atom_frac": np.ascontiguousarray(inst.atom_frac, dtype=np.float64).reshape(-1, 3),
        "atom_species": np.ascontiguousarray(inst.atom_species, dtype=np.int32),
        "species": list(inst.species),
        "k_frac": np.ascontiguousarray(kf, dtype=np.float64).reshape(-1, 3),
        "n_bands": int(inst.n_bands),
        "group": int(inst.group),
    }


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class _TorchAllocator:
    """Routes the library's device allocations through PyTorch's caching allocator."""

    def __init__(self):
        import torch

        self.torch = torch

        def alloc(nbytes, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
            except Exception:  # out of memory -> NULL, reported by the library
                return None

        def free(ptr, user):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = _lib.ALLOC_FN(alloc)
        self.free = _lib.FREE_FN(free)


class Propagator:
    """A set of independent TDDFT simulations advanced together on one GPU."""

    def __init__(self, instances: Sequence, k_fracs: Optional[Sequence] = None, precision: str = "fp64",
                 dt: float = 0.02, hxc_mode: str = "scf", v_hxc_frozen: Optional[Sequence] = None,
                 bands_per_group: int = 0, k_per_group: int = 0, block_size: int = 0,
                 graph_steps: int = 16, waves_per_simd: int = 0, use_torch: bool = True,
                 propagator: str = "taylor", norm_stride: int = 0, record_stride: int = 1,
                 tiling_rules: Optional[Sequence[dict]] = None):
        self._lib = _lib.load()
        self._ctx = None
        self.n_inst = len(instances)
        self.precision = precision
        self.dt = float(dt)
        self.arrays = [instance_arrays(inst, None if k_fracs is None else k_fracs[i])
                       for i, inst in enumerate(instances)]
        descs = (_lib.InstanceDesc * self.n_inst)()
        keep = []
        for i, a in enumerate(self.arrays):
            d = descs[i]
            for j, v in enumerate(a["lattice"].ravel()):
                d.lattice[j] = float(v)
            for j in range(3):
                d.grid[j] = a["grid"][j]
            d.n_atoms = len(a["atom_frac"])
            d.atom_frac = _ptr(a["atom_frac"])
            d.atom_species = _ptr(a["atom_species"], ctypes.c_int)
            sp = (_lib.Species * max(1, len(a["species"])))()
            for j, s in enumerate(a["species"]):
                sp[j] = _lib.Species(s.D, s.w, s.rc, s.Rc, s.Es, s.Ep)
            keep.append(sp)
            d.n_species = len(a["species"])
            d.species = sp
            d.n_k = len(a["k_frac"])
            d.k_frac = _ptr(a["k_frac"])
            d.k_weight = None
            d.n_bands = a["n_bands"]
            d.occ = None
            d.group = a["group"]
            if v_hxc_frozen is not None:
                vf = np.ascontiguousarray(v_hxc_frozen[i], dtype=np.float64).ravel()
                keep.append(vf)
                d.v_hxc_frozen = _ptr(vf)
            else:
                d.v_hxc_frozen = None
        opt = _lib.Options()
        self._lib.tdks_default_options(ctypes.byref(opt))
        opt.precision = {"fp64": _lib.FP64, "fp32": _lib.FP32_MIXED}[precision]
        opt.dt = self.dt
        opt.hxc_mode = {"scf": _lib.HXC_SCF, "frozen": _lib.HXC_FROZEN, "none": _lib.HXC_NONE}[hxc_mode]
        opt.bands_per_group = int(bands_per_group)
        opt.k_per_group = int(k_per_group)
        opt.block_size = int(block_size)
        opt.graph_steps = int(graph_steps)
        opt.propagator = {"taylor": _lib.PROP_TAYLOR, "pc": _lib.PROP_PC}[propagator]
        opt.waves_per_simd = int(waves_per_simd)
        opt.norm_stride = int(norm_stride)
        opt.record_stride = int(record_stride)
        self.record_stride = max(1, int(record_stride))
        if tiling_rules:
            # per-shape tilings (the autotuner's per-class results): grid, nonorth (-1 any),
            # n_bands (0 any) and the tiling fields, 0 = the context's option
            rules = (_lib.TilingRule * len(tiling_rules))()
            for j, r in enumerate(tiling_rules):
                for q in range(3):
                    rules[j].grid[q] = int(r["grid"][q])
                rules[j].nonorth = int(r.get("nonorth", -1))
                rules[j].n_bands = int(r.get("n_bands", 0))
                for f in ("block_size", "waves_per_simd", "bands_per_group", "k_per_group"):
                    setattr(rules[j], f, int(r.get(f, 0)))
            keep.append(rules)
            opt.tiling_rules = rules
            opt.n_tiling_rules = len(tiling_rules)
        self._alloc = None
        self._torch = None
        if use_torch:
            try:
                import torch
                if torch.cuda.is_available():
                    self._torch = torch
            except ImportError:
                self._torch = None
        if self._torch is not None:
            self._alloc = _TorchAllocator()
            opt.alloc = self._alloc.alloc
            opt.free = self._alloc.free
            opt.stream = ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)
        ctx = ctypes.c_void_p()
        _lib.check(self._lib.tdks_create(descs, self.n_inst, ctypes.byref(opt), ctypes.byref(ctx)))
        self._ctx = ctx
        self._keep = keep

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        if self._ctx is not None:
            self._lib.tdks_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ helpers
    def _shape(self, i):
        a = self.arrays[i]
        N1, N2, N3 = a["grid"]
        return (len(a["k_frac"]), a["n_bands"], N3, N2, N1)

    def _pointer_of(self, u, expect_shape):
        """(pointer, where, keepalive) for a complex128 array (numpy or torch cuda)."""
        if self._torch is not None and isinstance(u, self._torch.Tensor):
            if u.dtype != self._torch.complex128 or not u.is_contiguous():
                u = u.to(self._torch.complex128).contiguous()
            if tuple(u.shape) != tuple(expect_shape):
                raise ValueError(f"orbital shape {tuple(u.shape)} != {expect_shape}")
            if u.is_cuda:
                return ctypes.c_void_p(u.data_ptr()), _lib.DEVICE, u
            u = u.numpy()
        arr = np.ascontiguousarray(u, dtype=np.complex128)
        if arr.shape != tuple(expect_shape):
            raise ValueError(f"orbital shape {arr.shape} != {expect_shape}")
        return ctypes.c_void_p(arr.ctypes.data), _lib.HOST, arr

    # ------------------------------------------------------------------ ABI calls
    def load_orbitals(self, i: int, u):
        p, where, keep = self._pointer_of(u, self._shape(i))
        _lib.check(self._lib.tdks_load_orbitals(self._ctx, i, p, where))

    def step(self, A_tab):
        A = np.ascontiguousarray(A_tab, dtype=np.float64).reshape(-1, 2, 3)
        _lib.check(self._lib.tdks_step(self._ctx, len(A), _ptr(A)))

    def step_noalloc(self, A_dev, j_dev):
        """tdks_step_noalloc: A_dev and j_dev are float64 device tensors [n][2][3] and
        [n_inst][n][3] (contiguous); j_dev receives J^{n+1} of every step of the call."""
        t = self._torch
        if t is None or not (isinstance(A_dev, t.Tensor) and isinstance(j_dev, t.Tensor)):
            raise TypeError("step_noalloc takes torch device tensors")
        n = A_dev.shape[0]
        for x, shape in ((A_dev, (n, 2, 3)), (j_dev, (self.n_inst, n, 3))):
            if not (x.is_cuda and x.dtype == t.float64 and x.is_contiguous() and tuple(x.shape) == shape):
                raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")
        _lib.check(self._lib.tdks_step_noalloc(self._ctx, int(n), ctypes.c_void_p(A_dev.data_ptr()),
                                               ctypes.c_void_p(j_dev.data_ptr())))

    def ground_state(self, n_iter: int, tau: float, mix: float = 0.5) -> np.ndarray:
        """Imaginary-time ground-state preparation of every instance (tdks_ground_state);
        returns the last iteration's density residual per instance."""
        res = np.zeros(self.n_inst)
        _lib.check(self._lib.tdks_ground_state(self._ctx, int(n_iter), float(tau), float(mix), _ptr(res)))
        return res

    @property
    def steps_done(self) -> int:
        return int(self._lib.tdks_steps_done(self._ctx))

    def check(self) -> np.ndarray:
        """Health records of every instance (tdks_check; raises TdksError E_NUMERIC on a
        violation, with the records in the exception's `info`)."""
        info = (ctypes.c_ulonglong * self.n_inst)()
        rc = self._lib.tdks_check(self._ctx, info)
        rec = np.array(list(info), dtype=np.uint64)
        if rc != _lib.TDKS_OK:
            err = TdksError(rc, self._lib.tdks_last_error().decode(errors="replace"))
            err.info = rec
            raise err
        return rec

    def current(self, per: str = "instance") -> np.ndarray:
        ns = self.steps_done // self.record_stride
        mode = _lib.PER_GROUP if per == "group" else _lib.PER_INSTANCE
        rows = len(set(a["group"] for a in self.arrays)) if per == "group" else self.n_inst
        out = np.zeros((rows, ns, 3))
        n = ctypes.c_size_t()
        _lib.check(self._lib.tdks_current(self._ctx, mode, _ptr(out), out.size, ctypes.byref(n)))
        return out

    def current_pre(self) -> np.ndarray:
        out = np.zeros((self.n_inst, 3))
        _lib.check(self._lib.tdks_current_pre(self._ctx, _ptr(out)))
        return out

    def current_at(self, A) -> np.ndarray:
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(3)
        out = np.zeros((self.n_inst, 3))
        _lib.check(self._lib.tdks_current_at(self._ctx, _ptr(A), _ptr(out)))
        return out

    def density(self, i: int) -> np.ndarray:
        N1, N2, N3 = self.arrays[i]["grid"]
        out = np.zeros((N3, N2, N1))
        _lib.check(self._lib.tdks_density(self._ctx, i, _ptr(out)))
        return out

    def vhxc(self, i: int) -> np.ndarray:
        N1, N2, N3 = self.arrays[i]["grid"]
        out = np.zeros((N3, N2, N1))
        _lib.check(self._lib.tdks_vhxc(self._ctx, i, _ptr(out)))
        return out

    def vloc(self, i: int) -> np.ndarray:
        N1, N2, N3 = self.arrays[i]["grid"]
        out = np.zeros((N3, N2, N1))
        _lib.check(self._lib.tdks_vloc(self._ctx, i, _ptr(out)))
        return out

    def get_orbitals(self, i: int) -> np.ndarray:
        out = np.zeros(self._shape(i), dtype=np.complex128)
        _lib.check(self._lib.tdks_get_orbitals(self._ctx, i, ctypes.c_void_p(out.ctypes.data), _lib.HOST))
        return out

    def norms(self, i: int) -> np.ndarray:
        nk, nb = self._shape(i)[:2]
        out = np.zeros((nk, nb))
        _lib.check(self._lib.tdks_norms(self._ctx, i, _ptr(out)))
        return out

    def apply_h(self, i: int, w, A=(0.0, 0.0, 0.0)) -> np.ndarray:
        p, where, keep = self._pointer_of(w, self._shape(i))
        out = np.zeros(self._shape(i), dtype=np.complex128)
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(3)
        if where == _lib.DEVICE:
            dev = self._torch.empty(self._shape(i), dtype=self._torch.complex128, device=keep.device)
            _lib.check(self._lib.tdks_apply_h(self._ctx, i, p, ctypes.c_void_p(dev.data_ptr()), _ptr(A),
                                              _lib.DEVICE))
            return dev.cpu().numpy()
        _lib.check(self._lib.tdks_apply_h(self._ctx, i, p, ctypes.c_void_p(out.ctypes.data), _ptr(A), _lib.HOST))
        return out

    def time_kernels(self, A_tab) -> dict:
        """Advance len(A_tab) steps with HIP events around the kernels (ms per step)."""
        A = np.ascontiguousarray(A_tab, dtype=np.float64).reshape(-1, 2, 3)
        out = np.zeros(3)
        _lib.check(self._lib.tdks_time_kernels(self._ctx, len(A), _ptr(A), _ptr(out)))
        return {"propagate_ms": out[0], "reduce_hxc_ms": out[1], "step_ms": out[2]}

    def tiling(self) -> dict:
        v = [ctypes.c_int() for _ in range(6)]
        _lib.check(self._lib.tdks_tiling(self._ctx, *[ctypes.byref(x) for x in v]))
        return dict(zip(["block", "zl", "waves_per_simd", "bands_per_group", "k_per_group", "n_groups"],
                        [x.value for x in v]))
