"""Host-only checks of the C ABI: the library loads, exports every function that
include/tdks.h declares, the ctypes structures match the C layout, and argument
errors are reported before any device work."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_2112_00920_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdks.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdks_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (tdks_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)
    assert set(names) == set(_lib.SYMBOLS)


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "tdks.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(tdks_species), sizeof(tdks_instance_desc), sizeof(tdks_options));
  printf("%zu %zu %zu %zu\\n", offsetof(tdks_instance_desc, n_k), offsetof(tdks_instance_desc, group),
         offsetof(tdks_instance_desc, v_hxc_frozen), offsetof(tdks_instance_desc, species));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(tdks_options, stream), offsetof(tdks_options, alloc_user),
         offsetof(tdks_options, block_size), offsetof(tdks_options, graph_steps),
         offsetof(tdks_options, waves_per_simd));
  printf("%zu %zu %zu\\n", offsetof(tdks_options, propagator), offsetof(tdks_options, norm_stride),
         offsetof(tdks_options, record_stride));
  printf("%zu %zu %zu %zu\\n", offsetof(tdks_options, tiling_rules), offsetof(tdks_options, n_tiling_rules),
         sizeof(tdks_tiling_rule), offsetof(tdks_tiling_rule, k_per_group));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    D, O = _lib.InstanceDesc, _lib.Options
    assert vals[:3] == [ctypes.sizeof(_lib.Species), ctypes.sizeof(D), ctypes.sizeof(O)]
    assert vals[3:7] == [D.n_k.offset, D.group.offset, D.v_hxc_frozen.offset, D.species.offset]
    assert vals[7:12] == [O.stream.offset, O.alloc_user.offset, O.block_size.offset, O.graph_steps.offset,
                          O.waves_per_simd.offset]
    assert vals[12:15] == [O.propagator.offset, O.norm_stride.offset, O.record_stride.offset]
    assert vals[15:19] == [O.tiling_rules.offset, O.n_tiling_rules.offset, ctypes.sizeof(_lib.TilingRule),
                           _lib.TilingRule.k_per_group.offset]


def test_default_options():
    lib = _lib.load()
    opt = _lib.Options()
    lib.tdks_default_options(ctypes.byref(opt))
    assert opt.precision == _lib.FP64 and opt.taylor_order == 4 and opt.dt == 0.02
    assert opt.hxc_mode == _lib.HXC_SCF and opt.graph_steps == 16
    assert opt.norm_stride == 0 and opt.record_stride == 0


def _desc(inst, k):
    d = _lib.InstanceDesc()
    for j, v in enumerate(np.asarray(inst.lattice, float).ravel()):
        d.lattice[j] = v
    for j in range(3):
        d.grid[j] = inst.grid[j]
    frac = np.ascontiguousarray(inst.atom_frac, float)
    spc = np.zeros(len(frac), np.int32)
    sp = (_lib.Species * 1)(_lib.Species(*[getattr(inst.species[0], f) for f in ("D", "w", "rc", "Rc", "Es", "Ep")]))
    d.n_atoms = len(frac)
    d.atom_frac = frac.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.atom_species = spc.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    d.n_species = 1
    d.species = sp
    d.n_k = len(k)
    d.k_frac = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_bands = inst.n_bands
    return d, (frac, spc, sp, k)


@pytest.mark.parametrize("case", ["rc_too_large", "bad_order", "no_bands", "grid_too_big", "bad_species",
                                  "no_tiling", "axis_too_small", "norm_stride", "record_stride"])
def test_argument_errors_before_device_work(case):
    lib = _lib.load()
    sp = W.Species(D=-1.0, w=1.0, Rc=3.5)
    grid = (8, 8, 8)
    cell = "diamond8"
    if case == "rc_too_large":
        sp = W.Species(D=-1.0, w=1.0, Rc=4.0)
        cell = "fcc2"
    if case == "grid_too_big":
        grid = (64, 64, 64)
    if case == "no_tiling":  # 704 columns of 11 points: no built z-segment gives <= 1024 threads
        grid = (32, 22, 11)
    if case == "axis_too_small":
        grid = (8, 8, 3)
    inst = W.make_instance(cell, grid, 0 if case == "no_bands" else 2, [sp], W.KSpec((1, 1, 1)))
    k = np.zeros((1, 3))
    d, keep = _desc(inst, k)
    if case == "bad_species":
        bad = np.full(len(keep[0]), 3, np.int32)
        d.atom_species = bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    opt = _lib.Options()
    lib.tdks_default_options(ctypes.byref(opt))
    if case == "bad_order":
        opt.taylor_order = 2
    if case == "norm_stride":
        opt.norm_stride = -1
    if case == "record_stride":
        opt.record_stride = -3
    ctx = ctypes.c_void_p()
    rc = lib.tdks_create(ctypes.byref(d), 1, ctypes.byref(opt), ctypes.byref(ctx))
    want = {"rc_too_large": _lib.E_ARG, "bad_order": _lib.E_UNSUPPORTED, "no_bands": _lib.E_ARG,
            "grid_too_big": _lib.E_UNSUPPORTED, "bad_species": _lib.E_ARG, "no_tiling": _lib.E_UNSUPPORTED,
            "axis_too_small": _lib.E_UNSUPPORTED, "norm_stride": _lib.E_ARG, "record_stride": _lib.E_ARG}[case]
    assert rc == want, lib.tdks_last_error()
    assert ctx.value is None
    assert len(lib.tdks_last_error()) > 0


def test_tiling_rule_errors_before_device_work():
    """Rules that give one shape class two block sizes, and a rule count without rules, are
    argument errors found on the host."""
    lib = _lib.load()
    sp = W.Species(D=-1.0, w=1.0, Rc=3.5)
    insts = [W.make_instance("diamond8", (8, 8, 8), nb, [sp], W.KSpec((1, 1, 1))) for nb in (2, 3)]
    descs = (_lib.InstanceDesc * 2)()
    keep = []
    for i, inst in enumerate(insts):
        d, k = _desc(inst, np.zeros((1, 3)))
        descs[i] = d
        keep.append(k)
    opt = _lib.Options()
    lib.tdks_default_options(ctypes.byref(opt))
    rules = (_lib.TilingRule * 2)()
    for j, (nb, blk) in enumerate([(2, 512), (3, 256)]):
        rules[j].grid[:] = [8, 8, 8]
        rules[j].nonorth = -1
        rules[j].n_bands = nb
        rules[j].block_size = blk
    opt.tiling_rules = rules
    opt.n_tiling_rules = 2
    ctx = ctypes.c_void_p()
    assert lib.tdks_create(descs, 2, ctypes.byref(opt), ctypes.byref(ctx)) == _lib.E_ARG
    assert b"another block size" in lib.tdks_last_error()
    opt.tiling_rules = None
    opt.n_tiling_rules = 1
    assert lib.tdks_create(descs, 2, ctypes.byref(opt), ctypes.byref(ctx)) == _lib.E_ARG
    assert ctx.value is None
