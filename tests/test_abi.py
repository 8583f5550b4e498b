"""CPU-only checks of the C ABI: the library loads, exports every function
declared in include/mg.h, and rejects invalid arguments on the host before
touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2604_06035_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b((?:mg|mgnn)_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = abi.lib()
    decl = declared_functions()
    assert "mg_build_level" in decl and "mg_solve" in decl and "mg_residual_norm" in decl
    for name in decl:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    assert set(abi.EXPORTED) <= set(decl)
    assert set(abi.NN_EXPORTED) <= set(decl)
    abi._nn_lib()   # every mgnn_* signature binds


def test_host_argument_validation_without_gpu():
    lib = abi.lib()
    h = ctypes.c_void_p()
    bad = [
        dict(base_n=12),                       # not a power of two
        dict(base_n=8, n_oct=10),              # wrong octs for a full level
        dict(base_n=8, nu_pre=0, nu_post=0),   # no smoothing
        dict(base_n=8, precision=7),
        dict(base_n=8, load_factor=0.95),
        dict(base_n=8, level=1, n_oct=8),      # refined level without oct list / parent
        dict(base_n=8, coarsest_n=3),          # coarsest grid not 2, 4 or 8
        dict(base_n=16, coarsest_n=16),
        dict(base_n=8, coarsest_n=-4),
        dict(base_n=8, brick_shift=9),         # brick lattice shift outside [0, 8]
        dict(base_n=8, brick_shift=-1),
    ]
    for kw in bad:
        d = abi.MgLevelDesc(base_n=kw.get("base_n", 8), level=kw.get("level", 0),
                            n_oct=kw.get("n_oct", (kw.get("base_n", 8) // 2) ** 3), d_oct_ijk=None, parent=None,
                            nu_pre=kw.get("nu_pre", 2), nu_post=kw.get("nu_post", 2),
                            coarsest_n=kw.get("coarsest_n", 0), brick_shift=kw.get("brick_shift", 0),
                            precision=kw.get("precision", 0),
                            load_factor=kw.get("load_factor", 0.5), stream=None)
        assert lib.mg_build_level(ctypes.byref(d), ctypes.byref(h)) == abi.MG_ERR_ARG, kw
        assert h.value is None
        assert abi.last_error()
    assert lib.mg_build_level(None, ctypes.byref(h)) == abi.MG_ERR_ARG
    info = abi.MgSolveInfo()
    assert lib.mg_solve(None, None, 0.0, 1.0, None, None, 1e-10, 10, ctypes.byref(info)) == abi.MG_ERR_ARG
    assert lib.mg_fft_solve(None, None, 0.0, 1.0, None, ctypes.byref(info)) == abi.MG_ERR_ARG
    assert "handle is NULL" in abi.last_error()
    assert lib.mg_solve_chain(None, 0, None, 0.0, 1.0, None, 1e-10, 10, 0, None) == abi.MG_ERR_ARG
    assert lib.mg_force(None, None, 0x1000, 0x2000) == abi.MG_ERR_ARG
    assert "handle is NULL" in abi.last_error()
    assert lib.mg_op_force(12, 0.1, 0x1000, 0x2000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_force(16, 0.1, None, 0x2000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_force(16, 0.1, 0x1008, 0x2000, None) == abi.MG_ERR_ARG
    hh = ctypes.c_void_p()
    assert lib.mg_hash_create(3, 0, 0.7, None, ctypes.byref(hh)) == abi.MG_ERR_ARG
    assert lib.mg_hash_create(1, 0, 0.95, None, ctypes.byref(hh)) == abi.MG_ERR_ARG
    assert hh.value is None
    assert lib.mg_hash_insert(None, 4, 0x1000, 0x2000) == abi.MG_ERR_ARG
    assert lib.mg_hash_lookup(None, 4, 0x1000, 0x2000) == abi.MG_ERR_ARG
    assert lib.mg_hash_info(None, None, None, None) == abi.MG_ERR_ARG
    assert lib.mg_op_morton128(4, 0x1004, 0x2000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_smooth(12, 0.1, 0, None, None, 1, None, None) == abi.MG_ERR_ARG
    assert lib.mg_op_smooth(16, 0.1, 3, 1, 1, 1, None, None) == abi.MG_ERR_ARG
    assert lib.mg_op_coarse_solve(16, 0.1, 0, 1, 1, None) == abi.MG_ERR_ARG
    assert "n must be" in abi.last_error()
    # layout helpers: size, NULL, alignment and overlap are refused on the host
    assert lib.mg_dense_to_oct(12, 0x1000, 0x100000, None) == abi.MG_ERR_ARG
    assert lib.mg_dense_to_oct(1, 0x1000, 0x100000, None) == abi.MG_ERR_ARG
    assert lib.mg_oct_to_dense(8, None, 0x100000, None) == abi.MG_ERR_ARG
    assert lib.mg_oct_to_dense(8, 0x1008, 0x100000, None) == abi.MG_ERR_ARG
    assert lib.mg_dense_to_oct(8, 0x1000, 0x1000 + 8 * 8 * 8 * 8 - 16, None) == abi.MG_ERR_ARG
    assert "overlap" in abi.last_error()
    # the hash hook: key width and arguments
    assert lib.mg_op_hash(4, 3, 0x1000, 0x2000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_hash(4, 1, None, 0x2000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_hash(4, 1, 0x1004, 0x2000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_hash(0, 1, None, None, None) == abi.MG_OK      # nothing to do
    # the allocation-free residual: grids beyond its static scratch, NULL and misaligned arrays
    assert lib.mg_op_resid_restrict_noalloc(2048, 0.1, 0, 0x1000, 0x2000, 0x3000, 0x4000, None) == abi.MG_ERR_ARG
    assert "scratch" in abi.last_error()
    assert lib.mg_op_resid_restrict_noalloc(64, 0.1, 0, None, 0x2000, 0x3000, 0x4000, None) == abi.MG_ERR_ARG
    assert lib.mg_op_resid_restrict_noalloc(64, 0.1, 0, 0x1008, 0x2000, 0x3000, 0x4000, None) == abi.MG_ERR_ARG


def test_network_argument_validation_without_gpu():
    lib = abi._nn_lib()
    h = ctypes.c_void_p()
    assert lib.mgnn_create(16, 5, 0, ctypes.byref(h)) == abi.MG_ERR_ARG
    assert lib.mgnn_create(24, 4, 0, ctypes.byref(h)) == abi.MG_ERR_ARG
    assert lib.mgnn_num_params(None) == 0
    assert lib.mgnn_forward_raw(None, 16, None, None, None) == abi.MG_ERR_ARG
    assert lib.mgnn_backward(None, 16, 0x1000, None) == abi.MG_ERR_ARG


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors against the C compiler's own offsets and sizes of
    # mg_level_desc_t and mg_solve_info_t (include/mg.h compiled by gcc)
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mg_level_desc_t": abi.MgLevelDesc, "mg_solve_info_t": abi.MgSolveInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (ln.split() for ln in out if ln)}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
    # and every field of the header's structs is mirrored (count of fields)
    assert len(abi.MgLevelDesc._fields_) == 12 and len(abi.MgSolveInfo._fields_) == 6


def test_binding_raises_typed_errors():
    with pytest.raises(abi.MgError) as ei:
        abi._check(abi.MG_ERR_TABLE)
    assert ei.value.status == abi.MG_ERR_TABLE


def test_misaligned_pointers_are_rejected_on_host():
    lib = abi.lib()
    assert lib.mg_op_smooth(16, 0.1, 0, 0x1008, 0x2000, 1, None, None) == abi.MG_ERR_ARG
    assert "aligned" in abi.last_error()
    assert lib.mg_op_prolong(16, 0, 0x1000, 0x2004, None) == abi.MG_ERR_ARG


def test_binding_checks_shapes_before_calling():
    # the binding derives the key count from the key tensor and refuses
    # companion arrays of another length (no library call is made)
    import torch
    keys = torch.zeros(6, dtype=torch.int64)
    with pytest.raises(ValueError):
        abi.mg_hash_insert(None, keys, torch.zeros(5, dtype=torch.int32))
    with pytest.raises(ValueError):
        abi.mg_hash_lookup(None, torch.zeros((6, 3), dtype=torch.int64), torch.zeros(6, dtype=torch.int32))
    with pytest.raises(ValueError):
        abi.mg_hash_neighbours(None, keys, 8, torch.zeros((6, 5), dtype=torch.int32))
    with pytest.raises(ValueError):
        abi.mg_hash_erase(None, torch.zeros(6, dtype=torch.int32))
    with pytest.raises(ValueError):
        abi.mg_force(None, None, torch.zeros(64, dtype=torch.float64), torch.zeros(64, dtype=torch.float64))
    with pytest.raises(ValueError):
        abi.mg_op_force(4, 0.25, torch.zeros(64, dtype=torch.float64), torch.zeros(64, dtype=torch.float64))
    with pytest.raises(ValueError):
        abi.mg_op_morton128(torch.zeros((4, 3), dtype=torch.int64), torch.zeros((4, 3), dtype=torch.int64))
