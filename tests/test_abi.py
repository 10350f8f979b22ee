"""The C ABI library (no GPU needed): it loads, exports every function that
include/dg.h declares, and the host-only entry point validates its
arguments."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1911_01492_amd import dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(dg.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dg.LIB_PATH):
        pytest.fail("libdg.so is not built (python -m paper_1911_01492_amd.build)")
    out = subprocess.run(["nm", "-D", "--defined-only", dg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(dg_[A-Za-z0-9_]+)$", out, flags=re.M))
    missing = [f for f in _declared() if f not in exported]
    assert not missing, missing
    L = dg.lib()
    for f in _declared():
        assert hasattr(L, f)


def test_query_workspace_validates():
    L = dg.lib()
    n = ctypes.c_size_t(0)

    def q(**kw):
        d = dict(nx=4, ny=4, nz=4, degree=3, bc=0, reserved=0, penalty_hat=0.0, vertices=None,
                 theta=None, workspace=None, workspace_bytes=0)
        d.update(kw)
        desc = dg.MeshDesc(**d)
        return L.dg_query_workspace(ctypes.byref(desc), ctypes.byref(n))

    assert q() == dg.DG_OK and n.value > 0
    small = n.value
    assert q(degree=4) == dg.DG_OK and n.value > small
    assert q(nx=0) == dg.DG_ERR_ARG
    assert q(degree=0) == dg.DG_ERR_UNSUPPORTED
    assert q(degree=8) == dg.DG_ERR_UNSUPPORTED
    assert q(bc=7) == dg.DG_ERR_ARG
    assert q(reserved=1) == dg.DG_ERR_ARG
    assert q(nx=-3) == dg.DG_ERR_ARG
    # N_dof must stay below 2^31 (32-bit element offsets in the kernels)
    assert q(nx=161, ny=161, nz=161, degree=7) == dg.DG_OK      # 2.137e9 DOF
    assert q(nx=162, ny=162, nz=162, degree=7) == dg.DG_ERR_ARG  # 2.177e9 DOF
    assert b"2^31" in L.dg_last_error(None)
    assert L.dg_query_workspace(None, ctypes.byref(n)) == dg.DG_ERR_ARG
    assert b"NULL" in L.dg_last_error(None)
    # the workspace of the 64^3 Q4 workload holds the FP64 and FP32 CG vectors
    desc = dg.MeshDesc(64, 64, 64, 4, 0, 0, 0.0, None, None, None, 0)
    assert L.dg_query_workspace(ctypes.byref(desc), ctypes.byref(n)) == dg.DG_OK
    ndof = 64 ** 3 * 125
    assert n.value >= ndof * (8 * 4 + 4 * 5 + 2)


def test_setup_rejects_missing_workspace():
    L = dg.lib()
    h = ctypes.c_void_p()
    desc = dg.MeshDesc(2, 2, 2, 1, 0, 0, 0.0, None, None, None, 0)
    assert L.dg_setup(ctypes.byref(desc), ctypes.byref(h), None) == dg.DG_ERR_ARG
    assert not h.value
    assert L.dg_setup(None, ctypes.byref(h), None) == dg.DG_ERR_ARG


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structures of the binding have the field offsets and sizes of
    the C structures in include/dg.h (compiled here with gcc)."""
    structs = {"dg_mesh_desc": dg.MeshDesc, "dg_cg_opts": dg.CgOpts, "dg_cg_info": dg.CgInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dg.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
