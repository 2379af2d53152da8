"""The C ABI library loads on any host and exports every symbol that
include/fvm.h declares; the ctypes mirror of the descriptors has the C layout.
No compute calls (there may be no GPU here)."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(fvm_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def fvm_mod():
    from paper_2304_00140_amd import build, fvm
    if build.needs_build():
        build.build()
    return fvm


def test_library_exports_every_declared_symbol(fvm_mod):
    names = declared_functions()
    assert len(names) >= 30
    L = C.CDLL(fvm_mod.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_header(fvm_mod):
    assert set(declared_functions()) == set(fvm_mod.SIGNATURES)


def test_version(fvm_mod):
    assert fvm_mod.lib().fvm_version() == 4


def test_descriptor_layout_matches_c(fvm_mod, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fvm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(fvm_grid_desc), '
                   'sizeof(fvm_eos_desc), sizeof(fvm_scheme_desc), offsetof(fvm_grid_desc, in_seed), '
                   'offsetof(fvm_eos_desc, p_ref), offsetof(fvm_scheme_desc, eps_normal), '
                   'offsetof(fvm_eos_desc, kc), offsetof(fvm_scheme_desc, gravity), '
                   'offsetof(fvm_eos_desc, model), offsetof(fvm_eos_desc, bt_RT), offsetof(fvm_eos_desc, bt_mu_vap), '
                   'offsetof(fvm_eos_desc, bt_RT2));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    py = [C.sizeof(fvm_mod.fvm_grid_desc), C.sizeof(fvm_mod.fvm_eos_desc), C.sizeof(fvm_mod.fvm_scheme_desc),
          fvm_mod.fvm_grid_desc.in_seed.offset, fvm_mod.fvm_eos_desc.p_ref.offset,
          fvm_mod.fvm_scheme_desc.eps_normal.offset, fvm_mod.fvm_eos_desc.kc.offset,
          fvm_mod.fvm_scheme_desc.gravity.offset, fvm_mod.fvm_eos_desc.model.offset,
          fvm_mod.fvm_eos_desc.bt_RT.offset, fvm_mod.fvm_eos_desc.bt_mu_vap.offset,
          fvm_mod.fvm_eos_desc.bt_RT2.offset]
    assert out == py


def test_tile_tables_host_only(fvm_mod):
    L = fvm_mod.lib()
    for dim in (1, 2):
        n = L.fvm_tile_count(dim)
        assert n >= 2
        for t in range(n):
            tx, ty, nt = C.c_int(), C.c_int(), C.c_int()
            assert L.fvm_tile_shape(dim, t, C.byref(tx), C.byref(ty), C.byref(nt)) == 0
            # whole waves; a tile may have more or fewer cells than threads
            assert tx.value * ty.value > 0 and nt.value % 64 == 0
    assert L.fvm_tile_shape(2, 99, None, None, None) != 0
    # kernels per tile: one fused stage kernel in 1D/2D; in 3D the closure +
    # face pair, the z-marching kernel with the closure fused and after the
    # closure kernel, then the pair again
    for dim in (1, 2):
        assert {L.fvm_tile_kernels(dim, t) for t in range(L.fvm_tile_count(dim))} == {fvm_mod.FVM_TK_STAGE}
    kinds = [L.fvm_tile_kernels(3, t) for t in range(L.fvm_tile_count(3))]
    assert kinds == [fvm_mod.FVM_TK_PAIR] * 5 + [fvm_mod.FVM_TK_MARCH] * 5 + [fvm_mod.FVM_TK_PRIM_MARCH] * 5 + \
        [fvm_mod.FVM_TK_PAIR] * 5
    assert L.fvm_tile_kernels(3, len(kinds)) == fvm_mod.FVM_EINVAL and L.fvm_tile_kernels(4, 0) == fvm_mod.FVM_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2304_00140_amd import fvm
    monkeypatch.setattr(fvm, "_lib", None)
    monkeypatch.setattr(fvm, "LIB_PATH", "/nonexistent/libfvm.so")
    with pytest.raises(RuntimeError):
        fvm.lib()
