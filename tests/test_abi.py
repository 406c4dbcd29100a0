"""The C-ABI library loads and exports every symbol the header declares;
host-only calls work without a GPU; the ctypes structures match C."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fslbm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fslbm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    import paper_1604_01632_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libfslbm.so is not built (run __graft_entry__.build())")
    return pkg


def test_exports_every_declared_symbol(binding):
    L = binding.lib()
    names = _declared()
    assert {"fslbm_create", "fslbm_step", "fslbm_read_fields", "fslbm_bubbles"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (fslbm_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(binding, tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fslbm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(fslbm_params),'
                   ' offsetof(fslbm_params, tau), offsetof(fslbm_params, max_bubbles),'
                   ' sizeof(fslbm_bubble_init), sizeof(fslbm_bubble), sizeof(fslbm_scalars),'
                   ' sizeof(fslbm_timing), sizeof(fslbm_batch_info), offsetof(fslbm_batch_info, probe_ms));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [C.sizeof(binding.Params), binding.Params.tau.offset, binding.Params.max_bubbles.offset,
            C.sizeof(binding.BubbleInit), C.sizeof(binding.Bubble), C.sizeof(binding.Scalars),
            C.sizeof(binding.Timing), C.sizeof(binding.BatchInfo), binding.BatchInfo.probe_ms.offset]
    assert got == want


def test_workspace_bytes_host_only(binding):
    import scenes
    sc = scenes.config("c1")
    p64 = sc.params(precision=0)
    p32 = sc.params(precision=1)
    b64 = binding.fslbm_workspace_bytes(p64)
    b32 = binding.fslbm_workspace_bytes(p32)
    N = sc.n
    assert b64 >= 2 * 19 * 8 * N and b32 >= 2 * 19 * 4 * N and b64 > b32
    bad = dict(p64, tau=0.5)
    assert binding.fslbm_workspace_bytes(bad) == 0
    assert binding.fslbm_workspace_bytes(dict(p64, periodic=(0, 1, 1), nx=4)) == 0
    assert binding.fslbm_workspace_bytes(dict(p64, precision=7)) == 0
    assert binding.fslbm_batch_workspace_bytes(0) == 0
    assert binding.fslbm_batch_workspace_bytes(256) > 256 * 2 * 64


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1604_01632_amd as pkg
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        pkg.lib()


def test_workspace_bytes_at_the_size_limit(binding):
    """Cell indices are 32-bit: a box of 2^31 - 1 cells or fewer is sized
    (per cell at least the two lattices), one of 2^31 or more is rejected;
    the three precisions order as their storage does."""
    import scenes
    base = scenes.config("c1").params()
    big = dict(base, nx=1290, ny=1290, nz=1290)  # 2 146 689 000 cells
    n = 1290 ** 3
    sizes = {}
    for prec, s in ((0, 8), (1, 4), (2, 2)):
        b = binding.fslbm_workspace_bytes(dict(big, precision=prec))
        assert b >= 2 * 19 * s * n
        sizes[prec] = b
    assert sizes[0] > sizes[1] > sizes[2]
    assert binding.fslbm_workspace_bytes(dict(base, nx=2048, ny=1024, nz=1024)) == 0  # 2^31
    assert binding.fslbm_workspace_bytes(dict(base, nx=2048, ny=2048, nz=2048)) == 0
