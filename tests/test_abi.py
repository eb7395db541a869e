"""Host-side checks of the C ABI: the library exists, exports every function
include/bh.h declares, and the ctypes structures match the C layouts."""

import ctypes
import os
import subprocess

import pytest

import paper_1106_1900_amd as bh
from paper_1106_1900_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_boundary():
    names = bh.declared_functions()
    for want in ("bh_create", "bh_destroy", "bh_build_tree", "bh_compute_forces",
                 "bh_leapfrog_step", "bh_get_state", "bh_set_state", "bh_set_velocities",
                 "bh_energy", "bh_stats_get", "bh_export_tree", "bh_last_error",
                 "bh_default_params"):
        assert want in names


def test_library_exports_every_declared_symbol():
    path = bh.library_path()
    assert os.path.exists(path), "libbh.so is not built"
    out = subprocess.check_output(["nm", "-D", "--defined-only", path]).decode()
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [f for f in bh.declared_functions() if f not in exported]
    assert not missing, missing
    # and ctypes can bind each of them
    lib = bh.load_library()
    for f in bh.declared_functions():
        assert getattr(lib, f) is not None


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "bh.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(bh_params), sizeof(bh_stats),'
        ' sizeof(bh_tree_host), offsetof(bh_stats, ms_keys), offsetof(bh_stats, device_bytes));'
        'return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(binding.Params), ctypes.sizeof(binding.Stats),
            ctypes.sizeof(binding.TreeHost), binding.Stats.ms_keys.offset,
            binding.Stats.device_bytes.offset]
    assert got == want


def test_default_params_without_a_device():
    lib = bh.load_library()
    p = binding.Params()
    assert lib.bh_default_params(ctypes.byref(p)) == 0
    assert (p.nleaf, p.ncrit, p.max_n, p.hbm_budget_bytes) == (16, 64, 0, 0)
    assert lib.bh_default_params(None) == binding.BH_EINVAL
    assert lib.bh_last_error(None) == b"null context"


def test_binding_refuses_to_run_without_the_library(monkeypatch):
    monkeypatch.setenv("BH_LIBRARY", "/nonexistent/libbh.so")
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.load_library()
