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


STRUCTS = [("bh_params", "Params"), ("bh_stats", "Stats"), ("bh_tree_host", "TreeHost"),
           ("bh_cluster", "Cluster"), ("bh_server_params", "ServerParams"),
           ("bh_request", "Request"), ("bh_request_status", "RequestStatus"),
           ("bh_server_stats", "ServerStats"), ("bh_tune_entry", "TuneEntry"),
           ("bh_block_params", "BlockParams"), ("bh_block_stats", "BlockStats")]


def test_struct_layouts_match_the_header(tmp_path):
    # size and every field offset of each ctypes structure against the C compiler
    lines, want = [], []
    for cname, pyname in STRUCTS:
        cls = getattr(binding, pyname)
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        want.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, f))
            want.append(getattr(cls, f).offset)
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "bh.h"\n'
                   "int main(void){" + "".join(lines) + "return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == want


def test_default_params_without_a_device():
    lib = bh.load_library()
    p = binding.Params()
    assert lib.bh_default_params(ctypes.byref(p)) == 0
    assert (p.nleaf, p.ncrit, p.max_n, p.hbm_budget_bytes, p.max_clusters) == (16, 64, 0, 0, 0)
    assert lib.bh_default_params(None) == binding.BH_EINVAL
    assert lib.bh_last_error(None) == b"null context"
    binding._server_sigs(lib)
    assert lib.bh_server_last_error(None) == b"null server"
    assert lib.bh_server_create(None, None, None) == binding.BH_EINVAL


def test_binding_refuses_to_run_without_the_library(monkeypatch):
    monkeypatch.setenv("BH_LIBRARY", "/nonexistent/libbh.so")
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.load_library()


def test_create_validates_before_touching_the_device():
    import torch
    lib = bh.load_library()
    for field, value in (("nleaf", 0), ("nleaf", 65), ("ncrit", 0), ("ncrit", 129), ("max_n", -1),
                         ("hbm_budget_bytes", -1), ("max_clusters", -1)):
        p = binding.Params()
        lib.bh_default_params(ctypes.byref(p))
        setattr(p, field, value)
        h = ctypes.c_void_p()
        assert lib.bh_create(ctypes.byref(h), ctypes.byref(p), None) == binding.BH_EINVAL, field
        assert h.value is None
    assert lib.bh_create(None, None, None) == binding.BH_EINVAL
    if not torch.cuda.is_available():
        # no device: a valid request fails with BH_EDEVICE and leaves no context
        h = ctypes.c_void_p()
        assert lib.bh_create(ctypes.byref(h), None, None) == binding.BH_EDEVICE
        assert h.value is None
