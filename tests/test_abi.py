"""The C-ABI library exports every function include/dt.h declares, and the
binding can bind all of them (no compute call: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1902_07554_amd", "libdt.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "dt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(dt_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(LIB):
        from paper_1902_07554_amd import build
        build.build()
    return LIB


def test_header_declares_the_path():
    names = _declared()
    for f in ("dt_triangulate", "dt_batch_triangulate", "dt_result_copy", "dt_server_submit"):
        assert f in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [f for f in _declared() if f not in exported]
    assert not missing, missing


def test_library_loads_and_binds(libpath):
    lib = ctypes.CDLL(libpath)
    for f in _declared():
        assert hasattr(lib, f), f
    from paper_1902_07554_amd import binding
    b = binding.load()
    assert b.dt_strerror(binding.DT_E_DUPLICATE)
    o = binding.options()
    assert o.divide == 0
    # nothing cached yet: returns at once, without a device call
    assert b.dt_release_cached_memory() == binding.DT_OK


def test_binding_structs_match_header(tmp_path):
    """ctypes mirrors of dt_options and dt_stats have the C layout."""
    from paper_1902_07554_amd import binding
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dt.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dt_options), '
                   'sizeof(dt_stats), offsetof(dt_options, recursive), '
                   'offsetof(dt_stats, candidates), offsetof(dt_options, gift_wrap), '
                   'offsetof(dt_stats, wrap_levels), offsetof(dt_options, refine_swaps));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(binding.Options), ctypes.sizeof(binding.Stats),
            binding.Options.recursive.offset, binding.Stats.candidates.offset,
            binding.Options.gift_wrap.offset, binding.Stats.wrap_levels.offset,
            binding.Options.refine_swaps.offset]
    assert got == want
