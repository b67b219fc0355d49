"""The C ABI library builds, loads and exports what include/ess.h declares (no GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ess.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ess_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libess():
    import paper_2407_10449_amd as E
    if not os.path.exists(E.LIB_PATH):
        from paper_2407_10449_amd import build
        build.build()
    return E.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ess_init", "ess_step", "ess_run", "ess_get_state", "ess_set_state",
                     "ess_transition_explicit", "ess_destroy", "ess_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(libess):
    missing = [n for n in declared_functions() if not hasattr(libess, n)]
    assert not missing, missing


def test_exported_symbols_are_c_linkage():
    import paper_2407_10449_amd as E
    if not os.path.exists(E.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", E.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for n in declared_functions():
        assert n in exported, n


def test_problem_struct_layout_matches_header(libess):
    import ctypes
    import paper_2407_10449_amd as E
    # int32 x4, three pointers, uint64, double, uint32 (+ tail padding)
    assert ctypes.sizeof(E.EssProblem) == 64
    assert E.EssProblem.seed.offset == 40 and E.EssProblem.trim_eps.offset == 48


def test_last_error_without_gpu_work(libess):
    import paper_2407_10449_amd as E
    assert isinstance(E.ess_last_error(), str)


def test_binding_fails_loudly_when_library_missing(tmp_path, monkeypatch):
    import paper_2407_10449_amd as E
    monkeypatch.setattr(E, "_LIB", None)
    monkeypatch.setattr(E, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        E.lib()
