"""Host-side checks that need no GPU: the C-ABI library loads and exports every entry
point that include/echotrace.h declares; the header and the binding agree."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2602_19652_amd", "libechotrace.so")
HEADER = os.path.join(ROOT, "include", "echotrace.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(et_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2602_19652_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for must in ["et_create", "et_scene_build", "et_trace", "et_synthesize", "et_simulate",
                 "et_synthesize_backward", "et_simulate_batch", "et_simulate_batch_graph", "et_get_stats"]:
        assert must in names


def test_library_exports_every_declared_symbol(built):
    missing = [n for n in _declared() if not hasattr(built, n)]
    assert not missing, missing


def test_abi_version_and_status_strings(built):
    built.et_abi_version.restype = ctypes.c_int
    assert built.et_abi_version() == 4
    built.et_status_string.restype = ctypes.c_char_p
    built.et_status_string.argtypes = [ctypes.c_int]
    assert built.et_status_string(0) == b"ok"
    assert built.et_status_string(-2) == b"workspace too small"


def test_null_arguments_rejected_without_device(built):
    """Entry points reject NULL handles on the host before touching the device."""
    built.et_destroy.argtypes = [ctypes.c_void_p]
    assert built.et_destroy(None) == -1
    built.et_scene_free.argtypes = [ctypes.c_void_p]
    assert built.et_scene_free(None) == -1
    built.et_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    assert built.et_create(0, None, None) == -1


def test_binding_structs_match_header_field_order():
    """Every field of the ABI structs appears in the header in the binding's order."""
    import paper_2602_19652_amd as et
    txt = open(HEADER).read()
    for cls, cname in [(et.MeshDesc, "et_mesh_desc"), (et.SimDesc, "et_sim_desc"), (et.PathsDesc, "et_paths"),
                       (et.Stats, "et_stats"), (et.SceneInfo, "et_scene_info"), (et.Tuning, "et_tuning")]:
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", txt).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*(?:\[\d+\])?\s*[,;]", body)
        names = [n for n in names if n not in ("int32_t", "int64_t", "double", "float", "uint64_t", "uint32_t", "uint8_t")]
        assert [f[0] for f in cls._fields_] == names, cname


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits (status 2) with a message, before
    importing torch or touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
