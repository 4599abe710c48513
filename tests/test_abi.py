"""The C-ABI library loads and exports every function include/crisp.h declares (CPU, no compute)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "crisp.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(crisp_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2603_05180_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTED)


def test_version_and_error_string_without_gpu():
    from paper_2603_05180_amd import _lib
    assert _lib.lib.crisp_version().startswith(b"crisp-gfx950")
    assert isinstance(_lib.lib.crisp_last_error(), bytes)


def test_null_arguments_are_rejected_before_any_launch():
    from paper_2603_05180_amd import _lib
    size = ctypes.c_size_t(0)
    assert _lib.lib.crisp_index_derived_bytes(None, 0, ctypes.byref(size)) == -1
    desc = _lib.IndexDesc(1000, 100, 4, 8, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 0, ctypes.byref(size)) == -5   # D % 64
    desc = _lib.IndexDesc(1000, 128, 4, 8, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 0, ctypes.byref(size)) == 0
    assert size.value > 0
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 5000, ctypes.byref(size)) == -1  # not 2^k
    desc = _lib.IndexDesc(1000, 128, 4, 300, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 0, ctypes.byref(size)) == -5
    assert _lib.lib.crisp_search(None, None, 1, 1, None, None, None, None, 0, None, None) == -1
    assert _lib.lib.crisp_rotate_rows(None, 1, 64, None, None, None) == -1
    assert _lib.lib.crisp_build_csr(None, 1, 1, None, None, None, None) == -1


def test_new_entry_points_reject_bad_arguments_without_launching():
    from paper_2603_05180_amd import _lib
    lib = _lib.lib
    # misaligned or null copy: rejected before any launch
    assert lib.crisp_copy_probe(ctypes.c_void_p(16), ctypes.c_void_p(8), 32, None) == -1
    assert lib.crisp_copy_probe(None, ctypes.c_void_p(16), 32, None) == -1
    assert lib.crisp_copy_probe(ctypes.c_void_p(16), ctypes.c_void_p(32), 20, None) == -1
    size = ctypes.c_size_t(0)
    p = _lib.SearchParams(1, 0.01, 2, 40, None, 0, 0, 0, 0, 0)
    assert lib.crisp_plan_bytes(None, 16, 10, ctypes.byref(p), ctypes.byref(size)) == -1
    assert lib.crisp_plan_search(None, None, 0, None, None, None) == -1
    assert lib.crisp_plan_free(None) == 0
    assert lib.crisp_index_bf16_bytes(None, ctypes.byref(size)) == -1
    assert lib.crisp_feature_count(32) == 1 + 16 + 3 * 32 + 13
    assert lib.crisp_mlp_param_count(10) == 10 * 64 + 2 * 64 + 1


def test_engine_without_the_library_fails_loudly(tmp_path):
    """A copy of the package with no built library: importing the engine
    raises ImportError naming the missing file (no CPU fallback exists)."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2603_05180_amd")
    shutil.copytree(src, tmp_path / "paper_2603_05180_amd",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
    r = subprocess.run([sys.executable, "-c", "import paper_2603_05180_amd.engine"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, PYTHONPATH=str(tmp_path)))
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libcrisp.so is missing" in r.stderr


def test_static_scratch_entry_point():
    """crisp_search_static validates before touching the GPU, and the
    binding's copy of the scratch size matches the header."""
    from paper_2603_05180_amd import _lib
    assert _lib.lib.crisp_search_static(None, None, 1, 1, None, None, None, None) == -1
    with open(os.path.join(ROOT, "include", "crisp.h")) as f:
        m = re.search(r"#define CRISP_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", f.read())
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.STATIC_SCRATCH_BYTES


def test_binding_validates_outputs_on_the_host():
    """The binding's checks of caller-provided outputs and queries (CPU
    tensors stand in for device ones; nothing reaches the library)."""
    import pytest
    import torch
    from paper_2603_05180_amd import engine
    dev = torch.device("cpu")
    ids, d = engine._outputs(None, 4, 3, dev)
    assert ids.shape == (4, 3) and ids.dtype == torch.int64 and d.dtype == torch.float32
    ok = (torch.empty(4, 3, dtype=torch.int64), torch.empty(4, 3, dtype=torch.float32))
    assert engine._outputs(ok, 4, 3, dev)[0] is ok[0]
    for bad in [(ok[0],), (torch.empty(4, 2, dtype=torch.int64), ok[1]), (ok[0], torch.empty(4, 3, dtype=torch.float64)),
                (ok[0], torch.empty(3, 4, dtype=torch.float32).t()), (ok[0].int(), ok[1])]:
        with pytest.raises(ValueError):
            engine._outputs(bad, 4, 3, dev)
    engine._check_queries(torch.zeros(5, 64), 64, dev)
    for bad in [torch.zeros(5, 32), torch.zeros(320), torch.zeros(5, 64, dtype=torch.float64),
                torch.zeros(64, 5).t(), "queries"]:
        with pytest.raises(ValueError):
            engine._check_queries(bad, 64, dev)


def test_codebooks_above_64_are_refused():
    """K > 64 is switched off in the library (its selection path faulted the
    GPU at K = 256, cause not found): the shape check refuses it, no launch."""
    from paper_2603_05180_amd import _lib
    size = ctypes.c_size_t(0)
    desc = _lib.IndexDesc(1000, 128, 4, 80, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 0, ctypes.byref(size)) == -5
    assert b"K > 64" in _lib.lib.crisp_last_error()
    desc = _lib.IndexDesc(1000, 128, 4, 64, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 0, ctypes.byref(size)) == 0


def test_tile_and_posting_size_limits():
    """Collision-counting tiles hold at most 65,536 ids (a posting entry's
    counter position is 16 bits) and the posting lists at most 2^31 entries
    in all (their byte offsets are 32-bit); the derived buffer holds 2 bytes
    per posting entry."""
    from paper_2603_05180_amd import _lib
    size = ctypes.c_size_t(0)
    desc = _lib.IndexDesc(100_000, 128, 4, 8, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 65536, ctypes.byref(size)) == 0
    small = size.value
    assert small >= 4 * 100_000 * 2
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 131072, ctypes.byref(size)) == -1
    assert b"65536" in _lib.lib.crisp_last_error()
    desc = _lib.IndexDesc(40_000_000, 128, 64, 8, None, None, None, None, None, None)
    assert _lib.lib.crisp_index_derived_bytes(ctypes.byref(desc), 65536, ctypes.byref(size)) == -5
    assert b"M x N" in _lib.lib.crisp_last_error()
