"""CPU-only checks of the C ABI library: it loads, exports every symbol the
header declares, and its host-side error paths behave as documented.  No
kernel is launched here."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbgrb.h")


def _header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    funcs = set(re.findall(r"^\s*(?:GrB_Info|const char \*)\s*(\w+)\s*\(", text, flags=re.M))
    data = set()
    for line in re.findall(r"^extern\s+(?:GrB_\w+)\s+([^;]+);", text, flags=re.M):
        for name in line.split(","):
            data.add(name.strip().lstrip("*"))
    return funcs, data


@pytest.fixture(scope="module")
def grb():
    from paper_2509_14211_amd import grb as g
    if not os.path.exists(g.library_path()):
        from paper_2509_14211_amd import build
        build.build()
    g.load()
    return g


def test_header_parses():
    funcs, data = _header_symbols()
    assert "GrB_mxv" in funcs and "GrM_pagerank" in funcs and "GrM_error" in funcs
    assert "GrB_FP32" in data and "GrB_PLUS_TIMES_SEMIRING_FP32" in data


def test_library_exports_every_declared_symbol(grb):
    import ctypes
    lib = grb.load()
    funcs, data = _header_symbols()
    missing = [f for f in sorted(funcs | data) if not hasattr(lib, f)]
    assert not missing, missing
    # data symbols hold non-null addresses of static objects
    for name in data:
        assert ctypes.c_void_p.in_dll(lib, name).value


def test_binding_covers_every_function(grb):
    funcs, data = _header_symbols()
    bound = set(grb._FUNCS) | {"GrM_error"}
    assert funcs <= bound, sorted(funcs - bound)
    assert data <= set(grb.DATA_SYMBOLS), sorted(data - set(grb.DATA_SYMBOLS))


def test_calls_before_init_fail_cleanly(grb):
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_new(grb.builtin("GrB_FP32"), 10)
    assert e.value.info == -101  # GrB_PANIC: not initialised
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_size(None)
    assert e.value.info == -2  # GrB_NULL_POINTER
    # freeing NULL is a no-op
    grb.GrB_Vector_free(None)
    grb.GrB_finalize()
    assert "not" in grb.GrM_error() or grb.GrM_error() == ""


def test_init_without_gpu_reports_panic(grb):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_init(grb.GrB_NONBLOCKING)
    assert e.value.info == -101
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_init(7)
    assert e.value.info in (-3, -101)


def test_product_path_does_not_touch_oracle():
    """The product package never imports, loads or links the oracle."""
    pkg = os.path.join(ROOT, "paper_2509_14211_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text, f
                assert "from oracle" not in text, f


def test_allocator_exception_becomes_null():
    """An allocator callable that raises (torch's out-of-memory error) makes
    the C callback return NULL, which the library turns into
    GrB_OUT_OF_MEMORY; without the guard ctypes returns an undefined
    non-null pointer that kernels would then write to."""
    import ctypes
    from paper_2509_14211_amd import grb

    def oom(n):
        raise MemoryError("out of memory")

    freed = []
    ca, cf = grb.allocator_thunks(oom, freed.append)
    assert ca(1 << 40, None) is None
    ok, _ = grb.allocator_thunks(lambda n: 4096, freed.append)
    assert ok(16, None) == 4096
    cf(4096, None)
    assert freed == [4096]
    _, bad_free = grb.allocator_thunks(oom, oom)
    bad_free(4096, None)  # an exception in release is swallowed as well
