"""Host-side checks of the C ABI: the library builds, loads and exports every
entry point the header declares.  No GPU work is launched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spamm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib_path():
    from paper_1508_05856_amd import spamm
    if not os.path.exists(spamm.LIB_PATH):
        from paper_1508_05856_amd import build
        build.build()
    return spamm.LIB_PATH


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("spamm_norms", "spamm_multiply", "ns_sqrt", "spamm_create", "spamm_destroy",
                 "spamm_last_error", "spamm_pyramid_len", "spamm_ns_history"):
        assert want in names


def test_library_exports_every_declared_symbol(lib_path):
    from paper_1508_05856_amd import spamm
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(spamm.EXPORTS) == set(declared_functions())


def test_pyramid_len_host_function(lib_path):
    from paper_1508_05856_amd import spamm
    lib = spamm.load_library(lib_path)
    assert lib.spamm_pyramid_len(512, 32) == (4 ** 5 - 1) // 3       # nb = 16, L = 4
    assert lib.spamm_pyramid_len(100, 16) == (4 ** 4 - 1) // 3       # nb = 7 -> padded to 8
    assert lib.spamm_pyramid_len(32, 32) == 1
    assert lib.spamm_pyramid_len(0, 32) == -1
    assert lib.spamm_pyramid_len(64, 48) == -1


def test_null_context_is_rejected_without_gpu(lib_path):
    from paper_1508_05856_amd import spamm
    lib = spamm.load_library(lib_path)
    st = lib.spamm_norms(None, None, 16, 16, 16, None, None, None)
    assert st == spamm.EINVAL
    assert b"NULL" in lib.spamm_last_error()


def test_library_exports_nothing_else_unmangled(lib_path):
    """Every defined symbol with C linkage is one the header declares (helpers
    stay internal)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm is not available")
    out = subprocess.run([nm, "-D", "--defined-only", lib_path], check=True, capture_output=True, text=True).stdout
    c_names = {line.split()[-1] for line in out.splitlines()
               if len(line.split()) == 3 and line.split()[1] == "T" and not line.split()[-1].startswith("_")}
    assert c_names == set(declared_functions()), sorted(c_names ^ set(declared_functions()))
