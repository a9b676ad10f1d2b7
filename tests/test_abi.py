"""The C-ABI library loads and exports every entry point include/adept.h declares
(no compute call: this runs without a GPU); argument checks that need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adept.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adept_[a-z_]+)\s*\(", text)))


def test_header_declares_the_core_entry_points():
    names = declared()
    for core in ("adept_create", "adept_inject", "adept_step", "adept_run", "adept_tally", "adept_access_counts"):
        assert core in names


def test_library_exports_every_declared_symbol():
    import paper_2302_08252_amd as ad

    if not os.path.exists(ad.LIB_PATH):
        pytest.skip("libadept.so not built")
    L = ctypes.CDLL(ad.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(ad.EXPORTS) == declared()


def test_header_compiles_as_c_and_cpp(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "adept.h"\nint main(void){ adept_layout l = {0,0,1}; (void)l; return 0; }\n')
    import subprocess

    for cc, std in (("gcc", "-std=c99"), ("g++", "-std=c++11")):
        subprocess.check_call([cc, std, "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-x",
                               "c" if cc == "gcc" else "c++", str(src), "-o", str(tmp_path / "t")])


def test_create_rejects_bad_arguments():
    import paper_2302_08252_amd as ad

    if not os.path.exists(ad.LIB_PATH):
        pytest.skip("libadept.so not built")
    L = ad.lib()
    h = ctypes.c_void_p()
    assert L.adept_create(ad.Layout(0, 2, 3), 0, 1024, ctypes.byref(h)) == ad.E_INVALID  # lanes not a power of 2
    assert L.adept_create(ad.Layout(0, 2, 64), 0, 1000, ctypes.byref(h)) == ad.E_INVALID  # capacity % lanes
    assert L.adept_create(ad.Layout(2, 0, 1), 0, 1024, ctypes.byref(h)) == ad.E_INVALID
    assert L.adept_create(ad.Layout(0, 0, 1), 7, 1024, ctypes.byref(h)) == ad.E_INVALID
    assert L.adept_create(ad.Layout(0, 0, 1), 0, 0, ctypes.byref(h)) == ad.E_INVALID
    assert L.adept_create(ad.Layout(0, 0, 1), 0, (1 << 30) + 1, ctypes.byref(h)) == ad.E_INVALID
    L.adept_destroy(None)
