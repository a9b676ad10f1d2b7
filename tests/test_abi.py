"""The C-ABI library loads and exports every entry point include/adept.h declares
(no compute call: this runs without a GPU); argument checks that need no device."""
import ctypes
import os
import re

import numpy as np
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


def _comment_before(text, name):
    """The comment block right before the declaration of entry point `name`."""
    m = re.search(r"(/\*(?:(?!\*/).)*\*/)\s*adept_status\s+" + name + r"\s*\(", text, flags=re.S)
    return m.group(1) if m else ""


def test_core_declarations_cite_the_defining_passage():
    """Each of the six core calls says which section of the paper defines the
    operation it performs (and its error behaviour)."""
    text = open(HEADER).read()
    for core, sec in (("adept_create", "Sec. 2"), ("adept_inject", "Sec. 2"), ("adept_step", "Sec. 2"),
                      ("adept_run", "Sec. 2"), ("adept_tally", "Sec. 4"), ("adept_access_counts", "Sec. 5")):
        c = _comment_before(text, core)
        assert c, core
        assert sec in c, (core, c)
        assert "Errors" in c or "ADEPT_E_" in c, core


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


def _oracle_byte_map(oracle_mod, mapping, lanes, precision, capacity):
    """The oracle's byte map of a layout: every (slot, field) placed at its address."""
    total = oracle_mod.buffer_bytes(mapping, lanes, precision, capacity)
    m = np.full(total, -1, dtype=np.int8)
    for slot in range(capacity):
        for leaf in range(14):
            a = oracle_mod.leaf_addr(mapping, lanes, precision, capacity, slot, leaf)
            n = oracle_mod.leaf_size(precision, leaf)
            assert (m[a:a + n] == -1).all()  # no two fields share a byte
            m[a:a + n] = leaf
    return m


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("mapping,lanes,capacity", [(0, 1, 96), (1, 1, 96), (1, 1, 77), (2, 8, 96), (2, 64, 128),
                                                    (2, 2, 6)])
def test_layout_map_matches_oracle_byte_map(oracle_mod, mapping, lanes, capacity, precision):
    """The library's byte picture of a layout (inverse address arithmetic) equals the
    oracle's forward map, padding included, also through a window and past the end."""
    import paper_2302_08252_amd as ad

    if not os.path.exists(ad.LIB_PATH):
        pytest.skip("libadept.so not built")
    want = _oracle_byte_map(oracle_mod, mapping, lanes, precision, capacity)
    got = ad.adept_layout_map(mapping, precision, capacity, aosoa_lanes=lanes)
    assert np.array_equal(got, want)
    win = ad.adept_layout_map(mapping, precision, capacity, first_byte=37, n=len(want), aosoa_lanes=lanes)
    assert np.array_equal(win[:len(want) - 37], want[37:]) and (win[len(want) - 37:] == -1).all()
    pic = ad.layout_picture(got, 64, 4).split("\n")
    assert len(pic) == min(4, -(-len(want) // 64)) and all(len(r) <= 16 for r in pic)


def test_layout_map_rejects_bad_arguments():
    import paper_2302_08252_amd as ad

    if not os.path.exists(ad.LIB_PATH):
        pytest.skip("libadept.so not built")
    L = ad.lib()
    buf = np.zeros(8, dtype=np.int8)
    p = buf.ctypes.data_as(ctypes.c_void_p)
    assert L.adept_layout_map(ad.Layout(0, 2, 3), 0, 96, 0, 8, p, None) == ad.E_INVALID
    assert L.adept_layout_map(ad.Layout(0, 2, 64), 0, 100, 0, 8, p, None) == ad.E_INVALID
    assert L.adept_layout_map(ad.Layout(0, 3, 1), 0, 96, 0, 8, p, None) == ad.E_INVALID
    assert L.adept_layout_map(ad.Layout(0, 0, 1), 2, 96, 0, 8, p, None) == ad.E_INVALID
    assert L.adept_layout_map(ad.Layout(0, 0, 1), 0, 0, 0, 8, p, None) == ad.E_INVALID
    assert L.adept_layout_map(ad.Layout(0, 0, 1), 0, 96, 0, 8, None, None) == ad.E_INVALID
    assert L.adept_layout_map(ad.Layout(0, 0, 1), 0, 96, 0, 0, None, None) == ad.OK


def test_create_typed_rejects_bad_arguments():
    """Per-type layouts: each is checked as adept_create checks one, and all three
    must name the same scheme."""
    import paper_2302_08252_amd as ad

    if not os.path.exists(ad.LIB_PATH):
        pytest.skip("libadept.so not built")
    L = ad.lib()
    h = ctypes.c_void_p()

    def typed(*lays, cap=1024, prec=0):
        arr = (ad.Layout * 3)(*lays)
        return L.adept_create_typed(ctypes.cast(arr, ctypes.c_void_p), prec, cap, ctypes.byref(h))

    assert typed(ad.Layout(1, 0, 1), ad.Layout(0, 1, 1), ad.Layout(1, 2, 64)) == ad.E_INVALID  # schemes differ
    assert typed(ad.Layout(1, 0, 1), ad.Layout(1, 2, 3), ad.Layout(1, 1, 1)) == ad.E_INVALID  # lanes not a power of 2
    assert typed(ad.Layout(1, 0, 1), ad.Layout(1, 2, 64), ad.Layout(1, 1, 1), cap=1000) == ad.E_INVALID
    assert typed(ad.Layout(1, 0, 1), ad.Layout(1, 4, 1), ad.Layout(1, 1, 1)) == ad.E_INVALID
    assert typed(ad.Layout(1, 0, 1), ad.Layout(1, 1, 1), ad.Layout(1, 1, 1), prec=5) == ad.E_INVALID
    assert L.adept_create_typed(None, 0, 1024, ctypes.byref(h)) == ad.E_INVALID
    n = ctypes.c_size_t()
    assert L.adept_type_buffer_bytes(None, 0, ctypes.byref(n)) == ad.E_INVALID
