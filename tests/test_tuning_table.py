"""The process-wide autotune table: host-only import / export / clear through
the C ABI (no device call), its text format and its all-or-nothing import."""

import ctypes

import pytest

from paper_2501_11592_amd import clomp as C

HDR = "clomp-tuning 1\n"


@pytest.fixture(autouse=True)
def empty_table():
    C.tuning_table_clear()
    yield
    C.tuning_table_clear()


def test_round_trip_sorted_and_merged():
    text = HDR + "gfx950/f32/clomp/corr/m9/n11/c1 512\n# a comment\n\ngfx950/bf16/omp/resid/m6/n8/c9 64\n"
    assert C.tuning_table_import(text) == 2
    out = C.tuning_table_export()
    assert out == HDR + "gfx950/bf16/omp/resid/m6/n8/c9 64\ngfx950/f32/clomp/corr/m9/n11/c1 512\n"
    # a later import replaces an entry with the same key and keeps the others
    assert C.tuning_table_import(HDR + "gfx950/f32/clomp/corr/m9/n11/c1 1024\r\n") == 1
    out = C.tuning_table_export()
    assert "gfx950/f32/clomp/corr/m9/n11/c1 1024\n" in out and "m6/n8/c9 64\n" in out
    # export -> import in a fresh table reproduces it
    C.tuning_table_clear()
    assert C.tuning_table_export() == HDR
    assert C.tuning_table_import(out) == 2
    assert C.tuning_table_export() == out


@pytest.mark.parametrize("bad, why", [
    ("", "header"),
    ("clomp-tuning 2\nk 1\n", "header"),
    ("\n" + HDR, "header"),
    (HDR + "early/entry 7\nk\n", "expected"),
    (HDR + "early/entry 7\n 5\n", "expected"),
    (HDR + "early/entry 7\nk 0\n", "65536"),
    (HDR + "early/entry 7\nk 65537\n", "65536"),
    (HDR + "early/entry 7\nk -3\n", "65536"),
    (HDR + "early/entry 7\nk 12x\n", "65536"),
    (HDR + "early/entry 7\nk  5\n", "65536"),
    (HDR + "early/entry 7\nk\t5\n", "expected"),
    (HDR + "early/entry 7\na*b 5\n", "character"),
    (HDR + "early/entry 7\nk 5\nk 6\n", "repeated"),
    (HDR + "early/entry 7\n" + "x" * 128 + " 5\n", "expected"),
])
def test_malformed_import_changes_nothing(bad, why):
    """A bad line anywhere rejects the whole text: the valid entries before it
    are not imported either."""
    C.tuning_table_import(HDR + "kept/key 256\n")
    with pytest.raises(C.ClompError, match=why):
        C.tuning_table_import(bad)
    assert C.tuning_table_export() == HDR + "kept/key 256\n"


def test_limits_accepted():
    key = "k" * 127
    assert C.tuning_table_import(HDR + f"{key} 65536\nz 1\n") == 2
    assert C.tuning_table_export() == HDR + f"{key} 65536\nz 1\n"


def test_export_buffer_contract():
    lib = C.load_library()
    C.tuning_table_import(HDR + "a/b 128\n")
    n = ctypes.c_size_t(0)
    assert lib.clomp_tuning_table_export(None, 0, ctypes.byref(n)) == 0
    assert n.value == len(HDR) + len("a/b 128\n")
    small = ctypes.create_string_buffer(b"untouched", n.value)     # one byte short of the NUL
    assert lib.clomp_tuning_table_export(small, n.value, ctypes.byref(n)) == 1
    assert small.value == b"untouched"
    assert b"needs" in lib.clomp_last_error(None)
    assert lib.clomp_tuning_table_export(None, 0, None) == 1
    assert lib.clomp_tuning_table_import(None, None) == 1


def test_save_and_load_file(tmp_path):
    C.tuning_table_import(HDR + "gfx950/f32/clomp/corr/m7/n11/c1 384\n")
    f = tmp_path / "tuning.txt"
    C.save_tuning_table(f)
    C.tuning_table_clear()
    assert C.load_tuning_table(f) == 1
    assert f.read_text() == C.tuning_table_export()
