"""Host logic of the autotuner's table (no GPU): keys, the text format the
library reads, lookups, and the library's own parser (tsnmf_tune_load)."""

import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1402_6964_amd", "libtsnmf.so")


@pytest.fixture()
def tune(tmp_path, monkeypatch):
    from paper_1402_6964_amd import tune as t
    monkeypatch.setattr(t, "TUNED", str(tmp_path / "tuned.txt"))
    return t


def test_key_buckets_by_log2_rows(tune):
    assert tune.key("f32", "row", "f32", 1, 25, 10_000_000) == ("f32", "row", "f32", 1, 25, 23)
    assert tune.key("f32", "row", "f32", 1, 25, 2 ** 23) == tune.key("f32", "row", "f32", 1, 25, 2 ** 24 - 1)
    assert tune.key("f64", "col", "f64", 0, 64, 1)[-1] == 0


def test_save_and_load_round_trip(tune):
    t = {("f32", "row", "f32", 1, 25, 23): (4883, 16, 0, "0.40 ms"),
         ("f32", "row", "f64", 0, 25, 23): (1000, 0, 0, ""),
         ("f32", "col", "f32", 1, 64, 25): (0, 0, 16, "")}
    t[tune.BATCH] = ((0, 1, 2, 1), "70 ms")
    tune.save(t)
    assert tune.load() == t
    txt = open(tune.TUNED).read()
    assert "batch 0 1 2 1" in txt
    assert "tsqr f32 row f32 1 25 23 4883 16 0" in txt and "tsqr f32 row f64 0 25 23 1000 0 0" in txt
    assert "tsqr f32 col f32 1 64 25 0 0 16" in txt


def test_leaf_precision_and_contiguity_are_separate_keys(tune):
    """An entry measured on FP32 row blocks is not applied to the FP64-leaf
    kernels, nor to strided rows."""
    tune.save({("f32", "row", "f32", 1, 25, 23): (4883, 16, 0, "")})
    tab = tune.load()
    assert ("f32", "row", "f64", 1, 25, 23) not in tab
    assert ("f32", "row", "f32", 0, 25, 23) not in tab


def test_unreadable_table_is_empty(tune):
    with open(tune.TUNED, "w") as f:
        f.write("not a table\n")
    assert tune.load() == {}


def _lib():
    so = ctypes.CDLL(LIB)
    so.tsnmf_tune_load.restype = ctypes.c_int
    so.tsnmf_tune_load.argtypes = [ctypes.c_char_p]
    return so


def test_library_parser_accepts_the_table_and_rejects_bad_lines(tmp_path):
    so = _lib()
    good = tmp_path / "good.txt"
    good.write_text("# comment\n\ntsqr f32 row f32 1 25 23 4883 16  # 0.40 ms\ntsqr f64 col f64 0 64 20 0 0\n"
                    "tsqr f32 col f32 1 64 25 0 0 16\nbatch 0 1 2 1  # 68 ms\n")
    assert so.tsnmf_tune_load(str(good).encode()) == 0
    for bad in ("tsqr f32 row f32 1 25 23 4883\n",        # missing field
                "tsqr f16 row f32 1 25 23 4883 16\n",     # dtype
                "tsqr f64 row f32 1 25 23 0 0\n",         # FP64 input with FP32 leaves
                "tsqr f32 row f32 1 500 23 0 0\n",        # width
                "tsqr f32 row f32 1 25 23 0 1\n",         # arity 1
                "tsqr f32 col f32 1 64 25 0 0 8\n",       # WY panel width
                "batch s16 4096\n",                       # not four shifts
                "batch 0 1 2\n",                          # missing shift
                "batch 0 0 9 0\n"):                       # shift out of range
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        assert so.tsnmf_tune_load(str(p).encode()) == -1, bad
    assert so.tsnmf_tune_load(str(tmp_path / "missing.txt").encode()) == -1
    assert so.tsnmf_tune_load(None) == 0


def test_committed_table_parses(tune):
    """The table shipped with the package is read by the library."""
    path = os.path.join(ROOT, "paper_1402_6964_amd", "tuned.txt")
    if not os.path.exists(path):
        pytest.skip("no tuned table committed")
    assert _lib().tsnmf_tune_load(path.encode()) == 0
    assert _lib().tsnmf_tune_load(None) == 0
