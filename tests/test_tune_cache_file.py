"""The tune cache file format on the host (no GPU): a file written by
csk_tune_save carries the library version in its header and is read back by
csk_tune_load; a file of another version, or a missing one, reads as no
entries (-1), and a bad path is refused before anything is written."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_2004_02480_amd import _abi
    return _abi.load()


def test_save_then_load_empty_store(lib, tmp_path):
    from paper_2004_02480_amd import _abi
    lib.csk_tune_clear()
    path = tmp_path / "tune.txt"
    assert lib.csk_tune_save(str(path).encode()) == _abi.CSK_OK
    text = path.read_text()
    assert text.startswith("# csk tune cache, library version %d" % lib.csk_version())
    k = ctypes.c_int32(7)
    assert lib.csk_tune_load(str(path).encode(), ctypes.byref(k)) == _abi.CSK_OK
    assert k.value == 0


def test_other_version_and_missing_files_read_nothing(lib, tmp_path):
    from paper_2004_02480_amd import _abi
    other = tmp_path / "old.txt"
    other.write_text("# csk tune cache, library version 1\ngfx950|solve|d=1|n=1|dtype=0|vw=1\t1\t16\t2.0\n")
    k = ctypes.c_int32(0)
    assert lib.csk_tune_load(str(other).encode(), ctypes.byref(k)) == _abi.CSK_OK
    assert k.value == -1
    assert lib.csk_tune_load(str(tmp_path / "missing.txt").encode(), ctypes.byref(k)) == _abi.CSK_OK
    assert k.value == -1
    assert lib.csk_tune_save(b"") == _abi.CSK_ERR_INVALID_ARG
    assert lib.csk_tune_save(str(tmp_path / "no" / "such" / "dir.txt").encode()) == _abi.CSK_ERR_INVALID_ARG
