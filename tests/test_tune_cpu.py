"""Host side of the autotuner's table: lookup by size class, save/load round
trips, rejection of malformed files, and loading from SIGNTRI_TUNE_FILE.
None of this touches a GPU."""
import os
import subprocess
import sys

import pytest

from paper_1607_06303_amd import signtri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def lib():
    signtri.tune_clear()
    yield signtri
    signtri.tune_clear()


def write(path, lines):
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def test_empty_table_has_no_entries(lib):
    assert lib.tune_lookup(False, "fp64", "ph", 8192) is None


def test_load_lookup_by_size_class(lib, tmp_path):
    p = tmp_path / "t.txt"
    # dtype mode path log2n sweep tile wgs ms
    write(p, ["# comment", "0 0 1 13 2 32 0 23.4", "0 1 2 10 1 32 3 1.5"])
    lib.tune_load(str(p))
    e = lib.tune_lookup(False, "fp64", "ph", 8192)
    assert e["sweep_name"] == "superdiag" and e["tile"] == 32 and e["ms"] == pytest.approx(23.4)
    # ceil(log2 n) == 13 for 4097..8192
    assert lib.tune_lookup(False, "fp64", "ph", 4097)["log2n"] == 13
    assert lib.tune_lookup(False, "fp64", "ph", 4096) is None
    assert lib.tune_lookup(False, "fp64", "ph", 8193) is None
    assert lib.tune_lookup(False, "mixed", "ps", 1000)["wgs_per_cu"] == 3
    assert lib.tune_lookup(False, "mixed", "ph", 1000) is None
    assert lib.tune_lookup(True, "fp64", "ph", 8192) is None


def test_save_load_round_trip_and_replace(lib, tmp_path):
    p, q = tmp_path / "a.txt", tmp_path / "b.txt"
    write(p, ["0 0 1 12 1 32 2 10.0", "1 0 1 12 2 32 0 40.0"])
    lib.tune_load(str(p))
    write(q, ["0 0 1 12 2 64 0 9.0"])  # same key: replaces
    lib.tune_load(str(q))
    lib.tune_save(str(tmp_path / "c.txt"))
    lib.tune_clear()
    assert lib.tune_lookup(False, "fp64", "ph", 4000) is None
    lib.tune_load(str(tmp_path / "c.txt"))
    e = lib.tune_lookup(False, "fp64", "ph", 4000)
    assert (e["sweep"], e["tile"]) == (2, 64)
    assert lib.tune_lookup(True, "fp64", "ph", 4000)["ms"] == pytest.approx(40.0)


def test_batched_key(lib, tmp_path):
    """Batched entries (path 8): the dataflow sweep on 32 x 32 blocks only, keyed by
    the size class of the batch's largest order."""
    p = tmp_path / "b.txt"
    write(p, ["0 1 8 9 1 32 2 5.0"])
    lib.tune_load(str(p))
    e = lib.tune_lookup(False, "mixed", "batched", 400)
    assert e["wgs_per_cu"] == 2 and e["path"] == 8
    assert lib.tune_lookup(False, "mixed", "ph", 400) is None
    for bad in ("0 1 8 9 2 32 2 5.0", "0 1 8 9 1 64 2 5.0"):  # superdiag, 64 blocks
        write(p, [bad])
        with pytest.raises(OSError):
            lib.tune_load(str(p))


def test_autotune_batched_argument_checks(lib):
    import ctypes

    L = lib.lib()
    e = lib.TuneEntry()
    # reps and the result pointer are checked before any call
    assert L.signtri_autotune_batched(None, None, None, None, None, 1, 0, 0, None, 0,
                                      ctypes.byref(e)) == -12
    assert L.signtri_autotune_batched(None, None, None, None, None, 1, 0, 0, None, 1, None) == -13
    # then the batched call's own checks (-1: T is NULL)
    assert L.signtri_autotune_batched(None, None, None, None, None, 1, 0, 0, None, 1,
                                      ctypes.byref(e)) == -1


@pytest.mark.parametrize("bad", [
    "0 0 1 12 1 32 2",            # too few fields
    "0 0 1 12 1 32 2 1.0 extra",  # too many
    "5 0 1 12 1 32 2 1.0",        # dtype out of range
    "0 0 0 12 1 32 2 1.0",        # trivial path is never tuned
    "0 0 1 12 3 32 2 1.0",        # sweep out of range
    "0 0 1 12 1 48 2 1.0",        # block size
    "0 0 1 12 1 32 2 nan",        # time
])
def test_malformed_file_merges_nothing(lib, tmp_path, bad):
    p = tmp_path / "bad.txt"
    write(p, ["0 0 1 11 1 32 1 1.0", bad])
    with pytest.raises(OSError):
        lib.tune_load(str(p))
    assert lib.tune_lookup(False, "fp64", "ph", 2000) is None


def test_missing_file(lib, tmp_path):
    with pytest.raises(OSError):
        lib.tune_load(str(tmp_path / "nope.txt"))


def test_env_file_is_read_at_first_lookup(tmp_path):
    p = tmp_path / "env.txt"
    write(p, ["0 2 1 9 1 32 1 0.5"])
    code = ("from paper_1607_06303_amd import signtri; "
            "e = signtri.tune_lookup(False, 'fp32', 'ph', 300); "
            "print(e['wgs_per_cu'] if e else 'none')")
    env = dict(os.environ, SIGNTRI_TUNE_FILE=str(p))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"
