"""The schedule cache's file format (lp_schedule_cache_save / _load /
_clear): host-only calls, no GPU. A file round-trips; a malformed line or an
unsupported schedule rejects the whole file and leaves the cache as it was;
LP_SCHEDULE_CACHE is loaded on first use."""
import os
import subprocess
import sys

import pytest

from paper_2009_10247_amd import lp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEAD = "# lp-sched-v1"
GOOD = ["lp-sched-v1 1 23 9 1 2 64 2 0 4 16 0",    # batched driver, LDS step
        "lp-sched-v1 0 22 8 0 3 0 1 0 8 8 0",      # persistent driver, global step
        "lp-sched-v1 1 12 5 0 2 64 1 0 8 4 0"]


def _lines(path):
    return [ln.strip() for ln in open(path) if ln.strip() and not ln.startswith("#")]


def test_round_trip_and_clear(tmp_path):
    src, out = tmp_path / "a.txt", tmp_path / "b.txt"
    src.write_text(HEAD + "\n" + "\n".join(GOOD) + "\n")
    lp.schedule_cache_clear()
    lp.schedule_cache_load(str(src))
    lp.schedule_cache_save(str(out))
    assert sorted(_lines(out)) == sorted(GOOD)
    assert open(out).readline().startswith(HEAD)
    lp.schedule_cache_clear()
    lp.schedule_cache_save(str(out))
    assert _lines(out) == []


@pytest.mark.parametrize("bad", [
    "lp-sched-v2 1 23 9 1 2 64 1 0 4 16 0",      # unknown format
    "lp-sched-v1 1 23 9 1 2 64 1 0 4 16",        # a field missing
    "lp-sched-v1 1 23 9 1 2 64 1 0 4 16 0 7",    # a field too many
    "lp-sched-v1 1 23 9 1 2 64 1 0 4 5 0",       # unroll 5
    "lp-sched-v1 1 23 9 1 9 64 1 0 4 16 0",      # unknown driver
    "lp-sched-v1 2 23 9 1 2 64 1 0 4 16 0",      # lds flag 2
    "lp-sched-v1 1 23 99 1 2 64 1 0 4 16 0",     # row length bucket past 64
    "lp-sched-v1 1 23 9 1 2 64 1 0 4 16 300",    # block 300
    "lp-sched-v1 1 23 9 1 2 64 3 0 4 16 0",      # unknown step variant
])
def test_malformed_file_leaves_the_cache(tmp_path, bad):
    good, broken, out = tmp_path / "g.txt", tmp_path / "x.txt", tmp_path / "o.txt"
    good.write_text(GOOD[0] + "\n")
    broken.write_text(GOOD[1] + "\n" + bad + "\n")
    lp.schedule_cache_clear()
    lp.schedule_cache_load(str(good))
    with pytest.raises(lp.LPError) as e:
        lp.schedule_cache_load(str(broken))
    assert e.value.code == lp.LP_E_INVAL
    lp.schedule_cache_save(str(out))
    assert _lines(out) == [GOOD[0]]


def test_missing_file_and_bad_paths(tmp_path):
    with pytest.raises(lp.LPError):
        lp.schedule_cache_load(str(tmp_path / "none.txt"))
    with pytest.raises(lp.LPError):
        lp.schedule_cache_save(str(tmp_path / "no_dir" / "c.txt"))
    with pytest.raises(lp.LPError):
        lp.schedule_cache_save("")


def test_environment_file_loaded_on_first_use(tmp_path):
    env_file, out = tmp_path / "env.txt", tmp_path / "out.txt"
    env_file.write_text(GOOD[1] + "\n")
    code = ("from paper_2009_10247_amd import lp; import sys; lp.schedule_cache_save(sys.argv[1])")
    env = dict(os.environ, LP_SCHEDULE_CACHE=str(env_file))
    subprocess.run([sys.executable, "-c", code, str(out)], check=True, cwd=ROOT, env=env)
    assert _lines(out) == [GOOD[1]]
