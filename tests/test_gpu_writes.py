"""One writer per bitmap word: every kind of build, run against the
write-counting build of the library (libwtree_check.so, built beside the
product library), stores every 16-bit granule of its bitmaps exactly once
(tests/writecheck.py).  The counting build is a different library file, so
it runs in a process of its own."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_bitmap_granule_has_one_writer():
    from paper_1610_05994_amd import wtree
    lib = wtree.CHECK_LIB_PATH
    assert os.path.exists(lib), "the write-counting build is missing: run __graft_entry__.build()"
    env = dict(os.environ, WT_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-u", "-m", "tests.writecheck"], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    print(r.stdout[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "write check: ok" in r.stdout
