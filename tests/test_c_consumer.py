"""The C ABI from plain C: tests/c_consumer.c, built by build() against
include/dragexp.h, the in-tree library and the oracle.

CPU: argument errors and host-side calls (no device work).  GPU: one
drag_expm_apply per case, from C, against the oracle cell by cell (the
one-lane, two-lane and MFMA mappings), with the sticky status word read back.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c_consumer")


def _binary(tmp_path_factory=None):
    if os.path.exists(BIN):
        return BIN
    if tmp_path_factory is None:
        pytest.fail("tests/c_consumer is missing: run __graft_entry__.build() first")
    sys.path.insert(0, ROOT)
    import __graft_entry__
    out = str(tmp_path_factory.mktemp("c_consumer") / "c_consumer")
    return __graft_entry__.build_c_consumer(out)


def _run(binary, *args, timeout=120):
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = os.pathsep.join(
        [os.path.join(ROOT, "paper_2509_25347_amd"), os.path.join(ROOT, "oracle"),
         env.get("LD_LIBRARY_PATH", "")])
    return subprocess.run([binary, *map(str, args)], capture_output=True, text=True,
                          timeout=timeout, env=env)


def test_c_consumer_host_only(tmp_path_factory):
    r = _run(_binary(tmp_path_factory), "--host-only")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host-only ok" in r.stdout


@pytest.mark.gpu
@pytest.mark.parametrize("N,C,D,seed", [(4, 1000, 3, 11), (1, 65, 1, 12), (9, 517, 2, 13),
                                        (12, 300, 3, 14), (16, 301, 3, 15)])
def test_c_consumer_forward(N, C, D, seed):
    print(f"c_consumer N={N} C={C} D={D} seed={seed}", flush=True)
    r = _run(_binary(), N, C, D, seed)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "status 0 oracle 0" in r.stdout
