"""Host planners of the traversal kernels, checked on the CPU.

tests/plan_check.cpp replays the index arithmetic of the post- and
pre-order walks (level walks, top region, depth-first clade walks with their
deliberate dummy and past-the-end loads, LDS stacks) and the dirty-path
schedules of partial re-evaluation against the plans of
paper_1905_12146_amd/csrc/plan.cpp, built with AddressSanitizer and
UndefinedBehaviorSanitizer, for Yule trees, a caterpillar and a balanced
tree.  No GPU is involved.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import yule_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_12146_amd", "csrc")


def caterpillar(n):
    """Internal node n + k joins node n + k - 1 (tip 0 for k = 0) and tip k + 1."""
    parent = np.full(2 * n - 1, -1, dtype=np.int64)
    parent[0] = n
    for k in range(n - 1):
        parent[k + 1] = n + k
        if k > 0:
            parent[n + k - 1] = n + k
    return parent


def balanced(n):
    """Complete binary tree over n = 2^d tips, internal nodes level by level."""
    parent = np.full(2 * n - 1, -1, dtype=np.int64)
    level = list(range(n))
    nxt = n
    while len(level) > 1:
        up = []
        for i in range(0, len(level), 2):
            parent[level[i]] = parent[level[i + 1]] = nxt
            up.append(nxt)
            nxt += 1
        level = up
    return parent


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("plan") / "plan_check"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(CSRC, "plan.cpp"), os.path.join(ROOT, "tests", "plan_check.cpp"), "-o", str(out)]
    subprocess.run(cmd, check=True)
    return str(out)


TREES = [("yule", 2), ("yule", 3), ("yule", 30), ("yule", 1000), ("yule", 3000),
         ("caterpillar", 300), ("balanced", 256), ("yule", 500)]


@pytest.mark.parametrize("kind,n", TREES)
def test_plans(checker, tmp_path, kind, n):
    if kind == "yule":
        parent = yule_tree(n, np.random.default_rng(7 + n))
    elif kind == "caterpillar":
        parent = caterpillar(n)
    else:
        parent = balanced(n)
    assert parent[-1] == -1 and len(parent) == 2 * n - 1
    path = tmp_path / "tree.txt"
    path.write_text(f"{n}\n" + " ".join(str(int(p)) for p in parent) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([checker, str(path)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checks passed" in r.stdout
