"""The library's host set-up (topology, element colours, partition, overlapping subdomains,
orderings, ILU(l) patterns, level schedules, factorization work lists, sweep slots) gives the
same products for any number of host threads: every array it produces hashes the same with
1, 3 and 8 threads.  CPU only: the set-up is built from its source with g++."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1810_04289_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_04289_amd", "csrc")
HIP_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(HIP_INC):
        pytest.skip("g++ or the HIP headers are missing")
    d = tmp_path_factory.mktemp("setup")
    exe = str(d / "setup_hash")
    cmd = ["g++", "-O2", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I", CSRC,
           "-I", os.path.join(ROOT, "include"), "-I", HIP_INC,
           os.path.join(ROOT, "tests", "native", "setup_hash.cpp"), os.path.join(CSRC, "setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    mesh = str(d / "tree1.bin")
    with open(mesh, "wb") as f:
        np.array([m.nverts, m.ntets, len(m.bfaces)], np.int32).tofile(f)
        np.ascontiguousarray(m.X, np.float64).tofile(f)
        np.ascontiguousarray(m.tets, np.int32).tofile(f)
        np.ascontiguousarray(m.tet_domain, np.int8).tofile(f)
        np.ascontiguousarray(m.bfaces, np.int32).tofile(f)
        np.ascontiguousarray(m.bface_tag, np.int8).tofile(f)
    part = str(d / "part9.bin")
    np.ascontiguousarray(W.uneven_partition(m, 9, sigma=0.5, seed=0), np.int32).tofile(part)
    return exe, mesh, part


@pytest.mark.parametrize("args", [("33", "1", "3", "0"), ("9", "2", "2", "1", "part")],
                         ids=["33 subdomains, overlap 1, ILU(3), RCM", "9 uneven, overlap 2, ILU(2), 1WD"])
def test_setup_products_do_not_depend_on_threads(harness, args):
    exe, mesh, part = harness
    argv = [exe, mesh] + [part if a == "part" else a for a in args]
    outs = {}
    for t in (1, 3, 8):
        r = subprocess.run(argv, capture_output=True, text=True, env=dict(os.environ, FSI_SETUP_THREADS=str(t)))
        assert r.returncode == 0, r.stdout + r.stderr
        outs[t] = r.stdout
    assert "all " in outs[1] and len(outs[1].splitlines()) > 30
    assert outs[3] == outs[1] and outs[8] == outs[1]
