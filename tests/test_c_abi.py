"""The C ABI from a plain C program (host-only plan, no GPU): levels and
permutation equal the oracle's, a schedule is built, and errors come back
as status codes with a message."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_12525_amd", "libmpk.so")

pytestmark = pytest.mark.skipif(not (shutil.which("gcc") and os.path.exists(LIB)),
                                reason="needs gcc and the built library")


def test_host_only_plan_from_c(tmp_path):
    from paper_2405_12525_amd import _capi
    exe = tmp_path / "abi_host"
    subprocess.run(["gcc", "-std=c99", "-O1", "-Wall", "-Werror", f"-I{ROOT}/include",
                    os.path.join(ROOT, "tests", "c", "abi_host.c"), "-o", str(exe),
                    f"-L{os.path.dirname(LIB)}", "-lmpk",
                    f"-Wl,-rpath,{os.path.dirname(LIB)}"], check=True)
    L = 9
    out = subprocess.run([str(exe), str(L)], check=True, capture_output=True,
                         text=True).stdout.splitlines()
    rows = {line.split()[0]: line.split()[1:] for line in out}
    A = w.stencil_2d5(L)
    levels, perm, _ = oracle.bfs_levels(A.n, A.rowptr, A.col, root=0)
    assert rows["n"][0] == str(A.n) and rows["n"][2] == str(A.nnz)
    assert int(rows["n"][4]) == len(levels)
    assert [int(v) for v in rows["level_ptr"]] == [0] + np.cumsum([len(v) for v in levels]).tolist()
    assert [int(v) for v in rows["perm"]] == perm.tolist()
    assert rows["schedule"][0] == str(_capi.MPK_OK) and int(rows["schedule"][4]) == 3 * int(rows["schedule"][2])
    assert rows["bad_csr"] == [str(_capi.MPK_EBADCSR), "message"]
    assert rows["bad_tune"] == [str(_capi.MPK_EINVAL)]
    assert rows["run_host_only"] != [str(_capi.MPK_OK)]
    assert rows["version"][0].startswith("mpk-mi355x")
