"""Structural checks of the gfx950 code the compiler emits for the kernels.

The persistent level-blocked kernel relies on two properties that source
review alone cannot guarantee:

* its task loop must be left by all lanes together.  If the compiler cannot
  prove the loop control uniform it may restructure the loop so that some
  lanes exit early (an exec-mask exit), which breaks the barriers inside it
  and can stall the workgroup forever;
* results must be stored write-through (agent scope) and have completed
  before the flag store publishes them, and a consumer must invalidate
  before reading (acquire).

These tests compile kernels.hip to AMD assembly (CPU only) and check both.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2405_12525_amd", "csrc", "kernels.hip")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-S",
           "--cuda-device-only", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2405_12525_amd/csrc", "-o", str(out), SRC]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def kernels(asm_text, name):
    """{symbol: [lines]} for every kernel whose mangled name contains `name`:
    the lines from its label to the end-of-function marker (a kernel may
    hold several s_endpgm, e.g. an early return placed first)."""
    out = {}
    cur = None
    for line in asm_text.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m and name in m.group(1):
            cur = m.group(1)
            out[cur] = []
            continue
        if cur is not None:
            if line.startswith(".Lfunc_end"):
                cur = None
                continue
            out[cur].append(line)
    return out


def loops_with_barrier_and_divergent_exit(lines):
    """Loops that contain a barrier (directly or in a nested loop) and are
    left through an exec-mask exit, i.e. not by all lanes together."""
    parent = {}      # loop header -> enclosing loop header
    own = {}         # loop header -> instructions of blocks directly in it
    cur = None       # innermost loop of the current block
    pending = []     # "Parent Loop" headers listed for the block being read
    label = None
    for line in lines:
        m = re.match(r"^(\.LBB\S+|; %bb\.\d+):", line)
        if m:
            label = m.group(1).lstrip(".").lstrip("; %")
            pending = re.findall(r"Parent Loop (\S+) Depth", line)
            h = re.search(r"in Loop: Header=(\S+) Depth", line)
            cur = h.group(1) if h else None
            continue
        pm = re.findall(r"Parent Loop (\S+) Depth", line)
        if pm and line.strip().startswith(";"):
            pending += pm
            continue
        if re.search(r"Loop Header: Depth=\d+", line):
            cur = label
            parent[cur] = pending[-1] if pending else None
            continue
        if cur is not None and not line.strip().startswith(";"):
            own.setdefault(cur, []).append(line.strip())
    def has_barrier(h):
        if any(l.startswith("s_barrier") for l in own.get(h, [])):
            return True
        return any(has_barrier(c) for c, p in parent.items() if p == h)
    bad = []
    for h in set(own) | set(parent):
        exits = [l for l in own.get(h, []) if l.startswith("s_andn2_b64 exec, exec")]
        if exits and has_barrier(h):
            bad.append(h)
    return bad


@pytest.mark.parametrize("name", ["lb_kernel", "lb_acc_kernel", "lb_sell_kernel",
                                  "lb_sell_acc_kernel"])
def test_task_loop_has_uniform_exit(asm, name):
    ks = kernels(asm, name)
    assert len(ks) == 12  # 6 right-hand-side variants x 2 value types
    for sym, lines in ks.items():
        assert any("s_barrier" in l for l in lines)
        assert loops_with_barrier_and_divergent_exit(lines) == [], sym


@pytest.mark.parametrize("name", ["xcd_kernel", "lbs_kernel", "xcd_acc_kernel", "lbs_acc_kernel"])
def test_other_task_loops_have_uniform_exit(asm, name):
    ks = kernels(asm, name)
    assert len(ks) == 12
    for sym, lines in ks.items():
        assert loops_with_barrier_and_divergent_exit(lines) == [], sym


def test_baseline_row_loop_has_uniform_exit(asm):
    ks = kernels(asm, "spmv_power_kernel")
    assert len(ks) == 24  # with and without the weighted sums
    for sym, lines in ks.items():
        assert loops_with_barrier_and_divergent_exit(lines) == [], sym


def test_sliced_layout_kernels_need_no_lds():
    """The sliced-layout kernels hold no LDS, so that their occupancy is set
    by registers alone (up to eight waves per SIMD)."""
    import subprocess
    out = subprocess.run(
        [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
         "-target-feature", "-Xclang", "-packed-fp32-ops", "-c", f"-I{ROOT}/include",
         f"-I{ROOT}/paper_2405_12525_amd/csrc", "-Rpass-analysis=kernel-resource-usage",
         "--cuda-device-only", "-o", os.devnull, SRC], capture_output=True, text=True).stderr
    names = re.findall(r"Function Name: (\S+)", out)
    lds = re.findall(r"LDS Size \[bytes/block\]: (\d+)", out)
    assert len(names) == len(lds) > 0
    sell = [(n, int(b)) for n, b in zip(names, lds)
            if "sell_kernel" in n or "sell_acc_kernel" in n]
    assert len(sell) >= 4 * 12
    for n, b in sell:
        assert b <= 64, n   # the ticket and status words of the persistent kernels


def _instructions_with_loop_flag(lines):
    """(instruction, inside a loop) for the kernel's instructions in order."""
    out, in_loop = [], False
    for line in lines:
        if re.match(r"^(\.LBB\S+|; %bb\.\d+):", line):
            in_loop = "in Loop:" in line
            continue
        if "Loop Header:" in line:
            in_loop = True
            continue
        t = line.strip()
        if t and not t.startswith(";") and not t.startswith("."):
            out.append((t, in_loop))
    return out


def _publish_ok(lines):
    """Every flag store inside the task loop (a dword store at agent scope)
    follows a barrier that is entered only through an s_waitcnt vmcnt(0):
    between that wait and the barrier lie neither labels nor global, buffer,
    flat or scratch memory instructions (scalar and vector arithmetic and LDS
    may), and no vector memory instruction lies between that barrier and the
    store."""
    ins = _instructions_with_loop_flag(lines)
    flags = [t for t, loop in ins if loop and re.match(r"global_store_dword .* sc1", t)]
    assert flags
    raw = [l.strip() for l in lines if l.strip() and not l.strip().startswith(";")]
    n_checked = 0
    for f, line in enumerate(raw):
        if not (re.match(r"global_store_dword .* sc1", line) and line in flags):
            continue
        b = max(j for j in range(f) if raw[j].startswith("s_barrier"))
        w = b - 1
        while not re.match(r"s_waitcnt .*vmcnt\(0\)", raw[w]):
            assert not raw[w].startswith(("global_", "buffer_", "flat_", "scratch_")), raw[w:b + 1]
            assert not re.match(r"^\.LBB", raw[w]) and not raw[w].endswith(":"), raw[w:b + 1]
            w -= 1
            assert w > 0, raw[b - 3:b + 1]
        between = [l for l in raw[b + 1:f] if l.startswith(("global_", "buffer_", "flat_"))
                   or re.match(r"^\.LBB", l)]
        assert not between, between
        n_checked += 1
    assert n_checked >= 1


@pytest.mark.parametrize("name", ["lb_kernel", "xcd_kernel", "lbs_kernel", "lb_acc_kernel",
                                  "xcd_acc_kernel", "lbs_acc_kernel", "lb_sell_kernel",
                                  "lb_sell_acc_kernel"])
def test_results_write_through_and_publish_after_completion(asm, name):
    for sym, lines in kernels(asm, name).items():
        body = [l.strip() for l in lines if l.strip() and not l.strip().startswith(";")]
        # results: 64-bit stores at agent scope (sc1), no L2 write-back anywhere
        assert any(re.match(r"global_store_dwordx2 .* sc1", l) for l in body), sym
        assert not any(re.match(r"global_store_dwordx2 ", l) and " sc1" not in l for l in body), sym
        assert not any(l.startswith("buffer_wbl2") for l in body), sym
        assert any(l.startswith("buffer_inv sc1") for l in body), sym
        _publish_ok(lines)
