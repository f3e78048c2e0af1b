"""The explicit waits of the staged reverse triangle passes, checked on the
compiled gfx950 code.

The staged passes load their inputs straight to LDS with asm the compiler
does not track, and order every read of that data with an explicit
`s_waitcnt vmcnt(N)`: vector memory operations complete in issue order, so
vmcnt(N) waits for every operation issued before the last N. A wait is
therefore correct only if, on every path through the kernel, at least N
vector memory operations were issued after the loads it waits for: after the
last direct load of any kind for a plain wait (the stores of the previous
batch's triangle come in between), after the last "late" load for a late
wait. This test compiles `rd_kernels.hip` to assembly (CPU only, no GPU) and
checks that property for every instance by a data-flow walk over each
kernel's basic blocks (minimum over paths, iterated to a fixed point round
the loop). The checker itself is pinned on small hand-written blocks where
the answer is known."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1705_02028_amd", "csrc")
INF = 10 ** 9
VMEM = ("global_store", "global_load", "scratch_store", "scratch_load", "buffer_")


def _blocks(body):
    """Basic blocks of one function's assembly: ordered names, their
    instructions (with the tags of staged loads and waits) and successors."""
    order, blocks, cur = ["entry"], {"entry": []}, "entry"
    for raw in body:
        s = raw.strip()
        lab = re.match(r"^(\.LBB\S+):", s)
        if lab or s.startswith("; %bb."):
            cur = lab.group(1) if lab else s.split()[1]
            order.append(cur)
            blocks[cur] = []
            continue
        if not s or s.startswith(";") or s.startswith("."):
            continue
        blocks[cur].append(s)
    succ = {}
    for i, b in enumerate(order):
        ins = blocks[b]
        targets = [m.group(1) for x in ins for m in [re.match(r"s_c?branch\S*\s+(\S+)", x)] if m]
        last = ins[-1] if ins else ""
        if not (last.startswith("s_branch") or last.startswith("s_endpgm")) and i + 1 < len(order):
            targets.append(order[i + 1])
        succ[b] = [t for t in targets if t in blocks]
    return order, blocks, succ


def check(body):
    """Returns (waits checked, violations) for one function: each item is
    (N, issued-after count on the worst path, late?)."""
    order, blocks, succ = _blocks(body)
    start = {b: None for b in order}
    start["entry"] = (INF, INF)
    seen = {}
    for _ in range(4 * len(order) + 8):
        changed = False
        for b in order:
            if start[b] is None:
                continue
            anyl, late = start[b]
            for x in blocks[b]:
                op = x.split()[0]
                if op.startswith("global_load_lds"):
                    if "staged load" not in x:
                        raise AssertionError("direct load to LDS without a staged tag: " + x)
                    anyl = 0
                    late = 0 if "staged load: late" in x else (late + 1 if late < INF else INF)
                elif op.startswith(VMEM):
                    anyl = anyl + 1 if anyl < INF else INF
                    late = late + 1 if late < INF else INF
                elif op == "s_waitcnt" and "staged wait" in x:
                    n = int(re.search(r"vmcnt\((\d+)\)", x).group(1))
                    is_late = "staged wait: late" in x
                    seen[(b, x)] = (n, late if is_late else anyl, is_late)
                    if n == 0:
                        anyl = late = INF
            for t in succ[b]:
                new = (anyl, late) if start[t] is None else (min(start[t][0], anyl), min(start[t][1], late))
                if new != start[t]:
                    start[t] = new
                    changed = True
        if not changed:
            break
    waits = list(seen.values())
    return waits, [w for w in waits if w[0] > 0 and w[1] < w[0]]


def functions(asm, pattern):
    out = {}
    for m in re.finditer(r"^(_Z\S*" + pattern + r"\S*):\s*(;.*)?$", asm, re.M):
        end = asm.index(".Lfunc_end", m.end())
        out[m.group(1)] = asm[m.end():end].split("\n")
    return out


def test_checker_on_known_blocks():
    # three stores after the loads: vmcnt(3) is enough, vmcnt(4) is not
    ok = ["global_load_lds_dwordx4 v[0:1], off ; staged load", "global_store_dwordx4 v[2:3], v[4:7], off",
          "global_store_dwordx4 v[2:3], v[4:7], off", "global_store_dwordx4 v[2:3], v[4:7], off",
          "s_waitcnt vmcnt(3) ; staged wait", "s_endpgm"]
    assert check(ok)[1] == []
    assert check([x.replace("vmcnt(3)", "vmcnt(4)") for x in ok])[1] == [(4, 3, False)]
    # a branch that skips one store makes the worst path count 2
    br = ["global_load_lds_dwordx4 v[0:1], off ; staged load", "global_store_dwordx4 v[2:3], v[4:7], off",
          "global_store_dwordx4 v[2:3], v[4:7], off", "s_cbranch_execz .LBB0_2", "; %bb.1:",
          "global_store_dwordx4 v[2:3], v[4:7], off", ".LBB0_2:", "s_waitcnt vmcnt(3) ; staged wait", "s_endpgm"]
    assert check(br)[1] == [(3, 2, False)]
    # a late wait counts from the last late load, past later plain loads
    late = ["global_load_lds_dwordx4 v[0:1], off ; staged load: late",
            "global_load_lds_dwordx4 v[0:1], off ; staged load", "global_load_lds_dword v[0:1], off ; staged load",
            "s_waitcnt vmcnt(2) ; staged wait: late", "s_waitcnt vmcnt(3) ; staged wait: late", "s_endpgm"]
    assert check(late)[1] == [(3, 2, True)]
    # round a loop: the back edge brings in the path without the stores
    loop = ["global_load_lds_dwordx4 v[0:1], off ; staged load", "global_store_dwordx4 v[2:3], v[4:7], off",
            ".LBB1_1:", "s_waitcnt vmcnt(1) ; staged wait", "global_load_lds_dwordx4 v[0:1], off ; staged load",
            "s_cbranch_scc1 .LBB1_1", "s_endpgm"]
    assert check(loop)[1] == [(1, 0, False)]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_staged_reverse_passes_wait_counts(tmp_path):
    out = tmp_path / "k.s"
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-S", "--cuda-device-only",
           os.path.join(CSRC, "rd_kernels.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    asm = out.read_text()
    fns = functions(asm, "k_adj_tri_staged")
    assert len(fns) == 10  # five schemes, two stages
    for name, body in fns.items():
        waits, bad = check(body)
        assert bad == [], (name, bad)
        ns = sorted({w[0] for w in waits})
        assert 0 in ns and any(w[2] for w in waits) and any(w[0] > 0 and not w[2] for w in waits), (name, ns)
