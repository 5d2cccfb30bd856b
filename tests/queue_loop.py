"""Static check of the register kernel's work-queue loop in the built code.

The work-queue kernel must run thread 0's queue hand-over (the pop of the
next group) on every trip around the loop that reads the group code: if the
compiler gives the other threads a loop of their own around the group code
that bypasses the hand-over, those threads never see a new group and the
work-group hangs at its next barrier.  This module takes the gfx950 code
object of the kernel's object file, disassembles it (llvm-objdump, our own
build), builds each wave_queue_kernel's control-flow graph, finds the natural
loops (back edges to a dominating header), and checks that every loop
containing the read of the group code (the first LDS read after the first
barrier that follows the pop) also contains the pop (a returning
global_atomic_add at offset 0 of the queue control words).
"""

from __future__ import annotations

import collections
import os
import re
import shutil
import subprocess
import tempfile

LLVM = "/opt/rocm/llvm/bin"
_LINE = re.compile(r"^\s+(\S+)(.*?)\s*//\s*([0-9A-Fa-f]+):\s*[0-9A-Fa-f ]+(?:<(\S+)\+0x([0-9a-fA-F]+)>)?\s*$")
_FUNC = re.compile(r"^([0-9a-f]+) <(\S+)>:$")


def tools_available():
    return all(os.path.exists(os.path.join(LLVM, t)) for t in ("llvm-objcopy", "clang-offload-bundler",
                                                               "llvm-objdump"))


def disassemble(obj_path, arch="gfx950"):
    """Disassembly of the device code object of a hipcc object file."""
    with tempfile.TemporaryDirectory() as tmp:
        fat = os.path.join(tmp, "fatbin")
        co = os.path.join(tmp, "code.o")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", obj_path,
                        os.path.join(tmp, "stripped.o")], check=True, capture_output=True)
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={fat}",
                        f"--targets=hipv4-amdgcn-amd-amdhsa--{arch}", f"--output={co}"],
                       check=True, capture_output=True)
        out = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--no-show-raw-insn", co],
                             check=True, capture_output=True, text=True)
    return out.stdout


def functions(text):
    """[(name, start address, [(addr, opcode, operands, target offset or None)])]."""
    funcs, cur = [], None
    for ln in text.splitlines():
        m = _FUNC.match(ln)
        if m:
            cur = (m.group(2), int(m.group(1), 16), [])
            funcs.append(cur)
            continue
        if cur is None:
            continue
        m = _LINE.match(ln)
        if m:
            op, rest, addr, _sym, off = m.groups()
            cur[2].append((int(addr, 16), op, rest, int(off, 16) if off else None))
    return funcs


def _cfg(start, ins):
    index = {a: i for i, (a, _, _, _) in enumerate(ins)}
    leaders, target = {0}, {}
    for i, (a, op, rest, off) in enumerate(ins):
        if op.startswith("s_branch") or op.startswith("s_cbranch"):
            t = start + off if off is not None else a + 4 + 4 * int(rest.split()[0])
            target[i] = index[t]
            leaders.add(index[t])
            if i + 1 < len(ins):
                leaders.add(i + 1)
        elif op in ("s_endpgm", "s_setpc_b64") and i + 1 < len(ins):
            leaders.add(i + 1)
    first = sorted(leaders)
    block = [0] * len(ins)
    for b, s0 in enumerate(first):
        for i in range(s0, first[b + 1] if b + 1 < len(first) else len(ins)):
            block[i] = b
    succ = [set() for _ in first]
    for b, s0 in enumerate(first):
        e = (first[b + 1] if b + 1 < len(first) else len(ins)) - 1
        op = ins[e][1]
        if op == "s_branch":
            succ[b].add(block[target[e]])
        elif op.startswith("s_cbranch"):
            succ[b].add(block[target[e]])
            if e + 1 < len(ins):
                succ[b].add(block[e + 1])
        elif op not in ("s_endpgm", "s_setpc_b64") and e + 1 < len(ins):
            succ[b].add(block[e + 1])
    return block, succ


def _loops(succ):
    nb = len(succ)
    pred = [set() for _ in range(nb)]
    for b in range(nb):
        for s in succ[b]:
            pred[s].add(b)
    reach, st = set(), [0]
    while st:
        x = st.pop()
        if x not in reach:
            reach.add(x)
            st.extend(succ[x])
    dom = [set(range(nb)) for _ in range(nb)]
    dom[0] = {0}
    changed = True
    while changed:
        changed = False
        for b in sorted(reach - {0}):
            ps = [dom[p] for p in pred[b] if p in reach]
            nd = (set.intersection(*ps) if ps else set()) | {b}
            if nd != dom[b]:
                dom[b], changed = nd, True
    loops = collections.defaultdict(set)
    for u in reach:
        for h in succ[u]:
            if h in dom[u]:                       # back edge u -> h
                body, st = {h, u}, ([u] if u != h else [])
                while st:
                    x = st.pop()
                    for p in pred[x]:
                        if p not in body and p in reach:
                            body.add(p)
                            st.append(p)
                loops[h] |= body
    return loops, reach


def _item_read(ins, block, succ, pop):
    """The first LDS read after the first barrier reachable from `pop`."""
    first_ins = {}
    for i, b in enumerate(block):
        first_ins.setdefault(b, i)
    pb = block[pop]
    seen, queue, bar = {pb}, collections.deque([pb]), None
    while queue and bar is None:
        b = queue.popleft()
        i = pop + 1 if b == pb else first_ins[b]
        while i < len(ins) and block[i] == b:
            if ins[i][1] == "s_barrier":
                bar = i
                break
            i += 1
        for s in sorted(succ[b]):
            if s not in seen:
                seen.add(s)
                queue.append(s)
    if bar is None:
        return None
    reads = [i for i in range(bar + 1, min(bar + 64, len(ins))) if ins[i][1].startswith("ds_read")]
    return reads[0] if reads else None


def check_queue_kernel(start, ins):
    """(ok, message) for one wave_queue_kernel's instructions: for every
    queue pop, every loop around the group-code read that follows it must
    also contain that pop, and the read must sit in a loop with it."""
    block, succ = _cfg(start, ins)
    loops, _ = _loops(succ)
    pops = [i for i, (_, op, rest, _) in enumerate(ins)
            if op == "global_atomic_add" and "sc0" in rest and "offset" not in rest]
    if not pops:
        return False, "no queue pop"
    for pop in pops:
        pb = block[pop]
        rd = _item_read(ins, block, succ, pop)
        if rd is None:
            return False, f"no barrier and LDS read after the pop at {ins[pop][0]:#x}"
        rb = block[rd]
        bad = [h for h, body in loops.items() if rb in body and pb not in body]
        if bad:
            return False, (f"the group code read at {ins[rd][0]:#x} is in {len(bad)} loop(s) "
                           f"without the queue pop at {ins[pop][0]:#x}")
    if not any(block[p] in body for p in pops for body in loops.values()):
        return False, "no queue pop inside a loop"
    return True, "ok"


def check_object(obj_path):
    """{kernel name: (ok, message)} for every wave_queue_kernel in obj_path."""
    out = {}
    for name, start, ins in functions(disassemble(obj_path)):
        if "wave_queue_kernel" in name:
            out[name] = check_queue_kernel(start, ins)
    return out
