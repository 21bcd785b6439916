"""Barriers inside lane-divergent loops, found in the gfx950 code objects
this repository builds (test infrastructure).

The device code of a built object (`.hip_fatbin` section, one clang offload
bundle) is unbundled and disassembled with the ROCm LLVM tools; each
function's instructions are split into basic blocks and natural loops are
found from the CFG (back-edge u -> h with h dominating u).  A loop is
lane-divergent when one of its latches takes lanes out of exec
(`s_andn2_b64 exec, exec, m`, how the compiler lowers a loop exit that
differs between lanes): the wave keeps running it while any lane is left
in it.  A branch on exec alone (`s_cbranch_execz/nz`) changes no lane's
exec and does not make a loop divergent.  A barrier in such a loop can be met by part of a wave while another
part of the same wave is parked outside the loop, so the block's barriers
no longer line up with the program's, which is how a claim-and-publish
loop that tests `threadIdx.x == 0` at its head and latch can compile into
a loop that never ends.
"""
import os
import re
import subprocess

LLVM = "/opt/rocm/llvm/bin"
FN = re.compile(r"^([0-9a-f]+) <(.+)>:$")
INS = re.compile(r"^\s+(\S+)\s*(.*?)\s*//\s*([0-9A-F]+):[^<]*(?:<(.+)\+0x([0-9a-f]+)>)?")
UNCOND = {"s_branch"}
ENDS = {"s_endpgm", "s_setpc_b64", "s_endpgm_saved"}


def disasm(obj, tmp):
    fb = os.path.join(tmp, "fb")
    co = os.path.join(tmp, "co")
    subprocess.run([f"{LLVM}/llvm-objcopy", "-O", "binary", "--only-section=.hip_fatbin", obj, fb], check=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fb}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True)
    r = subprocess.run([f"{LLVM}/llvm-objdump", "-d", "--mcpu=gfx950", co], check=True,
                       capture_output=True, text=True)
    return r.stdout


def functions(text):
    cur, out, base = None, {}, 0
    for ln in text.splitlines():
        m = FN.match(ln)
        if m:
            cur = m.group(2)
            out[cur] = []
            base = int(m.group(1), 16)
            continue
        if cur is None:
            continue
        m = INS.match(ln)
        if not m:
            continue
        addr = int(m.group(3), 16) - base
        tgt = int(m.group(5), 16) if m.group(5) and m.group(4) == cur else None
        out[cur].append((addr, m.group(1), m.group(2).replace(" ", ""), tgt))
    return out


def cfg(ins):
    addrs = [a for a, _, _, _ in ins]
    leaders = {addrs[0]} if addrs else set()
    for i, (a, op, _, t) in enumerate(ins):
        if t is not None:
            leaders.add(t)
        if (op.startswith("s_cbranch") or op in UNCOND or op in ENDS) and i + 1 < len(ins):
            leaders.add(ins[i + 1][0])
    blocks, cur = [], []
    for x in ins:
        if x[0] in leaders and cur:
            blocks.append(cur)
            cur = []
        cur.append(x)
    if cur:
        blocks.append(cur)
    index = {b[0][0]: i for i, b in enumerate(blocks)}
    succ = []
    for i, b in enumerate(blocks):
        a, op, _, t = b[-1]
        s = []
        if t is not None and t in index and (op.startswith("s_cbranch") or op in UNCOND):
            s.append(index[t])
        if op not in UNCOND and op not in ENDS and i + 1 < len(blocks):
            s.append(i + 1)
        succ.append(s)
    return blocks, succ


def dominators(n, succ):
    pred = [[] for _ in range(n)]
    for u, ss in enumerate(succ):
        for v in ss:
            pred[v].append(u)
    # reverse postorder from block 0
    order, seen, stack = [], [False] * n, [(0, 0)]
    seen[0] = True
    while stack:
        u, k = stack.pop()
        if k < len(succ[u]):
            stack.append((u, k + 1))
            v = succ[u][k]
            if not seen[v]:
                seen[v] = True
                stack.append((v, 0))
        else:
            order.append(u)
    rpo = order[::-1]
    pos = {u: i for i, u in enumerate(rpo)}
    idom = [None] * n
    idom[0] = 0

    def inter(a, b):
        while a != b:
            while pos[a] > pos[b]:
                a = idom[a]
            while pos[b] > pos[a]:
                b = idom[b]
        return a

    changed = True
    while changed:
        changed = False
        for u in rpo[1:]:
            ps = [p for p in pred[u] if idom[p] is not None and p in pos]
            if not ps:
                continue
            d = ps[0]
            for p in ps[1:]:
                d = inter(p, d)
            if idom[u] != d:
                idom[u] = d
                changed = True
    return idom, pred, pos


def dominates(idom, h, u):
    while True:
        if u == h:
            return True
        if idom[u] is None or idom[u] == u:
            return u == h
        u = idom[u]


def divergent_loops_with_barriers(ins):
    """Messages, one per lane-divergent natural loop that holds a barrier."""
    if not ins:
        return []
    blocks, succ = cfg(ins)
    idom, pred, pos = dominators(len(blocks), succ)
    body, latches = {}, {}
    for u in pos:
        for h in succ[u]:
            if not dominates(idom, h, u):
                continue
            latches.setdefault(h, set()).add(u)
            b = body.setdefault(h, {h})
            stack = [u]
            while stack:
                x = stack.pop()
                if x not in b:
                    b.add(x)
                    stack.extend(pred[x])
    problems = []
    for h, b in body.items():
        divergent = any(op == "s_andn2_b64" and args.startswith("exec,exec,")
                        for u in latches[h] for (_, op, args, _) in blocks[u])
        bars = [a for x in b for (a, op, _, _) in blocks[x] if op == "s_barrier"]
        if divergent and bars:
            problems.append(f"lane-divergent loop at {blocks[h][0][0]:#x} ({len(b)} blocks) "
                            f"holds {len(bars)} barrier(s)")
    return problems


def main_loop(ins):
    """Instructions (address order) of the function's largest natural loop."""
    if not ins:
        return []
    blocks, succ = cfg(ins)
    idom, pred, pos = dominators(len(blocks), succ)
    best = set()
    for u in pos:
        for h in succ[u]:
            if not dominates(idom, h, u):
                continue
            b, stack = {h}, [u]
            while stack:
                x = stack.pop()
                if x not in b:
                    b.add(x)
                    stack.extend(pred[x])
            if sum(len(blocks[x]) for x in b) > sum(len(blocks[x]) for x in best):
                best = b
    return sorted((i for x in best for i in blocks[x]), key=lambda t: t[0])


def waits_before_first_barrier(loop):
    """vmcnt waits between the loop's first global load (its prefetch) and
    the first barrier after that load, in address order, that wait for one
    of those loads: vmcnt(k) with fewer than the loads issued since allowed
    outstanding (an older load's wait, vmcnt(k) with k >= those, is not
    listed)."""
    first = next((k for k, (_, op, _, _) in enumerate(loop) if op.startswith("global_load")), None)
    if first is None:
        return None
    out, issued = [], 0
    for a, op, args, _ in loop[first:]:
        if op == "s_barrier":
            return out
        if op.startswith("global_load"):
            issued += 1
        if op == "s_waitcnt" and "vmcnt" in args:
            k = int(re.search(r"vmcnt\((\d+)\)", args).group(1))
            if k < issued:
                out.append((a, args))
    return out


def scan_object(obj, tmpdir):
    """{function name: messages} for every function of `obj` with a finding."""
    out = {}
    for fn, ins in functions(disasm(obj, tmpdir)).items():
        p = divergent_loops_with_barriers(ins)
        if p:
            out[fn] = p
    return out


def tools_present():
    return all(os.path.exists(os.path.join(LLVM, t))
               for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump"))
