"""Check the gfx950 assembly of the kernels for barriers in divergent loops,
for barriers not preceded by a wait for the wave's LDS operations, for
scratch use, and for static LDS in the scan kernels.

A workgroup barrier (s_barrier) is counted per wave: a wave arrives when its
active lanes reach it.  If the compiler gives a loop that holds a barrier a
divergent exit (some lanes of a wave leave the loop while the others go round
again), the lanes that stayed pass the barrier without the ones that left, and
any value those lanes publish for the next iteration is never seen: the
workgroup can spin for ever.  The optimizer produces such loops from code like

    for (;;) {
        if (threadIdx.x == 0) next = fetch();   // head
        __syncthreads();
        ...
        if (threadIdx.x == 0) publish();        // tail
    }

by threading the tail's branch straight into the head's.  This module reads
the assembly that hipcc writes with ``-save-temps`` (its loop annotations name
every block's innermost loop and every loop's parent) and reports each loop
that holds a barrier and also removes lanes from exec
(``s_andn2_b64 exec, exec, ...``) in one of its own blocks.

    python paper_1704_02278_amd/isa_check.py file.s [...]
"""

from __future__ import annotations

import re
import sys
from pathlib import Path

_FUNC = re.compile(r"^([A-Za-z_][\w.$]*):\s*;\s*@")
_END = re.compile(r"^\.Lfunc_end\d+:")
_LABEL = re.compile(r"^(\.LBB\d+_\d+):|^; %bb\.(\d+):")
_HEADER = re.compile(r"=>\s*This (?:Inner )?Loop Header: Depth=(\d+)")
_IN_LOOP = re.compile(r"in Loop: Header=BB(\d+_\d+) Depth=(\d+)")
_PARENT = re.compile(r"Parent Loop BB(\d+_\d+) Depth=(\d+)")
_DROP_LANES = re.compile(r"^\s*s_andn2_b64\s+exec,\s*exec,")
_BARRIER = re.compile(r"^\s*s_barrier\b")


def _functions(lines):
    name, body = None, []
    for line in lines:
        m = _FUNC.match(line)
        if m:
            name, body = m.group(1), []
            continue
        if name is None:
            continue
        if _END.match(line):
            yield name, body
            name = None
            continue
        body.append(line)


def _blocks(body):
    """Split a kernel into blocks: (own loop id, annotation text, instruction lines)."""
    blocks = []
    for line in body:
        lm = _LABEL.match(line)
        if lm:
            own = lm.group(1)[len(".LBB"):] if lm.group(1) else None
            blocks.append([own, line, [], True])
            continue
        if not blocks:
            continue
        stripped = line.strip()
        if stripped.startswith(";") and blocks[-1][3]:
            blocks[-1][1] += "\n" + stripped  # annotation lines right after the label
            continue
        blocks[-1][3] = False
        blocks[-1][2].append(line)
    return [(own, note, insts) for own, note, insts, _ in blocks]


_WAIT_LGKM0 = re.compile(r"^\s*s_waitcnt\b.*lgkmcnt\(0\)")
_DS = re.compile(r"^\s*ds_")
_ANY_LABEL = re.compile(r"^\S+:")


def unwaited_barriers(body):
    """Barriers that can be reached with the wave's LDS operations in flight.

    Other waves read, right after a barrier, what this wave's LDS atomics and
    stores wrote before it; the kernels wait for them explicitly (lgkmcnt(0))
    just before each barrier, because the compiler's own barrier omitted that
    wait on some paths.  Walking back from each s_barrier within its block,
    an ``s_waitcnt ... lgkmcnt(0)`` must come before any DS instruction and
    before the block's start.
    """
    bad = []
    for i, line in enumerate(body):
        if not _BARRIER.match(line):
            continue
        ok = False
        for j in range(i - 1, -1, -1):
            prev = body[j]
            if _WAIT_LGKM0.match(prev):
                ok = True
                break
            if _DS.match(prev) or _ANY_LABEL.match(prev):
                break
        if not ok:
            bad.append(i)
    return bad


def check_function(body):
    """Return a list of problems (strings) for one kernel's assembly."""
    parent = {}  # loop header -> enclosing loop header (None at depth 1)
    rows = []    # (innermost loop of the block, holds barrier, drops lanes)
    for own, note, insts in _blocks(body):
        loop = None
        if _HEADER.search(note) and own is not None:
            loop = own
            ps = sorted((int(d), h) for h, d in _PARENT.findall(note))
            parent[own] = ps[-1][1] if ps else None
            for (_, a), (_, b) in zip(ps, ps[1:]):
                parent.setdefault(b, a)
            if ps:
                parent.setdefault(ps[0][1], None)
        else:
            im = _IN_LOOP.search(note)
            if im:
                loop = im.group(1)
        rows.append((loop, any(_BARRIER.match(i) for i in insts), any(_DROP_LANES.match(i) for i in insts)))

    def ancestors(h):
        seen = []
        while h is not None and h not in seen:
            seen.append(h)
            h = parent.get(h)
        return seen

    holds_barrier = set()
    for loop, bar, _ in rows:
        if bar and loop is not None:
            holds_barrier.update(ancestors(loop))
    problems = {f"loop BB{loop} holds s_barrier and has a divergent exit"
                for loop, _, drop in rows if drop and loop in holds_barrier}
    return sorted(problems)


_KD = re.compile(r"^\s*\.amdhsa_kernel\s+(\S+)")
_PRIVATE = re.compile(r"^\s*\.amdhsa_private_segment_fixed_size\s+(\d+)")
_GROUP = re.compile(r"^\s*\.amdhsa_group_segment_fixed_size\s+(\d+)")
# Kernels whose LDS tables must start at address 0 (no static LDS): the scan
# kernels address their filter blocks by the masked hash alone.
_NO_STATIC_LDS = "glop_scan_kernel"


def group_sizes(lines):
    """Static LDS bytes of every kernel, from its kernel descriptor."""
    out, name = {}, None
    for line in lines:
        m = _KD.match(line)
        if m:
            name = m.group(1)
            continue
        m = _GROUP.match(line)
        if m and name is not None:
            out[name] = int(m.group(1))
    return out


def scratch_sizes(lines):
    """Per-lane scratch bytes of every kernel, from its kernel descriptor."""
    out, name = {}, None
    for line in lines:
        m = _KD.match(line)
        if m:
            name = m.group(1)
            continue
        m = _PRIVATE.match(line)
        if m and name is not None:
            out[name] = int(m.group(1))
            name = None
    return out


def check_file(path):
    """Problems in every kernel of one assembly file: {kernel: [problems]}.

    Besides barriers in divergent loops, a kernel that uses scratch memory (a
    register spill) is a problem: the kernels are written to fit their
    register budget, and a spill slot is memory no test of the result covers.
    """
    lines = Path(path).read_text().splitlines()
    out = {}
    for name, body in _functions(lines):
        p = check_function(body)
        if "glop_" in name:
            p += [f"s_barrier at body line {i} without a preceding lgkmcnt(0) wait" for i in unwaited_barriers(body)]
        if p:
            out[name] = p
    for name, size in scratch_sizes(lines).items():
        if size > 0:
            out.setdefault(name, []).append(f"uses {size} bytes of scratch per lane (register spill)")
    for name, size in group_sizes(lines).items():
        if _NO_STATIC_LDS in name and size > 0:
            out.setdefault(name, []).append(f"has {size} bytes of static LDS (its tables must start at address 0)")
    return out


def main(argv):
    bad = 0
    for path in argv:
        for name, probs in check_file(path).items():
            bad += 1
            for p in probs:
                print(f"{path}: {name}: {p}")
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
