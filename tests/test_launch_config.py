"""Static check of the HIP sources: every kernel launch uses the block size its
kernel declares in __launch_bounds__, and every kernel is launched (CPU only)."""
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = sorted(glob.glob(os.path.join(ROOT, "paper_1308_4011_amd", "csrc", "*.hip")))


def _consts(text):
    return {k: int(v) for k, v in re.findall(r"constexpr int (\w+) = (\d+);", text)}


def test_launch_block_sizes_match_bounds():
    text = "\n".join(open(p).read() for p in SRC)
    text += open(os.path.join(ROOT, "paper_1308_4011_amd", "csrc", "mm_dev.h")).read()
    consts = _consts(text)
    bounds = {}
    for val, name in re.findall(r"__launch_bounds__\((\w+)\)\s+void\s+(\w+)", text):
        bounds[name] = int(val) if val.isdigit() else consts[val]
    launches = []
    for mt in re.finditer(r"(\w+)(?:<[\w:]+>)?<<<(.*?)>>>", text):
        args, depth, cur = [], 0, ""
        for ch in mt.group(2):
            if ch == "," and depth == 0:
                args.append(cur.strip())
                cur = ""
                continue
            depth += ch in "([{"
            depth -= ch in ")]}"
            cur += ch
        args.append(cur.strip())
        launches.append((mt.group(1), args[1]))
    assert launches
    seen = set()
    for name, block in launches:
        b = int(block) if block.isdigit() else consts[block]
        if name in bounds:
            assert b <= bounds[name], f"{name} launched with {b} threads, bounds {bounds[name]}"
            assert b == bounds[name], f"{name} launched with {b} threads, kernel sized for {bounds[name]}"
        seen.add(name)
    missing = set(bounds) - seen
    assert not missing, f"kernels never launched: {missing}"
