"""Build the HIP library ``libsnn.so`` for gfx950 (MI355X) in-tree.

hipcc compiles every ``csrc/*.hip`` file for the gfx950 offload target and
links one shared library exporting the C ABI of ``include/snn.h``.  Packed
FP32 instructions are disabled (``-packed-fp32-ops``).  The compiler's
per-kernel resource report (registers, scratch, occupancy) is kept beside the
library as ``libsnn.resources.json``: a kernel that starts using scratch
memory (register spills to HBM) loses several times its speed, and the tests
check that none does.
"""
from __future__ import annotations

import glob
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsnn.so")
RESOURCES = os.path.join(HERE, "libsnn.resources.json")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


_REMARK = re.compile(r"remark:\s+(?:Function Name: (\S+)|(VGPRs|AGPRs|SGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]): (\d+))")
_EXCERPT = re.compile(r"^\s*\d*\s*\|")
_KEYS = {"VGPRs": "vgpr", "AGPRs": "agpr", "SGPRs": "sgpr", "ScratchSize [bytes/lane]": "scratch",
         "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "static_lds"}


def parse_resources(text: str) -> dict:
    """Per-kernel figures from hipcc's kernel-resource-usage remarks."""
    out, cur = {}, None
    for m in _REMARK.finditer(text):
        if m.group(1):
            cur = out.setdefault(m.group(1), {})
        elif cur is not None:
            cur[_KEYS[m.group(2)]] = int(m.group(3))
    return out


def build(verbose: bool = False, jobs: int = 8) -> str:
    objdir = tempfile.mkdtemp(prefix="snn_build_")
    objs, procs, logs = [], [], []

    def finish(pr, log):
        if pr.wait() != 0:
            with open(log) as f:
                sys.stderr.write("".join(ln for ln in f if "remark:" not in ln))
            raise RuntimeError("hipcc failed")

    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        log = obj + ".log"
        lang = ["-x", "hip", "-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        with open(log, "w") as f:
            procs.append((subprocess.Popen(cmd, stderr=f), log))
        objs.append(obj)
        logs.append(log)
        if len(procs) >= jobs:
            finish(*procs.pop(0))
    for pr, log in procs:
        finish(pr, log)
    resources = {}
    for log in logs:
        with open(log) as f:
            text = f.read()
        resources.update(parse_resources(text))
        # what remains besides the remarks and their source excerpts (the host
        # pass not knowing the GPU-only packed-FP32 feature is harmless)
        rest = "".join(ln for ln in text.splitlines(True)
                       if "remark:" not in ln and "packed-fp32-ops" not in ln and not _EXCERPT.match(ln))
        if rest.strip():
            sys.stderr.write(rest)
        os.remove(log)
    for name, r in sorted(resources.items()):
        if r.get("scratch", 0):
            print(f"warning: kernel {name} uses {r['scratch']} bytes of scratch per lane", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(RESOURCES, "w") as f:
        json.dump(resources, f, indent=1, sort_keys=True)
    for o in objs:
        os.remove(o)
    os.rmdir(objdir)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
