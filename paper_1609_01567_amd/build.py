"""Build the decoder's shared library (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libldpc_hip.so")
# per-kernel register, scratch and occupancy figures of the last build (compiler remarks)
RESOURCES = os.path.join(PKG, "libldpc_hip.resources.json")
SOURCES = ["graph.cpp", "decode.hip", "engine.hip", "serve.cpp"]
ARCH = os.environ.get("LDPC_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from emitting packed fp32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add contraction: the check and bit rules are inlined
    # into many kernels, and each must round every operation the same way
    # (fused operations are written out as fmaf where they are wanted)
    "-ffp-contract=off",
    "-fvisibility=hidden", "-DLDPC_BUILD", "-pthread",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


_REMARK_KEYS = {"VGPRs": "vgpr", "AGPRs": "agpr", "TotalSGPRs": "sgpr", "ScratchSize [bytes/lane]": "scratch",
                "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "lds"}


def parse_resource_remarks(text: str) -> dict:
    """{mangled kernel name: {vgpr, agpr, sgpr, scratch, occupancy, lds}} from the
    compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+(?:\[[^\]]*\])?): (\d+)", line)
        if m and cur is not None and m.group(1).strip() in _REMARK_KEYS:
            cur[_REMARK_KEYS[m.group(1).strip()]] = int(m.group(2))
    return out


def build_library(verbose: bool = False) -> str:
    """Compile csrc/*.{cpp,hip} into libldpc_hip.so next to this file.

    Each source compiles to its own object in a separate hipcc process (in
    parallel), then one hipcc call links the shared library.
    """
    import tempfile
    with tempfile.TemporaryDirectory(prefix="ldpc_build_") as tmpdir:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src + ".o")
            cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", "-o", obj,
                   os.path.join(CSRC, src)]
            if src.endswith(".hip"):
                cmd.append("-Rpass-analysis=kernel-resource-usage")
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        resources = {}
        for src, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                failed.append(src)
            elif src.endswith(".hip"):
                resources.update(parse_resource_remarks(out))
        if failed:
            raise RuntimeError(f"hipcc failed to compile {', '.join(failed)}")
        tmp = LIB + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed to link libldpc_hip.so")
    os.replace(tmp, LIB)
    with open(RESOURCES + ".tmp", "w") as f:
        json.dump(resources, f, indent=0, sort_keys=True)
    os.replace(RESOURCES + ".tmp", RESOURCES)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
