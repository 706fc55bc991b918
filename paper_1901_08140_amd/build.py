"""Build libswarm.so (HIP for gfx950) in-tree with hipcc.

Flags: -O3 for gfx950 only; -ffp-contract=off so that only explicitly written fused
multiply-adds are fused (identical per-electron arithmetic in every kernel variant);
packed FP32 instructions disabled (the code is written for scalar FP32 lanes)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libswarm.so")
SOURCES = ["swarm_kernels.hip", "swarm_api.cpp", "swarm_batch.cpp", "swarm_server.cpp", "swarm_noalloc.cpp"]
ARCH = os.environ.get("SWARM_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
        cmd = ["hipcc", *lang, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-command-line-argument", "-Wno-unused-function",
               "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs)
    _wait(procs)
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs, "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def _wait(procs):
    errs = []
    for src, p in procs:
        _, err = p.communicate()
        lines = [l for l in (err or "").splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            errs.append(f"{src}:\n" + "\n".join(lines))
        elif lines:
            sys.stderr.write("\n".join(lines) + "\n")
    procs.clear()
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    build(verbose=True)
