"""Build the executor library (libhiccl.so) for gfx950 with hipcc, in-tree.

The library is the C-ABI boundary: host planner (csrc/plan.cpp) and device
code (csrc/*.hip). Run ``python -m paper_2408_05962_amd.build``.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhiccl.so")
SOURCES = ["plan.cpp", "device.hip", "serve.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep packed-fp32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, *FLAGS, *lang, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    write_isa_digest(bdir)
    return LIB


ISA_DIGEST = os.path.join(HERE, "_build", "device_isa.sha256")


def write_isa_digest(bdir: str) -> str:
    """sha256 of the gfx950 instructions of every kernel in device.hip (directives, comments and
    metadata left out). Host-only edits of the source leave it unchanged; any kernel change alters it.
    Measurements recorded against one digest (profiles/traffic_*.json) apply while it is unchanged."""
    src = os.path.join(CSRC, "device.hip")
    asm = os.path.join(bdir, "device_isa.s")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "--cuda-device-only", "-S", src, "-o", asm]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed for {src}:\n{r.stderr}")
    h = hashlib.sha256()
    with open(asm) as f:
        for line in f:
            s = line.rstrip("\n")
            if not s.startswith("\t") or s.startswith("\t.") or s.startswith("\t;"):
                continue
            h.update(s.split(";")[0].rstrip().encode() + b"\n")
    os.remove(asm)
    digest = h.hexdigest()
    with open(ISA_DIGEST, "w") as f:
        f.write(digest + "\n")
    return digest


def build_sanitized() -> str:
    """A host-sanitized library for the CPU tests: AddressSanitizer and UndefinedBehaviorSanitizer on the
    host code only (device code is built as usual). Run the CPU suite against it with
    HICCL_LIB=<path> LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)"
    ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu"."""
    bdir = os.path.join(HERE, "_build", "sanitize")
    os.makedirs(bdir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"]
        r = subprocess.run([HIPCC, *flags, *san, *lang, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        objs.append(obj)
    out = os.path.join(bdir, "libhiccl_sanitize.so")
    # the host linker adds the sanitizer runtimes; the device code is already embedded in the objects
    r = subprocess.run(["g++", "-shared", "-fPIC", "-fsanitize=address,undefined", *objs, "-L/opt/rocm/lib",
                        "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", out], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return out


if __name__ == "__main__":
    print(build_sanitized() if "--sanitize" in sys.argv else build(verbose="-v" in sys.argv))
