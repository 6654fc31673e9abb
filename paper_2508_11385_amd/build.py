"""Build libcoot.so in-tree for gfx950.

The host C++ sources and the hand-written HIP kernels are compiled with hipcc;
generated kernels are compiled at run time by hipRTC, which needs the device
header embedded in the library (written here as a C++ raw-string literal).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libcoot.so")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


DEVICE_HEADERS = ("coot_dev.h", "coot_exp.h", "exp_tables.h", "coot_log.h", "log_tables.h")


def _embed_header() -> str:
    """Write the device headers into a C++ file as raw-string literals (name, text pairs)."""
    delim = "COOTDEV"
    parts = []
    for name in DEVICE_HEADERS:
        text = open(os.path.join(CSRC, "device", name)).read()
        assert ")" + delim + '"' not in text
        parts.append('  {"' + name + '", R"' + delim + "(" + text + ")" + delim + '"},')
    body = ("namespace coot {\nstruct EmbeddedHeader { const char* name; const char* text; };\n"
            "extern const EmbeddedHeader kDeviceHeaders[];\nextern const int kNumDeviceHeaders;\n"
            "const EmbeddedHeader kDeviceHeaders[] = {\n" + "\n".join(parts) + "\n};\n"
            "const int kNumDeviceHeaders = " + str(len(parts)) + ";\n}\n")
    out = os.path.join(BUILD, "coot_dev_embed.cpp")
    if not os.path.exists(out) or open(out).read() != body:
        with open(out, "w") as f:
            f.write(body)
    return out


def sources():
    host = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".cpp"))
    kern = sorted(os.path.join(CSRC, "kernels", f) for f in os.listdir(os.path.join(CSRC, "kernels"))
                  if f.endswith(".hip")) if os.path.isdir(os.path.join(CSRC, "kernels")) else []
    return host, kern


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source of libcoot for gfx950 and link libcoot.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    host, kern = sources()
    embed = _embed_header()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    procs = []
    for src in host + [embed] + kern:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        # hand-written kernels: keep SimplifyCFG from sinking the register-file stores of the batch
        # interpreter's switch into one indexed store (that would demote the registers to scratch)
        lang = ["-x", "hip", "-mllvm", "-simplifycfg-sink-common=false"] if src.endswith(".hip") else []
        cmd = [hipcc] + HIP_FLAGS + inc + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + \
          ["-L/opt/rocm/lib", "-lhiprtc", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def _drain(procs):
    while procs:
        src, p = procs.pop(0)
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            raise RuntimeError(f"compile failed: {src}\n{text}")
        noise = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if noise:
            sys.stderr.write("\n".join(noise) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
