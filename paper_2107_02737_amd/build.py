"""Build the gfx950 shared library ``lib/libsp2.so`` from ``csrc/`` with hipcc.

The library is the product: the C ABI of ``include/sp2.h`` with the HIP
kernels behind it.  It is compiled for gfx950 only.
"""

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB_DIR = os.path.join(PKG, "lib")
LIB_PATH = os.path.join(LIB_DIR, "libsp2.so")
SOURCES = ["sp2_capi.hip"]   # includes every csrc/*.hpp
# measurement helper beside the solver (include/sp2_probe.h), its own library
PROBE_PATH = os.path.join(LIB_DIR, "libsp2_probe.so")
PROBE_SOURCES = ["sp2_probe.hip"]


def hipcc():
    path = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found (set HIPCC)")
    return path


def compile_command(out=LIB_PATH, sources=SOURCES):
    return [
        hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-mcode-object-version=5",
        # packed FP32 instructions stay off: the compiler must not form them
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        *[os.path.join(CSRC, s) for s in sources],
        "-o", out,
    ]


def _hot_loop_scratch(text, name):
    """Scratch (spill) instructions between the kernel's first and last MFMA
    instruction, i.e. inside its matrix-core loop.  -1 if it has no MFMA."""
    start = text.find("\n" + name + ":")
    if start < 0:
        return -1
    end = text.find(".Lfunc_end", start)
    lines = text[start:end].splitlines()
    idx = [i for i, line in enumerate(lines) if "v_mfma" in line]
    if not idx:
        return -1
    return sum("scratch_" in line for line in lines[idx[0]:idx[-1] + 1])


def kernel_resources():
    """Compile the device code to gfx950 assembly and return, per kernel, its
    scratch (private segment) bytes, VGPR count and VGPR/SGPR spill counts."""
    import re
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "sp2.s")
        cmd = [c for c in compile_command(out) if c not in ("-shared", "-fPIC")]
        cmd += ["--offload-device-only", "-S"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + res.stderr)
        text = open(out).read()
    kernels = {}
    meta = text[text.index("amdhsa.kernels:"):]
    for block in meta.split("\n  - ")[1:]:
        if ".name:" not in block:
            continue
        name = re.search(r"\.name:\s+(\S+)", block).group(1)
        field = lambda k: int(re.search(r"\." + k + r":\s+(\d+)", block).group(1))  # noqa: E731
        kernels[name] = {"hot_loop_scratch": _hot_loop_scratch(text, name),
                         "private_segment_fixed_size": field("private_segment_fixed_size"),
                         "vgpr_count": field("vgpr_count"),
                         "vgpr_spill_count": field("vgpr_spill_count"),
                         "sgpr_spill_count": field("sgpr_spill_count"),
                         "group_segment_fixed_size": field("group_segment_fixed_size")}
    return kernels


def _compile(path, sources, verbose):
    tmp = path + ".tmp"
    cmd = compile_command(tmp, sources)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if verbose or res.returncode != 0:
        msg = "\n".join(line for line in (res.stdout + res.stderr).splitlines()
                        if "packed-fp32-ops" not in line)
        if msg.strip():
            print(msg)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed building {os.path.basename(path)}:\n" + " ".join(cmd))
    os.replace(tmp, path)


def build(verbose=False):
    """Compile the library and the probe library beside it (always, even when
    they are present) and return the library's path."""
    os.makedirs(LIB_DIR, exist_ok=True)
    _compile(LIB_PATH, SOURCES, verbose)
    _compile(PROBE_PATH, PROBE_SOURCES, verbose)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
