"""Build the okpz HIP library for gfx950 in-tree (``libokpz.so``).

The device compiles also report each kernel's register, scratch and LDS use
(the compiler's kernel-resource-usage remarks); they are kept in
``_build/kernel_resources.json`` for the resource checks of the tests."""
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["api.hip", "sweep.hip", "width.hip", "psd.hip", "batch.hip"]
HOST_SOURCES = ["host_logic.cpp"]  # plain C++, no device code
LIB = os.path.join(HERE, "libokpz.so")
RESOURCES = os.path.join(HERE, "_build", "kernel_resources.json")
_REMARK = re.compile(r"remark:\s+(Function Name|TotalSGPRs|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s+(\S+)")
_KEYS = {"TotalSGPRs": "sgpr", "VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
         "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "lds"}


def parse_resources(text):
    """Kernel name -> resource counts, from kernel-resource-usage remarks."""
    out, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val)
    return out


def hip_flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def build(verbose=False):
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmds.append([hipcc, *hip_flags(), "-Rpass-analysis=kernel-resource-usage", "-c",
                     os.path.join(HERE, "csrc", src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src.replace(".cpp", ".o"))
        cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-c",
                     os.path.join(HERE, "csrc", src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        # pass the compiler's output on, without the resource remarks
        rest = "\n".join(l for l in r.stderr.splitlines()
                         if "kernel-resource-usage" not in l and not re.match(r"\s*\d*\s*\|", l))
        if rest.strip():
            print(rest, file=sys.stderr, flush=True)
        if r.stdout.strip():
            print(r.stdout, flush=True)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        return parse_resources(r.stderr)

    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        found = list(ex.map(run, cmds))
    resources = {}
    for f in found:
        resources.update(f)
    with open(RESOURCES, "w") as fh:
        json.dump(resources, fh, indent=0, sort_keys=True)
    tmp = LIB + ".tmp"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
