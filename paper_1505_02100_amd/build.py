"""Build libkdeplugin.so (HIP for gfx950) in-tree.

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 VALU forms are
disabled for every HIP translation unit (the host pass warns that it does not
know the feature; that warning is harmless).

The library is linked against the HIP runtime that PyTorch ships
(torch/lib/libamdhip64.so), so it only uses entry points that runtime
exports.  Its dependency is recorded by soname (libamdhip64.so.7); when torch
is imported first, that soname resolves to torch's already loaded runtime, so
torch tensors' device pointers and streams and the library's launches share
one HIP runtime instance (the Python binding imports torch before loading the
library and checks that only one runtime is mapped).  A C program without
torch resolves the soname to the system ROCm runtime instead.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkdeplugin.so")

SOURCES = ["kde_device.hip", "kde_eval.hip", "kde_host.cpp", "kde_tune.cpp", "kde_server.cpp",
           "kde_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-fvisibility=hidden",
]


def torch_hip_libdir() -> str:
    """Directory of the HIP runtime bundled with the installed PyTorch."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("PyTorch is required: its HIP runtime is the one the library links")
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}")
    return d


# Per-kernel register, scratch and occupancy figures of the device code, as
# the compiler reports them, written next to the library by build() (tests
# check the ones the kernels' speed depends on).
RESOURCES = os.path.join(HERE, "kernel_resources.txt")
RESOURCE_SOURCES = ("kde_device.hip", "kde_eval.hip")


def _resource_lines(stderr: str):
    """'kernel vgprs scratch occupancy' for every kernel in hipcc's
    kernel-resource-usage remarks."""
    out, cur = [], {}
    for line in stderr.splitlines():
        if "remark:" not in line:
            continue
        text = line.split("remark:", 1)[1].strip()
        for key, field in (("Function Name:", "name"), ("VGPRs:", "vgprs"),
                           ("ScratchSize [bytes/lane]:", "scratch"), ("Occupancy [waves/SIMD]:", "occ")):
            if text.startswith(key):
                cur[field] = text[len(key):].split("[")[0].strip()
        if {"name", "vgprs", "scratch", "occ"} <= cur.keys():
            out.append(f"{cur['name']} {cur['vgprs']} {cur['scratch']} {cur['occ']}")
            cur = {}
    return out


def build(verbose: bool = False) -> str:
    objs = []
    resources = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if src in RESOURCE_SOURCES:
            cmd.append("-Rpass-analysis=kernel-resource-usage")
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if src in RESOURCE_SOURCES:
            resources += _resource_lines(r.stderr)
        objs.append(obj)
    with open(RESOURCES, "w") as f:
        f.write("# kernel vgprs scratch_bytes_per_lane waves_per_simd (gfx950, from hipcc)\n")
        f.write("\n".join(resources) + "\n")
    tmp = LIB + ".tmp"
    tlib = torch_hip_libdir()
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, "-L" + tlib, "-l:libamdhip64.so",
           "-Wl,--no-undefined", "-lstdc++", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


SAN_DIR = os.path.join(ROOT, "tests", "sanitize")
SAN_EXE = os.path.join(SAN_DIR, "kde_san_driver")
# the translation units whose host code the sanitizer build instruments; the
# device-heavy units are linked from the ordinary build unchanged
SAN_HOST_SOURCES = ["kde_host.cpp", "kde_tune.cpp", "kde_server.cpp", "kde_noalloc.hip"]
SAN_HOST_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all"]
CLANG = os.environ.get("KDE_CLANGXX", "/opt/rocm/llvm/bin/clang++")


def build_sanitized(verbose: bool = False) -> str:
    """tests/sanitize/kde_san_driver: the C ABI driver linked with the host
    runtime built under AddressSanitizer and UndefinedBehaviorSanitizer (host
    code only; kde_device.o and kde_eval.o come from build())."""
    objdir = os.path.join(SAN_DIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    base = [f for f in FLAGS if f not in ("-O3",)]
    for src, path in [(s_, os.path.join(CSRC, s_)) for s_ in SAN_HOST_SOURCES] + \
                     [("kde_san_driver.cpp", os.path.join(SAN_DIR, "kde_san_driver.cpp"))]:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *base, *SAN_HOST_FLAGS, "-I", INCLUDE, "-I", CSRC, "-x", "hip", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src} (sanitizer build):\n{r.stdout}\n{r.stderr}")
        objs.append(obj)
    for src in ("kde_device.hip", "kde_eval.hip"):
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj):
            raise RuntimeError(f"{obj} missing: build() first")
        objs.append(obj)
    tmp = SAN_EXE + ".tmp"
    cmd = [CLANG, "-fsanitize=undefined,address", "-o", tmp, *objs, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-lstdc++", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer driver link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_EXE)
    return SAN_EXE


PROBE_SRC = os.path.join(HERE, "probes", "issue_rate.hip")
PROBE = os.path.join(HERE, "probes", "issue_rate")


def build_probe(verbose: bool = False) -> str:
    """The issue-rate microbenchmark (a standalone HIP program, run by
    bench.py --workload issue-rate)."""
    tmp = PROBE + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PROBE_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
    print(build_sanitized(verbose=True))
