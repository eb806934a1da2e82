"""Build libparrep.so (HIP for gfx950) in-tree with hipcc.

Flags: -ffp-contract=off keeps every product and sum separately rounded (the
bit-level conventions the integer state sequence depends on);
-munsafe-fp-atomics lets FP64 atomic adds use the hardware instructions; the
packed-FP32 target feature is switched off.
"""
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libparrep.so")
SOURCES = ["parrep_kernels.hip", "parrep_api.hip", "parrep_batch.hip", "parrep_server.hip"]
# The instance kernel is compiled once per (species count, waves per workgroup).
INSTANCE_VARIANTS = [(ns, w) for ns in (1, 2, 4) for w in (1, 4, 16)]
ARCH = os.environ.get("PARREP_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-ffp-contract=off", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found; install ROCm to build libparrep")
    return h


def _includes(path, seen=None):
    """The quoted #include files of path, recursively (the object's header deps)."""
    seen = set() if seen is None else seen
    with open(path) as f:
        for line in f:
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                dep = os.path.normpath(os.path.join(os.path.dirname(path), m.group(1)))
                if dep not in seen and os.path.exists(dep):
                    seen.add(dep)
                    _includes(dep, seen)
    return seen


def build(force: bool = True, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit and link libparrep.so.  force=False
    returns at once when the library is newer than every source;
    incremental=True recompiles only the objects older than their source or
    one of the headers it includes."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    jobs = [(s, os.path.basename(s) + ".o", []) for s in srcs]
    inst = os.path.join(CSRC, "parrep_instance.hip")
    for ns, w in INSTANCE_VARIANTS:
        jobs.append((inst, "parrep_instance_ns%d_w%d.o" % (ns, w),
                     ["-DPARREP_NS=%d" % ns, "-DPARREP_WAVES=%d" % w]))
    wide = os.path.join(CSRC, "parrep_wide.hip")
    for ns in (1, 2, 4):
        jobs.append((wide, "parrep_wide_ns%d.o" % ns, ["-DPARREP_NS=%d" % ns]))
    deps = srcs + [inst, os.path.join(CSRC, "parrep_internal.h"), os.path.join(CSRC, "parrep_host.h"),
                   os.path.join(CSRC, "parrep_neglog.h"), os.path.join(CSRC, "parrep_fx.h"),
                   os.path.join(CSRC, "parrep_device.h"), os.path.join(CSRC, "parrep_wide.h"),
                   wide, os.path.join(ROOT, "include", "parrep.h")]
    if not force and os.path.exists(LIB):
        if os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
            return LIB
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()

    def compile_one(job):
        src, oname, defs = job
        obj = os.path.join(BUILD, oname)
        if incremental and os.path.exists(obj):
            newest = max(os.path.getmtime(d) for d in [src, *_includes(src)])
            if os.path.getmtime(obj) >= newest:
                return obj
        cmd = [cc, *FLAGS, *defs, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-20000:]))
        return obj

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, jobs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-20000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
