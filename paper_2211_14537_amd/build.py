"""Build the vfx HIP library for gfx950 (hipcc, in-tree): every source is
compiled to its own object in parallel, then the objects are linked.

``build()`` compiles every source each time it is called and keeps the
objects in ``_build/`` (each with the digest of its inputs).
``build_host_sanitized()`` builds a second copy of the library whose host
C++ (the C-ABI, plan construction, tables, stencil) is compiled with
AddressSanitizer and UndefinedBehaviorSanitizer by clang as plain C++, and
linked with the device objects of ``build()`` (compiled again only if their
inputs changed).  It is loaded by the CPU tests through ``VFX_LIBRARY`` with
the sanitizer runtime preloaded."""
import hashlib
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["api.cpp", "tables.cpp", "stencil.cpp", "plan.cpp", "kernels.hip", "near.hip", "mixed.hip", "mixed8.hip",
           "ext_batch.hip", "mlp.hip", "factor.hip"]
HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]
OUT = os.path.join(HERE, "lib", "libvfx.so")
BUILD_DIR = os.path.join(HERE, "_build")
SANITIZED_OUT = os.path.join(BUILD_DIR, "libvfx_sanitized.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = os.environ.get("VFX_CLANGXX", "/opt/rocm/llvm/bin/clang++")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fopenmp",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SAN_FLAGS = ["-x", "c++", "-std=c++17", "-O1", "-g", "-fPIC", "-fopenmp", "-D__HIP_PLATFORM_AMD__",
             "-I/opt/rocm/include", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]


def _filter(text):
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def _digest(src, flags):
    h = hashlib.sha256()
    for path in (os.path.join(HERE, "csrc", src), os.path.join(HERE, "csrc", "vfx_internal.h"),
                 os.path.join(ROOT, "include", "vfx.h")):
        with open(path, "rb") as f:
            h.update(f.read())
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def _compile(jobs):
    """jobs: (command, object path, digest); returns the combined messages."""
    def one(job):
        cmd, obj, dig = job
        r = subprocess.run(cmd + ["-o", obj + ".tmp"], capture_output=True, text=True)
        if r.returncode == 0:
            os.replace(obj + ".tmp", obj)
            with open(obj + ".key", "w") as f:
                f.write(dig)
        return r

    with ThreadPoolExecutor(max_workers=min(max(len(jobs), 1), max(1, os.cpu_count() or 1))) as ex:
        results = list(ex.map(one, jobs))
    msgs = "\n".join(_filter(r.stdout + r.stderr) for r in results)
    if any(r.returncode != 0 for r in results):
        raise RuntimeError("compile failed:\n" + msgs)
    return msgs


def _object(src):
    return os.path.join(BUILD_DIR, src + ".o")


def _hip_job(src):
    cmd = [HIPCC] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "csrc", src)]
    return cmd, _object(src), _digest(src, FLAGS)


def _fresh(obj, dig):
    try:
        with open(obj + ".key") as f:
            return os.path.exists(obj) and f.read() == dig
    except OSError:
        return False


def _link(out, objs, extra=()):
    tmp = out + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fopenmp", *extra, "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + _filter(r.stdout + r.stderr))
    os.replace(tmp, out)


def build(verbose=False):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(HERE, "csrc", s))]
    msgs = _compile([_hip_job(s) for s in srcs])
    _link(OUT, [_object(s) for s in srcs])
    if verbose and msgs.strip():
        print(msgs)
    return OUT


def build_host_sanitized(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    dev = [s for s in SOURCES if s not in HOST_SOURCES]
    jobs = [j for j in (_hip_job(s) for s in dev) if not _fresh(j[1], j[2])]
    host_objs = []
    for s in HOST_SOURCES:
        obj = os.path.join(BUILD_DIR, s + ".san.o")
        cmd = [CLANGXX] + SAN_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "csrc", s)]
        dig = _digest(s, SAN_FLAGS)
        if not _fresh(obj, dig):
            jobs.append((cmd, obj, dig))
        host_objs.append(obj)
    msgs = _compile(jobs) if jobs else ""
    # the sanitizer runtimes are linked for the host side only
    _link(SANITIZED_OUT, host_objs + [_object(s) for s in dev],
          extra=("-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"))
    if verbose and msgs.strip():
        print(msgs)
    return SANITIZED_OUT


def sanitizer_runtime():
    """Path of clang's AddressSanitizer runtime (to preload into python)."""
    r = subprocess.run([CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang's AddressSanitizer runtime was not found")
    return path


if __name__ == "__main__":
    print(build(verbose=True))
