"""Build the vfx HIP library for gfx950 (hipcc, in-tree): every source is
compiled to its own object in parallel, then the objects are linked."""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["api.cpp", "tables.cpp", "stencil.cpp", "plan.cpp", "kernels.hip", "near.hip", "mixed.hip", "mlp.hip", "factor.hip"]
OUT = os.path.join(HERE, "lib", "libvfx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fopenmp",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _filter(text):
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose=False):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(HERE, "csrc", s))]
    with tempfile.TemporaryDirectory(prefix="vfx_build_") as tmpdir:
        objs = [os.path.join(tmpdir, s + ".o") for s in srcs]

        def compile_one(i):
            cmd = [HIPCC] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-c",
                                     os.path.join(HERE, "csrc", srcs[i]), "-o", objs[i]]
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(max_workers=min(len(srcs), max(1, os.cpu_count() or 1))) as ex:
            results = list(ex.map(compile_one, range(len(srcs))))
        msgs = "\n".join(_filter(r.stdout + r.stderr) for r in results)
        if any(r.returncode != 0 for r in results):
            raise RuntimeError("hipcc failed:\n" + msgs)
        tmp = OUT + ".tmp"
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fopenmp", "-o", tmp] + objs,
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + _filter(r.stdout + r.stderr))
    if verbose and msgs.strip():
        print(msgs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
