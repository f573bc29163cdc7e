"""Build step of the HIP library: compiles csrc/*.hip for gfx950 into
libvanka_mg.so next to this file (run by ``__graft_entry__.build()`` or
``python -m paper_2203_11154_amd._build``)."""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["vmg_kernels.hip", "vmg_stream.hip", "vmg_transform.hip", "vmg_aux.hip", "vmg_tail.hip", "vmg_lfa.hip",
           "vmg_runtime.hip"]
LIB = os.path.join(HERE, "libvanka_mg.so")
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    """Compile every source and link the shared library; raises on failure."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-result",
             # keep the compiler from emitting packed FP32 ALU instructions
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = [os.path.join(objdir, src.replace(".hip", ".o")) for src in SOURCES]

    def compile_one(src, obj):
        cmd = [hipcc()] + flags + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return src, subprocess.run(cmd, capture_output=True, text=True)

    # the sources compile independently: in parallel, a few at a time
    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as pool:
        for src, res in pool.map(compile_one, SOURCES, objs):
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
