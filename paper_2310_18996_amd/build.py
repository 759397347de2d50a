"""Build liblyamock.so (HIP, gfx950) in-tree with hipcc: every source is
compiled to its own object in parallel (under _build/), then linked."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "liblyamock.so")
SOURCES = ["lya_abi.hip", "lya_timing.hip", "k_tables.hip", "k_fft.hip", "k_skewers.hip", "k_p1d.hip",
           "lya_tune.hip", "lya_mlp.hip", "lya_autotune.hip", "k_tune_eval.hip", "lya_tune_ps.hip",
           "lya_qso.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src, verbose):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    return obj, r.returncode, msg


def build(verbose=False, jobs=None):
    """Compile every HIP source and link liblyamock.so (always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    failed = False
    for (obj, rc, msg), src in zip(res, SOURCES):
        if msg.strip():
            print(msg, file=sys.stderr)
        if rc != 0:
            print("hipcc failed on %s" % src, file=sys.stderr)
            failed = True
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc")
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [r[0] for r in res]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    sys.exit(0)
