"""Build librwtrsv.so (all HIP sources, gfx950) in place next to this file."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librwtrsv.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed-FP32 instructions: they are emitted by the compiler from
         # plain float code and have given wrong results on these parts
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source (at most `jobs` compilers at once) and link the
    shared library, with the hash of the sources compiled in."""
    try:
        from ._srchash import source_hash
    except ImportError:            # run as a script
        sys.path.insert(0, HERE)
        from _srchash import source_hash
    os.makedirs(BUILD, exist_ok=True)
    digest = source_hash(FLAGS)
    defs = [f'-DRWT_SOURCE_HASH="{digest}"']
    running = []
    done = []
    objs = []

    def reap(block: bool) -> None:
        while running:
            for item in list(running):
                if item[1].poll() is not None:
                    running.remove(item)
                    done.append(item)
            if not block or len(running) < jobs:
                return
            running[0][1].wait()

    for src in sources():
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, *defs, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        reap(block=True)   # wait until fewer than `jobs` compilers run
        log = tempfile.TemporaryFile()
        running.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
    for item in running:
        item[1].wait()
    done.extend(running)
    failed = []
    for src, p, log in done:
        log.seek(0)
        text = log.read().decode(errors="replace")
        log.close()
        lines = [l for l in text.splitlines()
                 if "packed-fp32-ops" not in l and "warning generated" not in l]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n\n".join(f"{s}:\n{t}" for s, t in failed)
        raise RuntimeError("HIP compilation failed:\n" + msg)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
