"""Builds the host sanitizer drivers (test infrastructure).

* ``oracle_san``: the FP64 oracle and ``oracle_main.c``, built by gcc with
  AddressSanitizer (leak checks included) and UndefinedBehaviorSanitizer.
* ``capi_san``: every source of libpulsar and ``capi_main.cpp``, built by
  hipcc with both sanitizers on the host side only (each sanitizer flag goes
  to the host compilation through ``-Xarch_host``; the gfx950 code is built
  as usual and never runs here).

Results go to ``tests/sanitize/_build`` and are rebuilt only when a source or
a flag changes.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
CSRC = os.path.join(ROOT, "paper_2004_07484_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ORACLE_SRC = os.path.join(ROOT, "oracle", "pulsar_oracle.c")

LIB_SOURCES = ["capi.cpp", "project.hip", "binning.hip", "raster_fwd.hip", "raster_bwd.hip",
               "noalloc.hip"]
LIB_HEADERS = ["pulsar_internal.h", "device_common.h", "hit_geometry.h"]

SAN = ["address", "undefined"]
ORACLE_FLAGS = ["-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
                "-ffp-contract=off", "-fno-sanitize-recover=all"] + \
               ["-fsanitize=" + s for s in SAN]
HOST_SAN = [a for s in SAN for a in ("-Xarch_host", "-fsanitize=" + s)]
HIP_FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fno-sanitize-recover=all"] + HOST_SAN


def _digest(paths, flags) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def _fresh(exe: str, digest: str) -> bool:
    stamp = exe + ".sha256"
    return (os.path.exists(exe) and os.path.exists(stamp)
            and open(stamp).read().strip() == digest)


def _stamp(exe: str, digest: str) -> None:
    with open(exe + ".sha256", "w") as f:
        f.write(digest + "\n")


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_oracle() -> str:
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_san")
    srcs = [os.path.join(HERE, "oracle_main.c"), ORACLE_SRC]
    digest = _digest(srcs, ORACLE_FLAGS)
    if not _fresh(exe, digest):
        subprocess.run(["gcc", *ORACLE_FLAGS, *srcs, "-o", exe, "-lm"], check=True)
        _stamp(exe, digest)
    return exe


def build_capi() -> str:
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "capi_san")
    srcs = [os.path.join(CSRC, s) for s in LIB_SOURCES]
    driver = os.path.join(HERE, "capi_main.cpp")
    headers = [os.path.join(INCLUDE, "pulsar.h")] + \
              [os.path.join(CSRC, h) for h in LIB_HEADERS if os.path.exists(os.path.join(CSRC, h))]
    digest = _digest(srcs + [driver] + headers, HIP_FLAGS)
    if _fresh(exe, digest):
        return exe
    hipcc = _hipcc()
    objs, procs = [], []
    for src in srcs + [driver]:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
    errors = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            errors.append(f"{os.path.basename(src)}:\n{out.decode(errors='replace')[-4000:]}")
    if errors:
        raise RuntimeError("sanitizer build failed\n" + "\n".join(errors))
    subprocess.run([hipcc, "--offload-arch=gfx950", *HOST_SAN, *objs, "-o", exe], check=True)
    for o in objs:
        os.remove(o)
    _stamp(exe, digest)
    return exe


if __name__ == "__main__":
    print(build_oracle())
    print(build_capi())
    sys.exit(0)
