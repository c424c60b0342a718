"""Build tests/native/_build/abi_smoke_sanitized: the library's sources and the
C-ABI driver abi_smoke.cpp in one executable, with the host code under the
address and undefined-behaviour sanitizers (device code is compiled as in the
library build).  Run the result on a GPU host with
ASAN_OPTIONS=verify_asan_link_order=0 (another library may be preloaded) and
LSAN_OPTIONS=suppressions=tests/native/lsan.supp (allocations the ROCm runtime
keeps until exit).

    python tests/native/build_sanitized.py
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_1207_2192_amd.build import CSRC, HIPCC_FLAGS, SOURCES  # noqa: E402

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def main() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(HERE, "abi_smoke.cpp")]
    jobs = []
    for src in srcs:
        obj = os.path.join(out_dir, os.path.basename(src).rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        jobs.append((obj, [hipcc, *HIPCC_FLAGS, *SAN, *lang, "-c", "-o", obj, src]))

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        return r.returncode, "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)

    with ThreadPoolExecutor(min(len(jobs), os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda j: run(j[1]), jobs))
    for (obj, cmd), (rc, msg) in zip(jobs, results):
        if rc:
            raise RuntimeError(f"compile failed: {cmd[-1]}\n{msg}")
    exe = os.path.join(out_dir, "abi_smoke_sanitized")
    rc, msg = run([hipcc, "--offload-arch=gfx950", *SAN, "-o", exe, *[o for o, _ in jobs]])
    if rc:
        raise RuntimeError(f"link failed\n{msg}")
    return exe


if __name__ == "__main__":
    print(main())
