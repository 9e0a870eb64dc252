"""Build the HIP library (gfx950) and its host-emulation twin.

    python -m paper_1406_7803_amd.build            # both libraries
    python -m paper_1406_7803_amd.build --device   # libfde.so only

libfde.so       the product: hand-written HIP kernels for gfx950 behind the
                C ABI declared in include/fde.h.
libfde_emu.so   the same sources compiled for the host with FDE_EMULATE: every
                kernel body runs serially on the CPU. Used only by the CPU test
                suite to check indexing and arithmetic without a GPU; never
                loaded by the Python binding's product path.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["plan.cpp", "pw.hip", "grid.hip", "la.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

DEVICE_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-result"]
EMU_FLAGS = ["-x", "hip", "--offload-host-only", "-DFDE_EMULATE", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Wno-unused-result"]


def _compile(src: str, obj: str, flags) -> None:
    cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def _build(name: str, flags, link_extra) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tag = "dev" if "--offload-arch" in " ".join(flags) else "emu"
    objs = [os.path.join(BUILD, f"{os.path.splitext(s)[0]}.{tag}.o") for s in SOURCES]
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], flags), zip(SOURCES, objs)))
    out = os.path.join(HERE, name)
    tmp = out + ".tmp"
    cmd = [HIPCC] + link_extra + ["-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


def build_device() -> str:
    return _build("libfde.so", DEVICE_FLAGS, [f"--offload-arch={ARCH}"])


def build_emulation() -> str:
    return _build("libfde_emu.so", EMU_FLAGS, ["-lpthread"])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--device", action="store_true", help="only the gfx950 library")
    ap.add_argument("--emu", action="store_true", help="only the host-emulation library")
    a = ap.parse_args(argv)
    if not a.emu:
        print("built", build_device())
    if not a.device:
        print("built", build_emulation())
    return 0


if __name__ == "__main__":
    sys.exit(main())
