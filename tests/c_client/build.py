"""Build tests/c_client/pnce_c_client, a plain C caller of libpnce.so (test
infrastructure; linked against the in-tree library, found at run time next
to it through an rpath)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2206_05506_amd")
OUT = os.path.join(HERE, "pnce_c_client")


def build(verbose: bool = False) -> str:
    # compiled as HIP host code (no kernels in it) so hipcc supplies the
    # runtime headers and library; the rpath finds the in-tree libpnce.so
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-x", "hip", "-O2", "-Wall",
           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "pnce_c_client.c"),
           "-L" + PKG, "-lpnce", "-Wl,-rpath,$ORIGIN/../../paper_2206_05506_amd",
           "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
