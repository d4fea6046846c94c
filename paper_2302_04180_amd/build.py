"""Build librpk.so for gfx950 with hipcc, in-tree next to this file.

The templated kernels are instantiated once per FPE length (0 = plain FP64,
1, 2, 4, 8) in separate translation units compiled in parallel, then linked
with the host code into one shared library.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librpk.so")
# kernel instantiations: 0 = plain FP64, 1/2/3/4/8 = exact with that FPE length,
# 9 = lightweight FPE-8 dot products
FPE_LENGTHS = (0, 1, 2, 3, 4, 8, 9)

# -ffp-contract=off: no a*b+c contraction anywhere (every fma is explicit);
# packed FP32 instructions disabled; no fast-math.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-ffp-contract=off", "-fno-fast-math",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-result", "-Wno-pass-failed",
               "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose=False, jobs=None):
    with tempfile.TemporaryDirectory(prefix="rpk_build_") as tmp:
        units = [(["-DRPK_N=%d" % n], os.path.join(CSRC, "kern_inst.hip"), os.path.join(tmp, "kern_%d.o" % n))
                 for n in FPE_LENGTHS]
        for host in ("rpk", "batch", "server"):
            units.append(([], os.path.join(CSRC, host + ".hip"), os.path.join(tmp, host + ".o")))
        cmds = [["hipcc", *HIPCC_FLAGS, *extra, "-c", src, "-o", obj] for extra, src, obj in units]
        jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 2)))
        running = []
        errors = []
        pending = list(cmds)
        while pending or running:
            while pending and len(running) < jobs:
                c = pending.pop(0)
                if verbose:
                    print(" ".join(c), flush=True)
                running.append((c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            c, p = running.pop(0)
            out, _ = p.communicate()
            if p.returncode != 0:
                errors.append((c, out.decode(errors="replace")))
        if errors:
            for c, out in errors:
                sys.stderr.write(" ".join(c) + "\n" + out + "\n")
            raise RuntimeError("hipcc failed")
        tmp_so = OUT + ".tmp%d" % os.getpid()
        link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_so] + [u[2] for u in units]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp_so, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
