"""Build librpcg.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Flags that matter for the results:
  -ffp-contract=off   no a*b+c is fused unless fma is written (TwoSum/TwoProd
                      and the fma-only updates depend on it)
  no fast-math        IEEE division, denormals kept in binary64
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keep the compiler from emitting packed FP32 instructions
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librpcg.so")
# (source, object suffix, extra flags): the templated solver kernels are built
# once per value type so the compiles run in parallel
_TYPED = ["pcg_setup.hip", "pcg_spmv_dot.hip", "pcg_update.hip"]
SOURCES = ([("exdot.hip", "", []), ("exdot_noalloc.hip", "", []), ("sell.hip", "", []), ("ir.hip", "", []), ("batch_setup.hip", "", []),
            ("batch_iter.hip", "", []), ("pcg_factored_setup.hip", "", []), ("pcg_factored_iter.hip", "", []), ("api.cpp", "", []),
            ("batch_api.cpp", "", []), ("lp_conv.hip", "", []),
            ("lp_factor.hip", "", []), ("lp_loss.hip", "", []), ("lp_api.cpp", "", [])] +
           [(f, "." + t, [f"-DRPCG_VALUE_TYPE={t}"]) for f in _TYPED for t in ("double", "float")])
ARCH = os.environ.get("RPCG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    # binary32 division correctly rounded and binary32 subnormals kept, as
    # IEEE 754 binary32 arithmetic requires (the binary32 solver relies on it)
    "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src, suffix, extra in SOURCES:
        obj = os.path.join(objdir, src + suffix + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [hipcc(), *lang, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:  # noqa: B007
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"--- {s}\n{t}" for s, t in failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
