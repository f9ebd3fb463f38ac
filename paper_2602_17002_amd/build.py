"""Compile the HIP library ``libtlfea.so`` for gfx950, in-tree."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtlfea.so")
KERNELS = os.path.join(CSRC, "tlfea_kernels.hip")
VECTOR = os.path.join(CSRC, "tlfea_vec.hip")
JOINTS = os.path.join(CSRC, "tlfea_joints.hip")
HOST = os.path.join(CSRC, "tlfea_host.cpp")
# (element type, operation, adjoint with parameter gradients, variant) units
# of tlfea_kernels.hip; the adjoint is compiled once without and once with
# the parameter gradients, the forward and the tangent once plain and once
# as their step variant (step residual, Newton operator)
UNITS = [(e, o, g, md) for e in (0, 1, 2) for o in (0, 1, 2) for g in ((0, 1) if o == 1 else (0,))
         for md in ((0, 1) if o != 1 else (0,))]
# extra compiler flags per unit (element, operation, gradients): the adjoint
# holds two sets of nodal accumulators, and the scheduler that minimises
# register pressure keeps it (nearly) free of spills at two waves per SIMD.
# The T10 adjoint with the parameter gradients spills either way, and LLVM's
# default schedule runs it 7-13 % faster; the H8 one keeps the other.
_MAXOCC = ["-mllvm", "-amdgpu-sched-strategy=iterative-maxocc"]
UNIT_FLAGS = {(0, 1, 0, 0): _MAXOCC, (1, 1, 0, 0): _MAXOCC, (1, 1, 1, 0): _MAXOCC}


def hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, resource_usage=False):
    tmp = LIB + ".tmp"
    objs = []
    procs = []
    common = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
              # keep FP32 packed math off (only FP64 is used, this is a guard)
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
              "-I", INCLUDE, "-I", CSRC]
    if resource_usage:
        common += ["-Rpass-analysis=kernel-resource-usage"]
    jobs_list = [(HOST, [], os.path.join(CSRC, "tlfea_host.o")),
                 (VECTOR, ["-x", "hip"], os.path.join(CSRC, "tlfea_vec.o")),
                 (JOINTS, ["-x", "hip"], os.path.join(CSRC, "tlfea_joints.o"))]
    for e, o, g, md in UNITS:
        jobs_list.append((KERNELS, ["-x", "hip", f"-DTLFEA_ELEM={e}", f"-DTLFEA_OP={o}", f"-DTLFEA_VJP_GT={g}",
                                    f"-DTLFEA_MODE={md}"] + UNIT_FLAGS.get((e, o, g, md), []),
                          os.path.join(CSRC, f"tlfea_kernels_e{e}_o{o}_g{g}_m{md}.o")))
    for src, extra, obj in jobs_list:
        cmd = common + extra + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    logs = []
    failed = False
    for p in procs:
        out, _ = p.communicate()
        logs.append(out)
        failed |= p.returncode != 0
    if verbose or failed or resource_usage:
        for out in logs:
            if out:
                print(out, file=sys.stderr if failed else sys.stdout)
    if failed:
        raise RuntimeError("hipcc failed")
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, resource_usage="-r" in sys.argv))
