"""Algorithmic FP64 operation count of one RK2 step, from an op-counting build of the oracle.

TEST/MEASUREMENT INFRASTRUCTURE, like the rest of oracle/: it builds a separate counting copy of
grmhd_oracle.c and never touches the HIP library.

The oracle source is compiled to LLVM IR (clang -O1, no FP contraction, no fast-math, OpenMP off
so every pragma runs serially), and before every double-precision arithmetic instruction
(fadd/fsub, fmul, fdiv) and every call of sqrt, pow and the other libm functions a counter
increment is inserted; the IR is then compiled to a shared library with the oracle's exports and
driven through oracle.py.  Because -O1 neither vectorises nor fuses, each counted instruction is one
operation the oracle's source performs.  The count of one step is the count of a two-step run
minus that of a one-step run on the same state, which removes the set-up (metric tables, complex-
step derivatives).  The oracle evaluates every 4x4 contraction in full, zeros included, so its
count is an upper estimate of the method's own arithmetic.

Usage:  python -m oracle.count_flops [--out profiles/oracle_flop_count.json]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LLVM = os.environ.get("LLVM_BIN", "/opt/rocm/llvm/bin")

# counter slots
KINDS = ("add", "mul", "div", "sqrt", "pow", "other_libm")
_ARITH = {"fadd": "add", "fsub": "add", "fmul": "mul", "fdiv": "div"}
_CALLS = {"sqrt": "sqrt", "llvm.sqrt.f64": "sqrt", "pow": "pow", "llvm.pow.f64": "pow"}
_LIBM = ("exp", "log", "sin", "cos", "tan", "atan", "atan2", "cbrt", "llvm.exp.f64", "llvm.log.f64",
         "llvm.sin.f64", "llvm.cos.f64")


def instrument(ir: str) -> str:
    out = []
    n = 0
    arith = re.compile(r"^\s+%[\w.]+ = (fadd|fsub|fmul|fdiv)( [a-z ]*)? double ")
    call = re.compile(r"call [\w ]*double @([\w.]+)\(")
    for line in ir.splitlines():
        kind = None
        m = arith.match(line)
        if m:
            kind = _ARITH[m.group(1)]
        else:
            c = call.search(line)
            if c and not line.lstrip().startswith("declare"):
                name = c.group(1)
                if name in _CALLS:
                    kind = _CALLS[name]
                elif name in _LIBM:
                    kind = "other_libm"
        if kind is not None:
            slot = KINDS.index(kind)
            p = f"@__opcount_{slot}"
            out.append(f"  %__oc.{n} = load i64, ptr {p}, align 8")
            out.append(f"  %__oc.{n + 1} = add i64 %__oc.{n}, 1")
            out.append(f"  store i64 %__oc.{n + 1}, ptr {p}, align 8")
            n += 2
        out.append(line)
    for k in range(len(KINDS)):
        out.append(f"@__opcount_{k} = global i64 0, align 8")
    # accessor the driver reads the counters through
    out.append("define dso_local void @orc_opcounts(ptr %out) {")
    for k in range(len(KINDS)):
        out.append(f"  %v{k} = load i64, ptr @__opcount_{k}, align 8")
        out.append(f"  %p{k} = getelementptr inbounds i64, ptr %out, i64 {k}")
        out.append(f"  store i64 %v{k}, ptr %p{k}, align 8")
        out.append(f"  store i64 0, ptr @__opcount_{k}, align 8")
    out.append("  ret void")
    out.append("}")
    return "\n".join(out) + "\n"


def build_counting_library(tmp: str) -> str:
    src = os.path.join(HERE, "grmhd_oracle.c")
    ll = os.path.join(tmp, "oracle.ll")
    subprocess.check_call([os.path.join(LLVM, "clang"), "-O1", "-ffp-contract=off", "-fno-fast-math",
                           "-fno-vectorize", "-fno-slp-vectorize", "-fPIC", "-S", "-emit-llvm", "-o", ll, src])
    with open(ll) as fh:
        ir = fh.read()
    ll2 = os.path.join(tmp, "oracle_count.ll")
    with open(ll2, "w") as fh:
        fh.write(instrument(ir))
    lib = os.path.join(tmp, "liboracle_count.so")
    subprocess.check_call([os.path.join(LLVM, "clang"), "-O1", "-fPIC", "-shared", "-o", lib, ll2, "-lm"])
    return lib


def count_step(lib_path: str, cfg_obj, P) -> dict:
    import ctypes
    sys.path.insert(0, ROOT)
    from oracle import oracle as orc
    buf = (ctypes.c_int64 * len(KINDS))()
    with orc.using_library(lib_path):
        L = orc.lib()
        L.orc_opcounts.argtypes = [ctypes.c_void_p]
        cfg = orc.make_cfg(cfg_obj)
        counts = []
        for nsteps in (1, 2):
            L.orc_opcounts(buf)                      # reset
            orc.step(cfg, P, nsteps)
            L.orc_opcounts(buf)
            counts.append(np.array(list(buf), dtype=np.int64))
    per_step = counts[1] - counts[0]
    zones = cfg_obj.n1 * cfg_obj.n2 * cfg_obj.n3
    d = {k: float(per_step[i]) / zones for i, k in enumerate(KINDS)}
    d["total"] = float(per_step.sum()) / zones
    return d


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "oracle_flop_count.json"))
    args = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    sys.path.insert(0, ROOT)
    from paper_2205_02484_amd.torus_init import TorusConfig, make_torus
    from paper_2205_02484_amd.workloads import torus_2d_64
    cases = {
        "torus2d_64x64": torus_2d_64(),
        # the 256^3 benchmark torus's physics and radial extent on a 64^3 grid
        "torus3d_256x256x256_physics_at_64cubed": TorusConfig(
            n1=64, n2=64, n3=64, spin=0.9375, h=0.3, r_out=1000.0, gam=5.0 / 3.0, r_in=20.0, r_max=41.0,
            beta=100.0, beta_mode="max_ratio", delta=0.04, seed=3, cfl=0.45),
    }
    res = {"method": "LLVM-IR op-counting build of oracle/grmhd_oracle.c (clang -O1, no contraction, no "
                     "vectorisation, serial); per zone-update = (2-step count - 1-step count) / zones; "
                     "add = fadd + fsub, mul = fmul, div = fdiv, each 1 flop; sqrt, pow and other libm "
                     "calls counted as 1 each in 'total'",
           "command": "python -m oracle.count_flops", "per_zone_update": {}}
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_counting_library(tmp)
        for name, c in cases.items():
            res["per_zone_update"][name] = count_step(lib, c, make_torus(c))
            print(name, json.dumps(res["per_zone_update"][name]), flush=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(args.out)


if __name__ == "__main__":
    main()
