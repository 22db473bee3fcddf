"""Real Tier 1 data on MI355X: hardware counters of every version of the two
programs in versions.hip (Section 2, Tier 1: counters plus the cycle count of
each profiled run), gathered with rocprofv3 in three counter passes.

    python -m paper_1910_07776_amd.profiling.collect OUT.npz [--runs 3]

Needs the built sugg_versions program and rocprofv3 on a GPU machine.  Each
pass runs the program once as a child process (nothing here touches the GPU
itself); dispatches are matched across passes by their order.  The cycle
count is GRBM_GUI_ACTIVE (GPU busy cycles of the dispatch).  Counters are
stored as measured (zero where an event did not occur).
"""
from __future__ import annotations

import argparse
import csv
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BINARY = os.path.join(os.path.dirname(HERE), "_lib", "sugg_versions")

# at most 8 SQ, 4 TCC and 2 GRBM counters per pass
PASSES = [
    ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
     "SQ_INSTS_BRANCH", "SQ_INSTS_SMEM"],
    ["SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_TRANS_F32",
     "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAVE_CYCLES"],
    ["TCC_HIT_sum", "TCC_MISS_sum", "GRBM_GUI_ACTIVE"],
]
CYCLES = "GRBM_GUI_ACTIVE"
PROGRAMS, INPUTS, VERSIONS = 2, 3, 64


def run_pass(counters, runs: int, workdir: str, timeout: int = 240):
    """One profiled run of the program; returns [(kernel, {counter: value})]
    in dispatch order."""
    out = os.path.join(workdir, "p")
    cmd = ["rocprofv3", "--pmc", *counters, "--output-format", "csv", "-d", out, "-o", "run", "--",
           BINARY, str(runs)]
    r = subprocess.run(cmd, cwd=workdir, capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0:
        sys.stderr.write(r.stdout[-2000:] + r.stderr[-4000:])
        raise RuntimeError(f"rocprofv3 failed ({r.returncode}) for {counters}")
    path = None
    for root, _, files in os.walk(out):
        for f in files:
            if f.endswith("counter_collection.csv"):
                path = os.path.join(root, f)
    if path is None:
        raise RuntimeError("no counter_collection.csv")
    disp = {}
    for row in csv.DictReader(open(path)):
        d = int(row["Dispatch_Id"])
        name, vals = disp.setdefault(d, (row["Kernel_Name"], {}))
        vals[row["Counter_Name"]] = vals.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    subprocess.run(["rm", "-rf", out], check=False)
    return [disp[d] for d in sorted(disp) if "versions::" in disp[d][0]]


def collect(runs: int = 3):
    names = [c for p in PASSES for c in p if c != CYCLES]
    n = PROGRAMS * INPUTS * runs * VERSIONS
    counters = np.zeros((n, len(names)))
    cycles = np.zeros(n)
    kernels = None
    with tempfile.TemporaryDirectory(dir="/tmp") as wd:
        for p in PASSES:
            rows = run_pass(p, runs, wd)
            if len(rows) != n:
                raise RuntimeError(f"expected {n} dispatches, got {len(rows)}")
            ks = [k for k, _ in rows]
            if kernels is None:
                kernels = ks
            elif ks != kernels:
                raise RuntimeError("dispatch order differs between passes")
            for c in p:
                col = np.array([v[c] for _, v in rows])
                if c == CYCLES:
                    cycles[:] = col
                else:
                    counters[:, names.index(c)] = col
            print(f"pass {p}: {len(rows)} dispatches", flush=True)
    # row order: program, input, run, version S
    prog, inp, run, ver = np.meshgrid(np.arange(PROGRAMS), np.arange(INPUTS), np.arange(runs), np.arange(VERSIONS),
                                      indexing="ij")
    return {"counters": counters, "cycles": cycles, "names": np.array(names), "kernels": np.array(kernels),
            "program": prog.ravel(), "input": inp.ravel(), "run": run.ravel(), "version": ver.ravel()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--runs", type=int, default=3)
    args = ap.parse_args()
    data = collect(args.runs)
    np.savez_compressed(args.out, **data)
    print(f"wrote {args.out}: {data['counters'].shape[0]} rows x {data['counters'].shape[1]} counters", flush=True)


if __name__ == "__main__":
    main()
