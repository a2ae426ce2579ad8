"""Full-size comparison of whole GPU steps with the FP64 oracle.

    python tests/fullsize_oracle_check.py --case four_field_ocean_lie [--steps 2] [--workers 16] [--json PATH]

Cases (every one FP64, in the launch shape the autotuner picks, as the
benchmark runs it):

  four_field_ocean_lie   199,712 triangles x 30 sigma layers, 4 fields, SSP-RK3 + vertical solve
  four_field_ocean_imex  the same mesh and fields, the split-IMEX step
  zlevel_ensemble_lie    16 members, 5-60 z-level layers per column (36.6 M prisms), 4 fields

The GPU steps run in a child process, which saves the gathered state and
exits; this process never initialises the GPU, so it can fork the oracle's
workers (``oracle.parallel``), which evaluate the same steps from the same
seeded inputs.  The check is the parity metric of the GPU tests: per field,
max |x_gpu - x_oracle| / max |x_oracle| <= 1e-12.  Not collected by pytest
(minutes of host CPU): run by hand on a GPU machine.
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

CASES = {
    "four_field_ocean_lie": ("four_field_ocean", "lie"),
    "four_field_ocean_imex": ("four_field_ocean", "imex"),
    "zlevel_ensemble_lie": ("zlevel_ensemble", "lie"),
}


def log(*a):
    print(*a, flush=True)


def workload(name):
    import workloads as W
    return getattr(W, name)()


def gpu_part(case, steps, out_path):
    import paper_2605_16082_amd as P
    wname, scheme = CASES[case]
    w = workload(wname)
    log(f"gpu: {case}, {w.n_prisms} prisms, {w.n_fields} fields, {steps} steps")
    ts = P.SDG_SCHEME_SPLIT_IMEX if scheme == "imex" else P.SDG_SCHEME_SSPRK3_LIE
    s, U, kappa, state = P.from_workload(w, P.SDG_FP64, time_scheme=ts)
    log("gpu: autotuned shape", s.autotune(reps=2))
    s.scatter(w.T0, out=state)
    s.step(steps)
    s.sync()
    np.save(out_path, s.gather(state))
    log("gpu: state saved")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), required=True)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--json", default=None)
    ap.add_argument("--gpu-part", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpu_part:
        gpu_part(args.case, args.steps, args.gpu_part)
        return
    import oracle as O
    import oracle.parallel as OP

    wname, scheme = CASES[args.case]
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "gpu_state.npy")
        t0 = time.time()
        subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--case", args.case, "--steps",
                        str(args.steps), "--gpu-part", path], check=True, timeout=900)
        log(f"gpu part done ({time.time() - t0:.0f} s)")
        w = workload(wname)
        m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
        log(f"oracle: {m.P} prisms, {m.C} columns, {args.workers} workers")
        ref = OP.run_steps(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, args.steps, scheme, w.penalty,
                           workers=args.workers, log=log)
        got = np.load(path, mmap_mode="r")
        F = ref.shape[0]
        err = [float(np.abs(got[f] - ref[f]).max() / np.abs(ref[f]).max()) for f in range(F)]
    rec = {"case": args.case, "steps": args.steps, "prisms": int(m.P), "fields": F,
           "max_rel_err_per_field": err, "bar": 1e-12, "pass": bool(max(err) <= 1e-12),
           "seconds": round(time.time() - t0, 1)}
    log(json.dumps(rec))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(rec, f)
    sys.exit(0 if rec["pass"] else 1)


if __name__ == "__main__":
    main()
