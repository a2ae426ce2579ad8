"""Writes four_field_ocean_100steps.npz: the FP64 oracle's state after 100
SSP-RK3 + vertical-solve steps of the four-field ocean workload (199,712
jittered triangles x 30 sigma layers, fields u, v, temperature, salinity),
the reference of the precision forms' error after 100 steps.

    python tests/golden/make_four_field_ocean_reference.py [--workers 8] [--steps 100]

Calls only the oracle (``oracle.parallel.run_steps``, which evaluates the
oracle's own step functions over prism and column ranges in forked
processes) and the seeded workload generator.  The full state is 1.15 GB, so
the file keeps per field: max |x| and the total mass of the final state,
and 20,000 seeded random entries (index d = i * P + p for node i of prism p,
natural order).  About an hour on 8 cores.
"""

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import oracle.parallel as OP  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "four_field_ocean_100steps.npz")
N_SAMPLE = 20000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--steps", type=int, default=100)
    args = ap.parse_args()
    w = W.four_field_ocean()
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    t0 = time.time()
    x = OP.run_steps(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, args.steps, "lie", w.penalty, workers=args.workers,
                     log=lambda s: print(s, flush=True))
    F = x.shape[0]
    rng = np.random.default_rng(2605)
    idx = np.stack([np.sort(rng.choice(6 * m.P, N_SAMPLE, replace=False)) for _ in range(F)])
    flat = x.reshape(F, -1)
    vals = np.stack([flat[f, idx[f]] for f in range(F)])
    np.savez_compressed(OUT, steps=args.steps, idx=idx, vals=vals, fmax=np.abs(flat).max(axis=1),
                        mass=O.mass(m, x), mass0=O.mass(m, w.T0))
    print("wrote", OUT, "in %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
