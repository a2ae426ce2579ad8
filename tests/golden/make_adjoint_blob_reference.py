"""Writes adjoint_blob_200steps.npz: the oracle's gradient of J = ||x_N||_M
after 200 SSP-RK3 + vertical-solve steps of the differentiation workload
(49,928 triangles x 20 sigma layers = 998,560 prisms, one field), with
respect to the initial field and the per-layer diffusivity.

    python tests/golden/make_adjoint_blob_reference.py [--workers 8]

Calls only the oracle and the seeded workload generator: the forward states
come from ``oracle.parallel.run_steps`` (the oracle's own step functions over
prism and column ranges in forked processes), the reverse sweep from
``oracle.adjoint.gradient`` on its assembled sparse operators.  The gradient
is exact for the discrete step, so it does not depend on the checkpoint
interval the GPU uses.  Stored: J; per layer dJ/dkappa_l and the sum of its
terms' magnitudes; max |dJ/dT0| and its 2-norm; dJ/dT0 at 20,000 seeded
random degrees of freedom and at the 64 largest (index d = i * P + p for
node i of prism p, natural order).  About an hour and 30 GB of memory on
8 cores.
"""

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import oracle.adjoint as OA  # noqa: E402
import oracle.parallel as OP  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "adjoint_blob_200steps.npz")
N_SAMPLE = 20000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--steps", type=int, default=None, help="fewer steps, for a timing trial (not written)")
    args = ap.parse_args()
    w = W.adjoint_blob()
    n = args.steps or w.n_steps
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    t0 = time.time()

    def log(s):
        print(s, flush=True)

    xs = OP.run_steps(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n, "lie", w.penalty, workers=args.workers,
                      log=log, states=True)
    log("forward states done (%.0f s)" % (time.time() - t0))
    J, gT, gk, gk_abs = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n, w.penalty, return_scale=True,
                                    xs=xs)
    log("reverse sweep done (%.0f s)" % (time.time() - t0))
    g = gT[0].ravel()                       # (6 * P,), index i * P + p
    rng = np.random.default_rng(2605)
    idx = np.union1d(rng.choice(g.size, N_SAMPLE, replace=False), np.argsort(np.abs(g))[-64:])
    if args.steps:
        log("J %.17e, max |dJ/dT0| %.6e (timing trial, not written)" % (J, np.abs(g).max()))
        return
    np.savez_compressed(OUT, steps=n, J=J, dkappa=gk, dkappa_abs=gk_abs, dT0_max=np.abs(g).max(),
                        dT0_norm2=np.sqrt(np.sum(g * g)), idx=idx, vals=g[idx])
    log("wrote %s in %.0f s" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
