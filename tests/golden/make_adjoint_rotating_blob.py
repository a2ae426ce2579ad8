"""Writes adjoint_rotating_blob_200steps.txt: the oracle's gradient of
J = ||x_N||_M after 200 steps of the SSP-RK3 + vertical-solve step on the
rotating-blob workload (1,800 triangles x 10 sigma layers), with respect to
the initial field and the per-layer diffusivity.

    python tests/golden/make_adjoint_rotating_blob.py

Calls only the oracle and the seeded workload generator.  Stored: J; per
layer dJ/dkappa_l and the sum of its terms' magnitudes; max |dJ/dT0| and the
2-norm of dJ/dT0; dJ/dT0 at 4,096 seeded random degrees of freedom and at the
64 largest.  DOF index d = (i * P + p) for node i of prism p (natural order).
Takes about 8 minutes on one core.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import oracle.adjoint as OA  # noqa: E402
import workloads as W  # noqa: E402

N_STEPS = 200
OUT = os.path.join(HERE, "adjoint_rotating_blob_200steps.txt")


def main():
    w = W.rotating_blob()
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    t0 = time.time()
    J, gT, gk, gk_abs = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, N_STEPS, w.penalty, return_scale=True)
    g = gT[0].ravel()                       # (6 * P,), index i * P + p
    rng = np.random.default_rng(2605)
    idx = np.union1d(rng.choice(g.size, 4096, replace=False), np.argsort(np.abs(g))[-64:])
    with open(OUT, "w") as f:
        f.write("# oracle gradient, rotating_blob(seed=0, n=30, n_layers=10), %d SSP-RK3 + solve steps\n" % N_STEPS)
        f.write("# written by tests/golden/make_adjoint_rotating_blob.py (oracle only)\n")
        f.write("J %.17e\n" % J)
        for l in range(len(gk)):
            f.write("dkappa %d %.17e %.17e\n" % (l, gk[l], gk_abs[l]))
        f.write("dT0_max %.17e\n" % np.abs(g).max())
        f.write("dT0_norm2 %.17e\n" % np.sqrt(np.sum(g * g)))
        for d in idx:
            f.write("dT0 %d %.17e\n" % (d, g[d]))
    print("wrote", OUT, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
