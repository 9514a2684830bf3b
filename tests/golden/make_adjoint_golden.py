"""Writes the FP64 oracle's adjoint gradients for the full-size torus adjoint
workload (N = 16384, 400 RK4 steps, dt = 0.02) to torus16384_adjoint.npz.

Calls only the oracle and the seeded workload generators.  Run from the
repository root:  python tests/golden/make_adjoint_golden.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import neural_field as NF  # noqa: E402
from oracle import quadrature as Q  # noqa: E402
from workloads import configs as C  # noqa: E402


def main(n=16384, steps=400, out=None):
    out = out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "torus%d_adjoint.npz" % n)
    t0 = time.time()
    w = C.torus_adjoint(n, steps)
    q = Q.surface_weights(w.surface)
    tp = w.extra["target_params"]
    print("weights %.1fs" % (time.time() - t0), flush=True)
    target = NF.rk4(NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, tuple(tp[:4])), w.u0, w.beta, tp[4],
                    w.dt, w.steps)
    print("target %.1fs" % (time.time() - t0), flush=True)
    op = NF.ParamOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    L, gu, gp = NF.adjoint_gradients(op, w.u0, w.beta, float(w.theta[0]), w.dt, w.steps, target)
    uT = NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)
    print("adjoint %.1fs L=%.6e" % (time.time() - t0, L), flush=True)
    np.savez(out, q=q, target=target, uT=uT, loss=L, grad_u0=gu, grad_p=gp, n=n, steps=steps)
    print("wrote", out)


if __name__ == "__main__":
    main(*(int(a) for a in sys.argv[1:3]))
