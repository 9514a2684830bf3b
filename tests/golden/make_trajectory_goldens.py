"""Writes the FP64 oracle's RK4 end states u(T) for the three full-size forward
workloads, with the oracle's own RBF quadrature weights q, to this folder:

  torus32768_rk4.npz       torus R = 1, r = 0.4, N = 32768, exponential Mexican
                           hat, one state, dt = 0.02, 500 steps: q and the whole
                           of u(T).
  ellipsoid65536_rk4.npz   ellipsoid (1, .8, .6), N = 65536, Gaussian Mexican
                           hat, 64 states with their own thresholds, dt = 0.05,
                           200 steps: q, u(T) of every state on a fixed sample of
                           rows (4096 seeded rows plus each state's largest-|u|
                           row), and max_i |u_i(T)| per state over all rows.
  batch48_rk4.npz          the 48-problem uneven batch (sphere, torus,
                           ellipsoid, bumpy sphere; N log-uniform in
                           [1000, 40000]; 1, 4 or 16 states), dt = 0.05,
                           100 steps: per problem q, u(T) on up to 512 seeded
                           rows plus each state's largest-|u| row, and the
                           per-state max |u(T)|.

The operator is the dense sum of eq. NFODETilde (section 2.2) built once per
problem in FP64, the weights are the surface RBF-QF of section 3.3 (phs r^3,
degree 2, k = 32), the stepper is classical RK4.  Only the oracle and the
seeded workload generators are called.  Run from the repository root:

  python tests/golden/make_trajectory_goldens.py [torus|ellipsoid|batch ...]

Memory: the ellipsoid's FP64 kernel matrix takes 32 GiB; run the parts one
after the other.
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

HERE = os.path.dirname(os.path.abspath(__file__))
ELLIPSOID_SAMPLE = 4096
BATCH_SAMPLE = 512


def _log(t0, msg):
    print("[%7.1fs] %s" % (time.time() - t0, msg), flush=True)


def _sample_rows(n, k, seed, uT):
    """k seeded distinct rows (all rows if n <= k) plus every state's largest-|u| row."""
    rng = np.random.default_rng(seed)
    rows = np.arange(n) if n <= k else rng.choice(n, size=k, replace=False)
    peaks = np.argmax(np.abs(uT), axis=1)
    return np.unique(np.concatenate([rows, peaks])).astype(np.int64)


def _run(w, q, t0):
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    _log(t0, "%s: kernel matrix built" % w.name)
    uT = NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)
    _log(t0, "%s: %d RK4 steps done" % (w.name, w.steps))
    del op
    return uT


def torus():
    t0 = time.time()
    w = C.torus_exp()
    q = Q.surface_weights(w.surface)
    _log(t0, "torus weights, sum q = %.15g" % q.sum())
    uT = _run(w, q, t0)
    out = os.path.join(HERE, "torus32768_rk4.npz")
    np.savez_compressed(out, q=q, uT=uT, n=w.n, steps=w.steps, dt=w.dt)
    _log(t0, "wrote " + out)


def ellipsoid():
    t0 = time.time()
    w = C.ellipsoid_ensemble()
    q = Q.surface_weights(w.surface)
    _log(t0, "ellipsoid weights, sum q = %.15g" % q.sum())
    uT = _run(w, q, t0)
    rows = _sample_rows(w.n, ELLIPSOID_SAMPLE, 20, uT)
    out = os.path.join(HERE, "ellipsoid65536_rk4.npz")
    np.savez_compressed(out, q=q, rows=rows, uT_rows=uT[:, rows], uT_absmax=np.max(np.abs(uT), axis=1),
                        n=w.n, steps=w.steps, dt=w.dt)
    _log(t0, "wrote " + out)


def batch():
    t0 = time.time()
    ws = C.uneven_batch()
    qs, rows, uts, amax = [], [], [], []
    for p, w in enumerate(ws):
        q = Q.surface_weights(w.surface)
        uT = _run(w, q, t0)
        r = _sample_rows(w.n, BATCH_SAMPLE, 300 + p, uT)
        qs.append(q)
        rows.append(r)
        uts.append(uT[:, r])
        amax.append(np.max(np.abs(uT), axis=1))
    out = os.path.join(HERE, "batch48_rk4.npz")
    arrays = {"n": np.array([w.n for w in ws]), "b": np.array([w.b for w in ws]), "steps": ws[0].steps,
              "dt": ws[0].dt}
    for p in range(len(ws)):
        arrays["q%02d" % p] = qs[p]
        arrays["rows%02d" % p] = rows[p]
        arrays["uT%02d" % p] = uts[p]
        arrays["absmax%02d" % p] = amax[p]
    np.savez_compressed(out, **arrays)
    _log(t0, "wrote " + out)


if __name__ == "__main__":
    parts = sys.argv[1:] or ["torus", "ellipsoid", "batch"]
    for part in parts:
        {"torus": torus, "ellipsoid": ellipsoid, "batch": batch}[part]()
