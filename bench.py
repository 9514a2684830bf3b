"""Throughput of the neural-field hot path on one MI355X.

Headline workload (one "step" = one whole integration): the ellipsoid
(1, .8, .6) ensemble, N = 65536 nodes with the FP64 oracle's RBF-QF weights,
Gaussian Mexican hat w(r) = exp(-r^2/.15^2) - .5 exp(-r^2/.4^2), B = 64 states
(one seeded bump each, thresholds theta_b ~ U(.15, .3), sigmoid beta = 20),
classical RK4 with dt = 0.05 for 200 steps (800 operator applications of
N^2 B pair-interactions each), FP64 state updates.  Inputs are resident on the
GPU before the timed region.  Every form runs: the split-precision ones (W or
fused on-the-fly, BF16 or FP16 hi + lo products on the matrix cores) and the
FP32 ones (vector-unit and matrix-core pair sums); `value` is the fastest
split form's median over the timed integrations, and every form's u(T) is
compared member by member with the oracle's stored u(T)
(tests/golden/ellipsoid65536_rk4.npz, written by the oracle alone).

Sub-legs: the torus (N = 32768, B = 1, 500 steps; on-the-fly FP32 and FP32 W,
against the oracle's whole u(T)), the small sphere (N = 2000, time per step),
the 48-problem uneven batch (100 steps, against the oracle), the adjoint and
the GPU quadrature weights.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # bytes/s, MI355X HBM3E
# FP32 vector issue: 157.3 TFLOP/s = 256 CUs x 128 FP32 lanes/clock x 2 flop (FMA) x 2.4 GHz,
# i.e. 78.6e12 full-rate lane-operations/s; transcendental instructions (exp2, sqrt)
# issue at a quarter of that rate, so each costs 4 full-rate slots.
VALU_LANES_PER_S = 256 * 128 * 2.4e9
TRANS_COST = 4.0
MFMA_BF16_PEAK = 2.5e15      # dense BF16 / FP16 matrix-core flop/s
MFMA_F32_PEAK = 157.3e12     # dense FP32 matrix-core flop/s
# Algorithmic lane-operation slots per unordered pair {i, j} of the B = 1
# on-the-fly kernel (the kernel is radial, so one evaluation serves y_i and y_j):
#   evaluation: 3 sub + 1 mul + 2 fma (r^2) + 1 mul (rho t) = 7 full-rate, plus
#   2 exp2 (Gaussian) or sqrt + 2 exp2 (exponential) at 4 slots each, and 1 fma
#   for the normalised kernel u = exp2(-t) + kappa exp2(-rho t);
#   accumulation: 1 fma into y_i and 1 fma into y_j.
# With length scales in the ratio rho = 1/m (m = 2, 3, 4) the kernel takes the
# excitatory exponential as the m-th power of the inhibitory one and scales the
# coordinates by the inhibitory length: one exp2 and the rho t multiply fewer;
# u = e (e^(m-1) + kappa) then takes 2 (m = 2, 3) or 3 (m = 4) operations.


def eval_slots(kind, m):
    """Slots to evaluate u for one pair (see above)."""
    trans = (2 if kind == 0 else 3) - (1 if m else 0)
    return (6 if m else 7) + trans * TRANS_COST + (1 if not m else (2 if m <= 3 else 3))


def sym_pow(kind, s_e, s_i):
    """m when s_e/s_i (squared for the Gaussian) is 1/m with m in {2, 3, 4}, else 0."""
    rho = s_e / s_i
    if kind == 0:
        rho *= rho
    m = 1.0 / rho
    mi = int(round(m))
    return mi if 2 <= mi <= 4 and abs(m - mi) <= 1e-12 * mi else 0


def slots_per_unordered_pair(kind, m):
    return eval_slots(kind, m) + 2


def fused_slots_per_w(kind, m, fp16=False, norm=False, far=None):
    """Slots per W entry of the fused on-the-fly split forms: the evaluation of u
    above (the weights sit in G) and the hi/lo split: FP16 3 (two conversions of
    a pair of entries at half a slot each, the hi value back to FP32, the
    subtraction) plus the lift of u; BF16 2 (the remainder w - hi is one
    dot-product instruction).  With the norm expansion (BF16, see
    fused_norm_path) t comes from the FP32 matrix cores (FUSED_T_FLOPS_PER_W):
    the 3 subtractions, the square and the 2 multiply-adds of r^2 leave the
    vector units.  The far form (far not None: BF16, norm expansion, two
    exponentials, nfr_far_blocks) takes rho t from the matrix product and splits
    by shift and subtraction (3 slots, as the dot-product instruction does not
    run beside the matrix cores): an entry of a far block is one exp2 and the
    split (7), of a near block t = (rho t) / rho, two exp2, a multiply-add and
    the split (13)."""
    if far is not None:
        return TRANS_COST + 3 if far else 1 + 2 * TRANS_COST + 1 + 3
    split = 3 + 1 if fp16 else 2
    return eval_slots(kind, m) - (6 if norm else 0) + split


# FP32 matrix-core flops per W entry of the norm expansion: t is the product of
# the column's 4 values and the row's 4 values (32x32x2 FP32 MFMAs).
FUSED_T_FLOPS_PER_W = 8.0
# BF16 matrix-core flops per W entry of the split forms: 3 products x 2 flop x 64 states.
FUSED_BF16_FLOPS_PER_W = 384.0


# The fused BF16 kernel evaluates r^2 of Gaussian kernels on non-periodic
# surfaces by the norm expansion while sig^2 max|x|^2, for the steeper of the
# two exponentials, is at most this bound.
NORM_MAX_T = 96.0


def fused_norm_path(kind, kernel, m, max_r2):
    """Whether the fused BF16 kernel takes the norm expansion for this Gaussian or
    exponential kernel on a non-periodic surface with max |x|^2 = max_r2 (of the
    FP32 coordinates)."""
    import math
    if kind != 0:
        return False
    s_e, s_i = kernel[1], kernel[3]
    if m:
        sig2, steep = math.log2(math.e) / (s_i * s_i), m
    else:
        sig2, steep = math.log2(math.e) / (s_e * s_e), max(1.0, (s_e / s_i) ** 2)
    return sig2 * steep * max_r2 <= NORM_MAX_T


def sym_kernel_name(kind, m, periodic=False):
    return "k_otf_sym<%d>" % (kind + (2 if periodic else 0) + ((m - 1) << 2 if m else 0))


# Sources that define the profiled kernels (their code and tile constants).
TRAFFIC_SOURCES = ("common.h", "kernels_core.h", "kernels_mfma.h", "kernels_tile.h")


def traffic_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2504_13379_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernels' sources changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if traffic_sources_sha256() != rec.get("sources_sha256") or kernel not in rec:
        return None
    return rec[kernel]["bytes"]


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_golden(name):
    """Stored FP64 oracle results (written by tests/golden/make_trajectory_goldens.py)."""
    import numpy as np
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        raise SystemExit("bench.py: missing %s (the oracle's stored trajectory)" % path)
    return np.load(path)


def finite(x):
    """A float for the JSON line, None where nothing was measured (NaN)."""
    x = float(x)
    return x if x == x else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed integrations of the headline form")
    ap.add_argument("--warmup", type=int, default=1, help="untimed integrations of the headline form")
    ap.add_argument("--forms", default="otf_bf16x3,bf16x3,otf_fp16x3,fp16x3,otf_fp32_mfma,otf_fp32",
                    help="ensemble forms to run (the split ones compete for the headline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-torus", action="store_true", help="skip the N = 32768 torus leg")
    ap.add_argument("--no-small", action="store_true", help="skip the N = 2000 sphere time-per-step leg")
    ap.add_argument("--probes", action="store_true", help="also run the roofline microbenchmarks")
    ap.add_argument("--probes-only", action="store_true",
                    help="run only the roofline microbenchmarks and print their rates as one JSON line")
    ap.add_argument("--no-batch", action="store_true", help="skip the 48-problem uneven-batch leg")
    ap.add_argument("--ens-rk4-steps", type=int, default=200,
                    help="RK4 steps of the ensemble (200: the workload; fewer only for short profiler runs, "
                         "whose u(T) is then not compared with the oracle)")
    ap.add_argument("--torus-rk4-steps", type=int, default=500,
                    help="RK4 steps of the torus leg (500: the workload; fewer only for profiler runs)")
    ap.add_argument("--adjoint-rk4-steps", type=int, default=400,
                    help="RK4 steps of the torus adjoint leg (0 = skip it)")
    ap.add_argument("--quad-n", type=int, default=65536,
                    help="nodes of the surface-quadrature leg on the ellipsoid (0 = skip it)")
    return ap.parse_args()


def kernel_timing(P, ctx, fn):
    """Runs fn() with HIP events around every pair-sum launch on the context's stream;
    returns (launches, average ms per launch)."""
    import ctypes
    L = P.lib()
    L.nfr_context_set_timing(ctx.handle, 1)
    fn()
    launches, tot = ctypes.c_int64(), ctypes.c_double()
    P._lib.check(L.nfr_context_timing(ctx.handle, ctypes.byref(launches), ctypes.byref(tot)))
    L.nfr_context_set_timing(ctx.handle, 0)
    return int(launches.value), tot.value / max(1, launches.value)


def launches_per_step(P, ctx):
    """Kernel nodes per RK4 step of the graph the last graph-replayed call used."""
    import ctypes
    nodes, steps = ctypes.c_int64(), ctypes.c_int64()
    P._lib.check(P.lib().nfr_context_last_graph(ctx.handle, ctypes.byref(nodes), ctypes.byref(steps)))
    return {"graph_nodes": int(nodes.value), "graph_rk4_steps": int(steps.value),
            "launches_per_rk4_step": nodes.value / steps.value if steps.value else None}


# ------------------------------------------------------------------ headline: ellipsoid ensemble

ENS_FORMS = {"otf_bf16x3": 4, "bf16x3": 2, "otf_fp16x3": 5, "fp16x3": 3, "otf_fp32_mfma": 6, "otf_fp32": 0}
SPLIT_FORMS = ("otf_bf16x3", "bf16x3", "otf_fp16x3", "fp16x3")


def ensemble_roofline(nm, npad, kind, kernel, avg_s, max_r2, far_frac=0.0):
    """Roofline of the dominant (pair-sum) kernel of form `nm` at one launch per operator
    application; far_frac: the fraction of the fused BF16 form's W blocks that skip the
    steep exponential (nfr_far_blocks)."""
    m = sym_pow(kind, kernel[1], kernel[3])
    if nm in ("bf16x3", "fp16x3"):
        wbytes = 2.0 * 2 * npad * npad     # hi + lo, 2 bytes each, every element once
        kname = "k_mfma_apply<%s,2>" % nm[:4]
        return {"bound": "hbm", "achieved": wbytes / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": wbytes / avg_s / HBM_PEAK, "traffic": measured_traffic(kname), "kernel": kname,
                "algorithmic_bytes_per_launch": wbytes}
    if nm == "otf_fp32_mfma":
        kname = "k_mfma_otf_f32<%d,2>" % (kind + 4 * (m - 1 if m else 0))
        flops = 2.0 * float(npad) ** 2 * 64
        return {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": MFMA_F32_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": flops / avg_s / MFMA_F32_PEAK, "traffic": measured_traffic(kname), "kernel": kname,
                "alu_frac": float(npad) ** 2 * eval_slots(kind, m) / avg_s / VALU_LANES_PER_S}
    if nm == "otf_fp32":
        # one-sided multi-state pair sum: per target-source pair one evaluation of u per block
        # of 16 states (no integer-ratio shortcut in this kernel) + 1 FMA per state
        kname = "k_otf_pair_sum<%d,2,16>" % kind
        slots = float(npad) ** 2 * (-(-64 // 16) * eval_slots(kind, 0) + 64)
        return {"bound": "alu", "achieved": slots / avg_s / 1e12, "peak": VALU_LANES_PER_S / 1e12,
                "unit": "Tslot/s", "frac": slots / avg_s / VALU_LANES_PER_S, "traffic": measured_traffic(kname),
                "kernel": kname}
    # fused on-the-fly split forms: every W entry evaluated once per launch on the vector
    # units (t of the norm expansion on the FP32 matrix cores); the BF16 matrix cores do
    # 3 products x 2 flop x 64 states per entry.  The bound is the larger of the vector
    # slot share and the matrix-core time share (BF16 flops at the BF16 peak plus FP32
    # flops at the FP32 peak); for the matrix cores `achieved` is in BF16-equivalent
    # flop/s (FP32 flops weighted by the ratio of the two peaks).
    fp16 = nm == "otf_fp16x3"
    norm = not fp16 and fused_norm_path(kind, kernel, m, max_r2)
    kname = "k_mfma_otf<%s,%d,2,4>" % ("fp16" if fp16 else "bf16", kind + 4 * (m - 1 if m else 0))
    wvals = float(npad) ** 2
    far_frac = far_frac if (norm and not fp16) else 0.0
    if far_frac > 0.0:
        kname = "k_mfma_otf<bf16,%d,2,8>" % kind      # the far form runs in eight-wave workgroups
    if far_frac > 0.0:
        spw = (1.0 - far_frac) * fused_slots_per_w(kind, m, far=False) + far_frac * fused_slots_per_w(kind, m, far=True)
    else:
        spw = fused_slots_per_w(kind, m, fp16, norm)
    alu = wvals * spw / avg_s
    f32 = FUSED_T_FLOPS_PER_W if norm else 0.0
    mtime = wvals * (FUSED_BF16_FLOPS_PER_W / MFMA_BF16_PEAK + f32 / MFMA_F32_PEAK)
    mfrac = mtime / avg_s
    common = {"traffic": measured_traffic(kname), "kernel": kname, "slots_per_w": spw, "far_block_fraction": far_frac,
              "r2": "norm expansion (t on the FP32 matrix cores)" if norm else "differences",
              "alu_frac": alu / VALU_LANES_PER_S,
              "mfma_bf16_tflops": wvals * FUSED_BF16_FLOPS_PER_W / avg_s / 1e12,
              "mfma_f32_tflops": wvals * f32 / avg_s / 1e12, "mfma_time_frac": mfrac}
    if mfrac >= alu / VALU_LANES_PER_S:
        return {"bound": "mfma", "achieved": mfrac * MFMA_BF16_PEAK / 1e12, "peak": MFMA_BF16_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": mfrac, "achieved_is": "BF16-equivalent (FP32 flops x BF16/FP32 peak)",
                **common}
    return {"bound": "alu", "achieved": alu / 1e12, "peak": VALU_LANES_PER_S / 1e12, "unit": "Tslot/s",
            "frac": alu / VALU_LANES_PER_S, **common}


def ensemble_headline(P, torch, args):
    """Every requested form of the ellipsoid ensemble: one warm-up step and one timed whole
    integration each, u(T) per member against the oracle; then the fastest split form again
    with args.warmup + args.steps whole integrations (the headline, median)."""
    import numpy as np

    from workloads import configs as C
    gold = load_golden("ellipsoid65536_rk4.npz")
    w = C.ellipsoid_ensemble(steps=args.ens_rk4_steps)
    assert w.n == int(gold["n"])
    compare = w.steps == int(gold["steps"])
    rows, ref_rows, ref_max = gold["rows"], gold["uT_rows"], gold["uT_absmax"]
    # max |x|^2 of the FP32 coordinates, as the library's problem packing computes it
    xf = w.surface.xyz.astype(np.float32).astype(np.float64)
    max_r2 = float(np.max(np.sum(xf * xf, axis=1).astype(np.float32)))

    def member_err():
        if not compare:
            return np.full(w.b, np.nan)
        return np.max(np.abs(u.cpu().numpy()[:, rows] - ref_rows), axis=1) / ref_max
    ctx = P.Context(0, torch.cuda.Stream())
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(gold["q"]).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, torch.from_numpy(w.theta).cuda())
    u0 = torch.from_numpy(w.u0.copy()).cuda()
    u = u0.clone()
    pairs = 4.0 * w.steps * float(w.n) ** 2 * w.b
    far_blocks, all_blocks = prob.far_blocks(k)
    far_frac = far_blocks / all_blocks
    forms = {}
    keep = {}

    def integrate(form, W, ws, steps, graph=True):
        u.copy_(u0)
        prob.integrate(k, f, u, w.dt, steps, form=form, W=W, ws=ws, use_graph=graph)

    def timed(form, W, ws):
        ctx.stream.synchronize()
        t0 = time.perf_counter()
        integrate(form, W, ws, w.steps)
        ctx.stream.synchronize()
        return time.perf_counter() - t0

    def setup(form):
        W, t_build = None, 0.0
        if form in (P.FORM_W_BF16X3, P.FORM_W_FP16X3):
            ctx.stream.synchronize()
            tb = time.perf_counter()
            W = prob.w_build(k, form)
            ctx.stream.synchronize()
            t_build = time.perf_counter() - tb
        return W, t_build, prob.integrate_workspace(w.b, form)

    for nm in args.forms.split(","):
        form = ENS_FORMS[nm]
        print("bench: ensemble form %s" % nm, file=sys.stderr, flush=True)
        W, t_build, ws = setup(form)
        integrate(form, W, ws, 1)                         # warm-up (captures the step graph)
        sec = timed(form, W, ws)
        lps = launches_per_step(P, ctx)
        err = member_err()
        n_l, avg_ms = kernel_timing(P, ctx, lambda: integrate(form, W, ws, max(1, w.steps // 4), graph=False))
        forms[nm] = {"value": pairs / sec, "unit": "pair-interactions/s", "ms_per_integration": sec * 1e3,
                     "w_build_ms": t_build * 1e3, "kernel_avg_ms": avg_ms, **lps,
                     "rel_linf_vs_fp64_max": finite(err.max()), "rel_linf_vs_fp64_median": finite(np.median(err)),
                     "roofline": ensemble_roofline(nm, prob.npad, w.kernel_kind, w.kernel, avg_ms * 1e-3, max_r2, far_frac)}
        keep[nm] = err
        del W
        torch.cuda.empty_cache()
    split = [nm for nm in forms if nm in SPLIT_FORMS]
    best = max(split, key=lambda nm: forms[nm]["value"])
    form = ENS_FORMS[best]
    print("bench: headline form %s, %d warmup + %d timed integrations" % (best, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    W, _, ws = setup(form)
    for _ in range(args.warmup):
        integrate(form, W, ws, w.steps, graph=False)
    ctx.stream.synchronize()
    # the timed region: args.steps whole integrations launched directly, with HIP
    # events around every pair-sum launch on the context's stream (the kernel's
    # duration for the roofline comes from the same runs as the throughput)
    L = P.lib()
    L.nfr_context_set_timing(ctx.handle, 1)
    times = []
    t_all0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.stream.synchronize()
        t0 = time.perf_counter()
        integrate(form, W, ws, w.steps, graph=False)
        ctx.stream.synchronize()
        times.append(time.perf_counter() - t0)
    t_all = time.perf_counter() - t_all0
    import ctypes
    launches, tot = ctypes.c_int64(), ctypes.c_double()
    P._lib.check(L.nfr_context_timing(ctx.handle, ctypes.byref(launches), ctypes.byref(tot)))
    L.nfr_context_set_timing(ctx.handle, 0)
    n_l, avg_ms = int(launches.value), tot.value / max(1, launches.value)
    err = member_err()
    med = sorted(times)[len(times) // 2]
    head = {"form": best, "value": pairs / med, "ms_per_step": med * 1e3, "ms_all_timed": t_all * 1e3,
            "times_ms": [t * 1e3 for t in times], "kernel_avg_ms": avg_ms, "kernel_launches_timed": n_l,
            "timed_launch": "directly launched (HIP events around each pair-sum launch)",
            "rel_linf_vs_fp64": [finite(e) for e in err], "rel_linf_vs_fp64_max": finite(err.max()),
            "roofline": ensemble_roofline(best, prob.npad, w.kernel_kind, w.kernel, avg_ms * 1e-3, max_r2, far_frac),
            "launches": launches_per_step(P, ctx)}
    del W
    torch.cuda.empty_cache()
    return w, gold, head, forms


# ------------------------------------------------------------------ torus (B = 1)


def torus_leg(P, torch, args):
    """Torus N = 32768, B = 1, exponential Mexican hat, 500 RK4 steps with the oracle's
    weights: on-the-fly FP32 (symmetric kernel) and FP32 W (built inside each timed run),
    three timed integrations each, u(T) against the oracle's whole u(T)."""
    import numpy as np

    from workloads import configs as C
    gold = load_golden("torus32768_rk4.npz")
    w = C.torus_exp(steps=args.torus_rk4_steps)
    ctx = P.Context(0, torch.cuda.Stream())
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(gold["q"]).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    u0 = torch.from_numpy(w.u0.copy()).cuda()
    u = u0.clone()
    ref = gold["uT"]
    out = {"workload": "torus R=1 r=0.4, N=32768, exp Mexican hat, B=1, RK4 dt=0.02 x %d steps, oracle weights"
                       % w.steps}
    pairs = 4.0 * w.steps * float(w.n) ** 2
    for nm, form in (("otf_fp32", P.FORM_ONTHEFLY_FP32), ("w_fp32", P.FORM_W_FP32)):
        ws = prob.integrate_workspace(1, form)
        W = prob.w_build(k, form) if form == P.FORM_W_FP32 else None

        def one(graph=True, steps=w.steps):
            u.copy_(u0)
            if W is not None:
                P._lib.check(P.lib().nfr_w_build(prob.handle, __import__("ctypes").byref(k), form, W.data_ptr(),
                                                 W.numel()))
            prob.integrate(k, f, u, w.dt, steps, form=form, W=W, ws=ws, use_graph=graph)

        one()                                     # warm-up with graph replay (captures the step graph)
        lps = launches_per_step(P, ctx)
        one(graph=False)
        import ctypes
        L = P.lib()
        L.nfr_context_set_timing(ctx.handle, 1)   # events around every pair launch of the timed runs
        times = []
        for _ in range(3):
            ctx.stream.synchronize()
            t0 = time.perf_counter()
            one(graph=False)
            ctx.stream.synchronize()
            times.append(time.perf_counter() - t0)
        launches, tot = ctypes.c_int64(), ctypes.c_double()
        P._lib.check(L.nfr_context_timing(ctx.handle, ctypes.byref(launches), ctypes.byref(tot)))
        L.nfr_context_set_timing(ctx.handle, 0)
        avg_ms = tot.value / max(1, launches.value)
        gtimes = []
        for _ in range(3):
            ctx.stream.synchronize()
            t0 = time.perf_counter()
            one()
            ctx.stream.synchronize()
            gtimes.append(time.perf_counter() - t0)
        err = float(np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref))) if w.steps == int(gold["steps"]) \
            else None
        med = min(sorted(times)[1], sorted(gtimes)[1])
        entry = {"value": pairs / med, "unit": "pair-interactions/s", "ms_per_integration": med * 1e3,
                 "ms_launched": sorted(times)[1] * 1e3, "ms_graph": sorted(gtimes)[1] * 1e3,
                 "kernel_avg_ms": avg_ms, "rel_linf_vs_fp64": err, **lps}
        if nm == "otf_fp32":
            m = sym_pow(w.kernel_kind, w.kernel[1], w.kernel[3])
            name = sym_kernel_name(w.kernel_kind, m)
            ops = slots_per_unordered_pair(w.kernel_kind, m) * float(prob.npad) ** 2 / 2.0
            entry["roofline"] = {"bound": "alu", "achieved": ops / (avg_ms * 1e-3) / 1e12,
                                 "peak": VALU_LANES_PER_S / 1e12, "unit": "Tslot/s",
                                 "frac": ops / (avg_ms * 1e-3) / VALU_LANES_PER_S, "traffic": measured_traffic(name),
                                 "kernel": name, "slots_per_unordered_pair": slots_per_unordered_pair(w.kernel_kind, m)}
        else:
            b = float(w.n) * prob.npad * 4.0
            entry["roofline"] = {"bound": "hbm", "achieved": b / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                                 "unit": "GB/s", "frac": b / (avg_ms * 1e-3) / HBM_PEAK,
                                 "traffic": measured_traffic("k_w_gemv_f32<1>"), "kernel": "k_w_gemv_f32<1>"}
        out[nm] = entry
        del W
        torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ uneven batch


def batch_leg(P, torch, args):
    """The 48-problem uneven batch (N log-uniform in [1000, 40000], B in {1, 4, 16}) with the
    oracle's weights: tuned persistent launches, graph-replayed steps, 100 RK4 steps, every
    state against the oracle's stored u(T) (sampled rows)."""
    import numpy as np

    from workloads import configs as C
    gold = load_golden("batch48_rk4.npz")
    ws_list = C.uneven_batch()
    steps, dt = ws_list[0].steps, ws_list[0].dt
    stream = torch.cuda.Stream()
    ctx = P.Context(0, stream)
    probs, ks, fs, Bs, u0s = [], [], [], [], []
    with torch.cuda.stream(stream):
        for p, w in enumerate(ws_list):
            probs.append(P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(),
                                   torch.from_numpy(gold["q%02d" % p]).cuda()))
            ks.append(P.kernel_struct(w.kernel_kind, *w.kernel))
            fs.append(P.Firing(w.beta, torch.from_numpy(w.theta).cuda()))
            Bs.append(w.b)
            u0s.append(torch.from_numpy(w.u0.copy()).cuda())
    torch.cuda.synchronize()
    batch = P.Batch(ctx, probs, ks, fs, Bs)
    ws = batch.workspace()
    states = [u.clone() for u in u0s]
    t0 = time.perf_counter()
    best = batch.tune(states, ws)
    t_tune = time.perf_counter() - t0
    batch.integrate(states, dt, 1, use_graph=True, ws=ws)       # warm-up
    for s_, u in zip(states, u0s):
        s_.copy_(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.integrate(states, dt, steps, use_graph=True, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    worst = 0.0
    for p, u in enumerate(states):
        rows = gold["rows%02d" % p]
        err = np.max(np.abs(u.cpu().numpy()[:, rows] - gold["uT%02d" % p]), axis=1) / gold["absmax%02d" % p]
        worst = max(worst, float(err.max()))
    pair_ints = sum(4.0 * steps * float(w.n) ** 2 * w.b for w in ws_list)
    # algorithmic slots of the pair kernel per stage: per target-source pair and state block
    # one evaluation of u (eval_slots: 16 for the Gaussian), plus 1 FMA per state; blocks of
    # 1, 4 or 16 states
    slots = 0.0
    for w in ws_list:
        npad = -(-w.n // 256) * 256
        bs = 1 if w.b == 1 else (4 if w.b <= 4 else 16)
        slots += float(npad) ** 2 * (-(-w.b // bs) * eval_slots(0, 0) + w.b)
    slots *= 4.0 * steps
    chunk, wgs = batch.config
    return {"workload": "48 problems, N log-uniform [1000, 40000], sphere/torus/ellipsoid/bumpy, Gauss Mexican hat, "
                        "B in {1,4,16}, RK4 dt=0.05 x %d steps, graph-replayed, oracle weights" % steps,
            "value": pair_ints / (t1 - t0), "unit": "pair-interactions/s", "ms_per_integration": (t1 - t0) * 1e3,
            "rel_linf_vs_fp64_max": worst,
            "roofline": {"bound": "alu", "achieved": slots / (t1 - t0) / 1e12, "peak": VALU_LANES_PER_S / 1e12,
                         "unit": "Tslot/s", "frac": slots / (t1 - t0) / VALU_LANES_PER_S,
                         "note": "whole integration time (pair kernel, combine, launch gaps)"},
            "tuned": {"chunk": chunk, "wgs_per_cu": wgs, "best_stage_ms": best, "tune_ms": t_tune * 1e3},
            **launches_per_step(P, ctx)}


# ------------------------------------------------------------------ CPU baseline


def host_info():
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()]
    except Exception:                       # noqa: BLE001 - diagnostics only
        blas = []
    return {"os_cpu_count": os.cpu_count(), "sched_cores": len(os.sched_getaffinity(0)), "cpu_model": model,
            "blas": blas}


def cpu_baseline(w, q, n_rows):
    """The FP64 oracle's operator (its apply_K: kernel rows from the definition, then a
    BLAS product with the 64 states' q f(u)) on a bounded sample of one application of the
    headline workload: n_rows target rows x all sources x all states; one thread, then every
    host thread the process may use."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import neural_field as NF
    rows = np.random.default_rng(7).choice(w.n, n_rows, replace=False)
    cores = len(os.sched_getaffinity(0))
    out = {}
    for threads in (1, cores):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            NF.apply_K(w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows=rows)
            t1 = time.perf_counter()
        out[threads] = float(n_rows) * w.n * w.b / (t1 - t0)
    return {"value": out[cores], "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
            "value_1_thread": out[1],
            "sample": "one operator application of the ellipsoid ensemble: %d of %d target rows x all %d sources "
                      "x %d states, FP64 NumPy (elementwise kernel rows, BLAS product)" % (n_rows, w.n, w.n, w.b),
            "host": host_info()}


def small_leg(P, torch, args):
    """Unit sphere N = 2000, B = 1, Gaussian Mexican hat, 50 RK4 steps: at this size the step is
    launch-bound, so the figure of merit is time per RK4 step (graph replay vs launching every
    kernel); the two runs must agree bit for bit (parity with the oracle is the tests' job)."""
    import numpy as np

    from workloads import configs as C
    w = C.sphere_small(2000)
    q = C.area_share_weights(w.surface)
    ctx = P.Context(0, torch.cuda.Stream())
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    ws = prob.integrate_workspace(1, P.FORM_ONTHEFLY_FP32)
    out = {"workload": "unit sphere, Fibonacci N=2000, Gauss Mexican hat, B=1, RK4 dt=0.05 x %d steps" % w.steps}
    finals = {}
    for graph in (True, False):
        u = torch.from_numpy(w.u0.copy()).cuda()
        prob.integrate(k, f, u, w.dt, w.steps, form=P.FORM_ONTHEFLY_FP32, ws=ws, use_graph=graph)   # warm-up
        times = []
        for _ in range(5):
            u.copy_(torch.from_numpy(w.u0))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prob.integrate(k, f, u, w.dt, w.steps, form=P.FORM_ONTHEFLY_FP32, ws=ws, use_graph=graph)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = sorted(times)[len(times) // 2]
        nm = "graph" if graph else "launched"
        out[nm] = {"us_per_rk4_step": t / w.steps * 1e6,
                   "value": 4.0 * w.steps * float(w.n) ** 2 / t, "unit": "pair-interactions/s"}
        finals[nm] = u.cpu().numpy()
    out["graph_equals_launched"] = bool(np.array_equal(finals["graph"], finals["launched"]))
    return out


def adjoint_leg(P, torch, args):
    """Torus adjoint workload: N = 16384, RK4 dt = 0.02, checkpoints every 40 steps;
    forward with checkpoints + discrete adjoint (gradients w.r.t. u0 and 5 parameters),
    timed with graph replay on a side stream."""
    import ctypes

    import numpy as np

    from workloads import configs as C
    w = C.torus_adjoint(16384, args.adjoint_rk4_steps)
    q = C.area_share_weights(w.surface)
    stream = torch.cuda.Stream()
    params = torch.tensor(list(w.kernel) + [float(w.theta[0])], dtype=torch.float64)
    every = w.extra["ckpt_every"]

    def setup(ctx):
        prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
        u0 = torch.from_numpy(w.u0[0].copy()).cuda()
        return prob, u0, torch.zeros_like(u0)

    def run(prob, u0, target):
        x0 = u0.clone().requires_grad_(True)
        pp = params.clone().requires_grad_(True)
        uT = P.NeuralFieldRK4.apply(x0, pp, prob, w.kernel_kind, w.beta, w.dt, w.steps, every)
        loss = ((uT - target) ** 2).sum()
        loss.backward()
        return x0.grad, pp.grad

    # timed: a context with its own stream (forward steps and adjoint segments replay graphs)
    with torch.cuda.stream(stream):
        gctx = P.Context(0, stream)
        gargs = setup(gctx)
        run(*gargs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gu, gp = run(*gargs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    # pair-kernel durations: HIP events around every launch of one eager run on the null stream
    L = P.lib()
    null = torch.cuda.default_stream()
    with torch.cuda.stream(null):
        ctx = P.Context(0, null)
        eargs = setup(ctx)
        L.nfr_context_set_timing(ctx.handle, 1)
        run(*eargs)
        torch.cuda.synchronize()
    launches, tot = ctypes.c_int64(), ctypes.c_double()
    P._lib.check(L.nfr_context_timing(ctx.handle, ctypes.byref(launches), ctypes.byref(tot)))
    L.nfr_context_set_timing(ctx.handle, 0)
    evals = 3 * 4.0 * w.steps * float(w.n) ** 2        # forward, segment recompute, adjoint sweep
    # algorithmic slots: forward and recompute on the symmetric kernel, the adjoint sweep on its
    # four-channel symmetric transpose kernel (r^2 6, the rho t multiply only without an integer
    # ratio (with rho = 1/m the coordinates are in inhibitory units), e1 = e2^m, e*t products, 8 FMAs)
    npad = -(-w.n // 256) * 256
    m = sym_pow(w.kernel_kind, w.kernel[1], w.kernel[3])
    trans = (2 if w.kernel_kind == 0 else 3) - (1 if m else 0)
    adj_slots = (6 if m else 7) + trans * TRANS_COST + (0 if not m else (1 if m == 2 else 2)) + 2 + 8
    slots = 4.0 * w.steps * float(npad) ** 2 / 2 * (2 * slots_per_unordered_pair(w.kernel_kind, m) + adj_slots)
    return {"workload": "torus N=16384, exp Mexican hat, RK4 dt=0.02 x %d steps, checkpoints every %d, "
                        "loss |u(T)|^2" % (w.steps, every),
            "value": evals / (t1 - t0), "unit": "pair-evaluations/s (forward + recompute + adjoint)",
            "ms_forward_plus_gradient": (t1 - t0) * 1e3, "pair_kernel_launches": int(launches.value),
            "pair_kernel_avg_ms": tot.value / max(1, launches.value),
            "roofline": {"bound": "alu", "achieved": slots / (tot.value * 1e-3) / 1e12, "peak": VALU_LANES_PER_S / 1e12,
                         "unit": "Tlane-op/s", "frac": slots / (tot.value * 1e-3) / VALU_LANES_PER_S,
                         "note": "pair kernels only (forward, recompute, adjoint sweep)"},
            "grad_norm_u0": float(gu.norm()), "grad_params": [float(v) for v in gp]}


def quad_leg(P, torch, args):
    """Surface quadrature weights (stencils, projection points, planar RBF-QF
    solves, accumulation) on the GPU for the ellipsoid of the ensemble workload,
    at full size and at a quarter size (where the CPU baseline runs)."""
    from workloads import meshes
    from workloads import surfaces as S
    ctx = P.Context(0)
    out = {}
    for n in (args.quad_n // 4, args.quad_n):
        surf = S.ellipsoid(n)
        tris = meshes.triangulate(surf)
        x = torch.from_numpy(surf.xyz).cuda()
        nr = torch.from_numpy(surf.normals).cuda()
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q = P.quad_weights(ctx, x, nr, tris, True, 32)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out["n%d" % n] = {"triangles": int(tris.shape[0]), "gpu_ms": best * 1e3,
                          "triangles_per_s": tris.shape[0] / best}
        if n == args.quad_n // 4 and not args.no_cpu_baseline:
            out["n%d" % n]["cpu_baseline"] = cpu_baseline_quad(surf, q.cpu().numpy())
    return {"workload": "ellipsoid (1, .8, .6), convex-hull triangulation, k = 32, degree-2 polynomials", **out}


def cpu_baseline_quad(surf, q_gpu):
    """The FP64 oracle's surface weights for the same surface, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import quadrature as Q
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        q_ref = Q.surface_weights(surf, k=32)
        cpu = time.perf_counter() - t0
    return {"ms": cpu * 1e3, "cores": 1, "kind": "oracle",
            "max_rel_diff_gpu_vs_oracle": float(np.max(np.abs(q_gpu - q_ref)) / np.max(np.abs(q_ref)))}


def probes(P, torch, ctx):
    import ctypes
    L = P.lib()
    out = {}
    grid_threads = torch.cuda.get_device_properties(0).multi_processor_count * 8 * 256
    small = torch.empty(grid_threads * 4 + 256, dtype=torch.uint8, device="cuda")
    for name, which, size in (("fma_lane_ops", 0, 20000), ("fma_vop3_lane_ops", 6, 20000), ("exp_lane_ops", 1, 5000),
                              ("sqrt_lane_ops", 2, 5000), ("fma_exp_mix_lane_ops", 7, 5000),
                              ("mfma_bf16_flops", 5, 20000), ("mfma_f32_flops", 8, 20000),
                              ("mfma_f32_beside_fma_flops", 9, 20000), ("mfma_bf16_beside_fma_flops", 10, 20000),
                              ("mfma_bf16_beside_dot2_flops", 11, 20000), ("mfma_bf16_beside_mask_fma_flops", 12, 20000)):
        best = 0.0
        for _ in range(2):                          # the first launch may run before the clock has ramped
            r = ctypes.c_double()
            P._lib.check(L.nfr_probe(ctx.handle, which, size, small.data_ptr(), small.numel(), ctypes.byref(r)))
            best = max(best, r.value)
        out[name] = best
    nfl = 1 << 30                                   # 4 GiB read, 2 x 2 GiB copy
    big = torch.empty(nfl * 4 + grid_threads * 4 + 256, dtype=torch.uint8, device="cuda")
    for name, which, size in (("hbm_read_Bps", 3, nfl), ("hbm_copy_Bps", 4, nfl // 2)):
        best = 0.0
        for _ in range(3):
            r = ctypes.c_double()
            P._lib.check(L.nfr_probe(ctx.handle, which, size, big.data_ptr(), big.numel(), ctypes.byref(r)))
            best = max(best, r.value)
        out[name] = best
    del big
    return out



def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the path shards by target rows, "
              "see the design notes)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2504_13379_amd as P

    if args.probes_only:
        print(json.dumps({"probes": probes(P, torch, P.Context(0))}), flush=True)
        return
    w, gold, head, forms = ensemble_headline(P, torch, args)
    best = head["form"]
    line = {
        "metric": "kernel pair-interactions/s at stated rel err vs FP64; batched+MFMA vs plain FP32",
        "value": head["value"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": best.replace("otf_", ""),
        "data": "synthetic",
        "config": {"workload": "ellipsoid (1,.8,.6), N=65536, B=64 states, Gauss Mexican hat (1,.15,.5,.4), "
                               "beta=20, theta_b~U(.15,.3), RK4 dt=0.05 x %d steps, FP64 oracle RBF-QF weights"
                               % w.steps,
                   "form": best, "n": w.n, "B": w.b, "rk4_steps": w.steps},
        "rel_linf_vs_fp64": {"max": head["rel_linf_vs_fp64_max"], "per_member": head["rel_linf_vs_fp64"],
                             "rows": "%d sampled rows per member, normalised by max|u(T)| over all rows"
                                     % len(gold["rows"])},
        "roofline": head["roofline"],
        "launches": head["launches"],
        "timed": {"times_ms": head["times_ms"], "ms_all_timed": head["ms_all_timed"],
                  "kernel_avg_ms": head["kernel_avg_ms"]},
        "forms": forms,
    }
    if "otf_fp32" in forms:
        line["vs_plain_fp32"] = head["value"] / forms["otf_fp32"]["value"]
    if not args.no_cpu_baseline:
        print("bench: CPU baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, gold["q"], 1024)
    if not args.no_torus:
        print("bench: torus", file=sys.stderr, flush=True)
        line["torus"] = torus_leg(P, torch, args)
    if not args.no_small:
        print("bench: small sphere", file=sys.stderr, flush=True)
        line["small"] = small_leg(P, torch, args)
    if not args.no_batch:
        print("bench: uneven batch", file=sys.stderr, flush=True)
        line["batch"] = batch_leg(P, torch, args)
    if args.adjoint_rk4_steps > 0:
        print("bench: adjoint", file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_leg(P, torch, args)
    if args.quad_n > 0:
        print("bench: quadrature weights", file=sys.stderr, flush=True)
        line["quadrature"] = quad_leg(P, torch, args)
    if args.probes:
        line["probes"] = probes(P, torch, P.Context(0))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
