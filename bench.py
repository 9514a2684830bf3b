"""Throughput of the neural-field hot path on one MI355X.

Workload (one "step" = one whole integration): torus R = 1, r = 0.4 with
N = 32768 jittered-ring nodes, exponential Mexican hat
w(r) = 2 exp(-r/0.1) - exp(-r/0.3), sigmoid beta = 20, theta = 0.25, two
bumps as u0, classical RK4 with dt = 0.02 for 500 steps (2000 operator
applications of N^2 pairs each).  Inputs are resident on the GPU before the
timed region.  Quadrature weights are the area-share stand-in |D|/N (the
oracle's RBF-QF weights are used by the parity tests; the weight values do not
change the work).

Both evaluation forms run: on-the-fly FP32 pair sums, and precomputed FP32 W
(its build is inside every timed step).  `value` is the faster form's
pair-interactions per second; both forms are listed under "forms".

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


def fused_slots_per_w(kind, m, fp16=False):
    """Slots per W entry of the fused on-the-fly split forms: the evaluation of u
    above (the weights sit in G), and 3 for the hi/lo split (two conversions of a pair of entries at half a slot each, the hi value
    back to FP32, the subtraction); FP16 adds the lift of u (its 2^11 remainder
    scaling fuses into the subtraction)."""
    return eval_slots(kind, m) + 3 + (1 if fp16 else 0)


def sym_kernel_name(kind, m, periodic=False):
    return "k_otf_sym<%d>" % (kind + (2 if periodic else 0) + ((m - 1) << 2 if m else 0))


# Sources that define the profiled kernels (their code and tile constants).
TRAFFIC_SOURCES = ("common.h", "kernels_core.h", "kernels_mfma.h")


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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rk4-steps", type=int, default=500)
    ap.add_argument("--forms", default="otf,w32")
    ap.add_argument("--no-graph", action="store_true", help="launch every kernel instead of replaying graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the N = 2000 sphere time-per-step leg")
    ap.add_argument("--probes", action="store_true", help="also run the roofline microbenchmarks")
    ap.add_argument("--probes-only", action="store_true",
                    help="run only the roofline microbenchmarks and print their rates as one JSON line")
    ap.add_argument("--ens-rk4-steps", type=int, default=10,
                    help="RK4 steps of the ellipsoid-ensemble comparison leg (0 = skip it)")
    ap.add_argument("--batch-rk4-steps", type=int, default=20,
                    help="RK4 steps of the 48-problem uneven-batch leg (0 = skip it)")
    ap.add_argument("--adjoint-rk4-steps", type=int, default=400,
                    help="RK4 steps of the torus adjoint leg (0 = skip it)")
    ap.add_argument("--quad-n", type=int, default=65536,
                    help="nodes of the surface-quadrature leg on the ellipsoid (0 = skip it)")
    return ap.parse_args()


def run_form(P, torch, prob, w, q_t, form, args, u0_t):
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    L = P.lib()
    ctx = prob.ctx
    u = torch.empty_like(u0_t)
    ws = prob.integrate_workspace(1, form)
    wbytes = L.nfr_w_bytes(w.n, form) if form != P.FORM_ONTHEFLY_FP32 else 0
    Wbuf = None
    if wbytes:
        from paper_2504_13379_amd.api import _dev_buffer
        Wbuf = _dev_buffer(wbytes, ctx.device)

    def one():
        u.copy_(u0_t)
        if Wbuf is not None:
            P._lib.check(L.nfr_w_build(prob.handle, __import__("ctypes").byref(k), form, Wbuf.data_ptr(), wbytes))
        prob.integrate(k, f, u, w.dt, args.rk4_steps, form=form, W=Wbuf, ws=ws, use_graph=not args.no_graph)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    import ctypes
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # dominant-kernel duration: HIP events around every pair-sum launch of one
    # more integration (events are not recorded inside replayed graphs)
    L.nfr_context_set_timing(ctx.handle, 1)
    u.copy_(u0_t)
    prob.integrate(k, f, u, w.dt, args.rk4_steps, form=form, W=Wbuf, ws=ws, use_graph=False)
    launches = ctypes.c_int64()
    tot_ms = ctypes.c_double()
    P._lib.check(L.nfr_context_timing(ctx.handle, ctypes.byref(launches), ctypes.byref(tot_ms)))
    L.nfr_context_set_timing(ctx.handle, 0)
    sec = (t1 - t0) / args.steps
    pairs = 4.0 * args.rk4_steps * float(w.n) ** 2
    return {
        "ms_per_step": sec * 1e3,
        "value": pairs / sec,
        "kernel_launches": int(launches.value),
        "kernel_avg_ms": tot_ms.value / max(1, launches.value),
        "u": u,
    }


def roofline(form_name, res, n, npad, kernel):
    avg_s = res["kernel_avg_ms"] * 1e-3
    if form_name == "w32":
        bytes_per_launch = float(n) * npad * 4.0          # every W element once per application
        ach = bytes_per_launch / avg_s
        return {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ach / HBM_PEAK, "traffic": measured_traffic("k_w_gemv_f32<1>"), "kernel": "k_w_gemv_f32<1>"}
    # on-the-fly: slots per unordered pair x npad^2 / 2 pairs per launch
    kind, s_e, s_i = kernel[0], kernel[2], kernel[4]
    m = sym_pow(kind, s_e, s_i)
    name = sym_kernel_name(kind, m)
    ops = slots_per_unordered_pair(kind, m) * float(npad) * npad / 2.0
    ach = ops / avg_s
    return {"bound": "alu", "achieved": ach / 1e12, "peak": VALU_LANES_PER_S / 1e12, "unit": "Tlane-op/s",
            "frac": ach / VALU_LANES_PER_S, "traffic": measured_traffic(name), "kernel": name,
            "slots_per_unordered_pair": slots_per_unordered_pair(kind, m)}


def ensemble_leg(P, torch, args):
    """Ellipsoid (1, .8, .6), N = 65536, B = 64 Gaussian-kernel ensemble: the split-precision
    MFMA W forms against the plain FP32 on-the-fly path on the same GPU."""
    import ctypes

    from workloads import configs as C
    w = C.ellipsoid_ensemble(65536, 64, steps=args.ens_rk4_steps)
    q = C.area_share_weights(w.surface)
    ctx = P.Context(0)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    L = P.lib()
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, torch.from_numpy(w.theta).cuda())
    u0 = torch.from_numpy(w.u0.copy()).cuda()
    out = {"workload": "ellipsoid (1,.8,.6), N=65536, B=64, Gauss Mexican hat, RK4 dt=0.05 x %d steps"
                       % args.ens_rk4_steps}
    finals = {}
    for nm, form in (("bf16x3", P.FORM_W_BF16X3), ("fp16x3", P.FORM_W_FP16X3), ("otf_bf16x3", P.FORM_ONTHEFLY_BF16X3),
                     ("otf_fp16x3", P.FORM_ONTHEFLY_FP16X3), ("otf_fp32_mfma", P.FORM_ONTHEFLY_FP32_MFMA),
                     ("otf_fp32", P.FORM_ONTHEFLY_FP32)):
        print("bench: ensemble form %s" % nm, file=sys.stderr, flush=True)
        W = None
        t_build = 0.0
        if form in (P.FORM_W_BF16X3, P.FORM_W_FP16X3):
            torch.cuda.synchronize()
            tb = time.perf_counter()
            W = prob.w_build(k, form)
            torch.cuda.synchronize()
            t_build = time.perf_counter() - tb
        ws = prob.integrate_workspace(64, form)
        u = u0.clone()
        prob.integrate(k, f, u, w.dt, 1, form=form, W=W, ws=ws)          # warm-up
        u.copy_(u0)
        torch.cuda.synchronize()
        L.nfr_context_set_timing(ctx.handle, 1)
        t0 = time.perf_counter()
        prob.integrate(k, f, u, w.dt, args.ens_rk4_steps, form=form, W=W, ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        launches, tot = ctypes.c_int64(), ctypes.c_double()
        P._lib.check(L.nfr_context_timing(ctx.handle, ctypes.byref(launches), ctypes.byref(tot)))
        L.nfr_context_set_timing(ctx.handle, 0)
        pairs = 4.0 * args.ens_rk4_steps * float(w.n) ** 2 * 64
        avg = tot.value / max(1, launches.value) * 1e-3
        entry = {"value": pairs / (t1 - t0), "unit": "pair-interactions/s", "ms_per_integration": (t1 - t0) * 1e3,
                 "w_build_ms": t_build * 1e3, "kernel_avg_ms": avg * 1e3}
        if W is not None:
            wbytes = 2.0 * 2 * prob.npad * prob.npad     # hi + lo, 2 bytes each, every element once
            kname = "k_mfma_apply<%s,2>" % ("bf16" if nm == "bf16x3" else "fp16")
            entry["roofline"] = {"bound": "hbm", "achieved": wbytes / avg / 1e9, "peak": HBM_PEAK / 1e9,
                                 "unit": "GB/s", "frac": wbytes / avg / HBM_PEAK,
                                 "traffic": measured_traffic(kname), "kernel": kname}
        elif form == P.FORM_ONTHEFLY_FP32_MFMA:
            # products on the FP32 matrix cores: 2 flop per pair-interaction (64 states, each
            # kernel value once per launch on the vector units)
            m = sym_pow(w.kernel_kind, w.kernel[1], w.kernel[3])
            kname = "k_mfma_otf_f32<%d,2>" % (w.kernel_kind + 4 * (m - 1 if m else 0))
            flops = 2.0 * float(prob.npad) ** 2 * 64
            entry["roofline"] = {"bound": "mfma", "achieved": flops / avg / 1e12, "peak": MFMA_F32_PEAK / 1e12,
                                 "unit": "TFLOP/s", "frac": flops / avg / MFMA_F32_PEAK,
                                 "traffic": measured_traffic(kname), "kernel": kname,
                                 "alu_frac": float(prob.npad) ** 2 * eval_slots(w.kernel_kind, m) / avg / VALU_LANES_PER_S}
        elif form == P.FORM_ONTHEFLY_FP32:
            # one-sided multi-state pair sum: per target-source pair one evaluation of u per
            # block of 16 states (no integer-ratio shortcut in this kernel) + 1 FMA per state
            kname = "k_otf_pair_sum<%d,2,16>" % w.kernel_kind
            slots = float(prob.npad) ** 2 * (-(-64 // 16) * eval_slots(w.kernel_kind, 0) + 64)
            entry["roofline"] = {"bound": "alu", "achieved": slots / avg / 1e12, "peak": VALU_LANES_PER_S / 1e12,
                                 "unit": "Tslot/s", "frac": slots / avg / VALU_LANES_PER_S,
                                 "traffic": measured_traffic(kname), "kernel": kname}
        elif form in (P.FORM_ONTHEFLY_BF16X3, P.FORM_ONTHEFLY_FP16X3):
            # every W entry evaluated once per launch (64 states share it) on the vector
            # units; the matrix cores do 3 products x 2 flops x 64 states per entry
            m = sym_pow(w.kernel_kind, w.kernel[1], w.kernel[3])
            wvals = float(prob.npad) ** 2
            kname = "k_mfma_otf<%s,%d,2>" % ("bf16" if nm == "otf_bf16x3" else "fp16",
                                             w.kernel_kind + 4 * (m - 1 if m else 0))
            fp16 = nm == "otf_fp16x3"
            achieved = wvals * fused_slots_per_w(w.kernel_kind, m, fp16) / avg
            entry["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_LANES_PER_S / 1e12,
                                 "unit": "Tslot/s", "frac": achieved / VALU_LANES_PER_S,
                                 "traffic": measured_traffic(kname), "kernel": kname,
                                 "slots_per_w": fused_slots_per_w(w.kernel_kind, m, fp16),
                                 "mfma_tflops": wvals * 384.0 / avg / 1e12,
                                 "mfma_frac": wvals * 384.0 / avg / MFMA_BF16_PEAK}
        out[nm] = entry
        finals[nm] = u.cpu().numpy()
        del W
        torch.cuda.empty_cache()
    import numpy as np
    ref = finals["otf_fp32"]
    for nm in ("bf16x3", "fp16x3", "otf_bf16x3", "otf_fp16x3", "otf_fp32_mfma"):
        out[nm]["max_rel_linf_vs_otf_fp32"] = float(np.max(np.max(np.abs(finals[nm] - ref), axis=1) /
                                                            np.max(np.abs(ref), axis=1)))
    return out


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


def batch_leg(P, torch, args):
    """The 48-problem uneven batch (N log-uniform in [1000, 40000], B in {1, 4, 16}):
    tuned persistent launches with graph-captured steps."""
    import ctypes

    from workloads import configs as C
    ws_list = C.uneven_batch(steps=args.batch_rk4_steps)
    stream = torch.cuda.Stream()
    ctx = P.Context(0, stream)
    probs, ks, fs, Bs, u0s = [], [], [], [], []
    with torch.cuda.stream(stream):
        for w in ws_list:
            q = C.area_share_weights(w.surface)
            probs.append(P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda()))
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
    batch.integrate(states, 0.05, 1, use_graph=True, ws=ws)       # warm-up
    for s_, u in zip(states, u0s):
        s_.copy_(u)
    torch.cuda.synchronize()
    L = P.lib()
    t0 = time.perf_counter()
    batch.integrate(states, 0.05, args.batch_rk4_steps, use_graph=True, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pair_ints = sum(4.0 * args.batch_rk4_steps * float(w.n) ** 2 * w.b for w in ws_list)
    # algorithmic slots of the (one-sided) pair kernel per stage: per target-source pair and
    # state block one evaluation of u (eval_slots: 16 for the Gaussian), plus 1 FMA per
    # state; blocks of 1, 4 or 16 states
    slots = 0.0
    for w in ws_list:
        npad = -(-w.n // 256) * 256
        bs = 1 if w.b == 1 else (4 if w.b <= 4 else 16)
        slots += float(npad) ** 2 * (-(-w.b // bs) * eval_slots(0, 0) + w.b)
    slots *= 4.0 * args.batch_rk4_steps
    chunk, wgs = batch.config
    return {"workload": "48 problems, N log-uniform [1000, 40000], sphere/torus/ellipsoid/bumpy, Gauss Mexican hat, "
                        "B in {1,4,16}, RK4 dt=0.05 x %d steps, graph-captured" % args.batch_rk4_steps,
            "value": pair_ints / (t1 - t0), "unit": "pair-interactions/s", "ms_per_integration": (t1 - t0) * 1e3,
            "roofline": {"bound": "alu", "achieved": slots / (t1 - t0) / 1e12, "peak": VALU_LANES_PER_S / 1e12,
                         "unit": "Tlane-op/s", "frac": slots / (t1 - t0) / VALU_LANES_PER_S,
                         "note": "whole integration time (pair kernel, combine, launch gaps)"},
            "tuned": {"chunk": chunk, "wgs_per_cu": wgs, "best_stage_ms": best, "tune_ms": t_tune * 1e3},
            "launches_per_rk4_step": 1}


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
    # four-channel symmetric transpose kernel (rho t multiply kept, e1 = e2^m, e*t products, 8 FMAs)
    npad = -(-w.n // 256) * 256
    m = sym_pow(w.kernel_kind, w.kernel[1], w.kernel[3])
    trans = (2 if w.kernel_kind == 0 else 3) - (1 if m else 0)
    adj_slots = 7 + trans * TRANS_COST + (0 if not m else (1 if m == 2 else 2)) + 2 + 8
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


def cpu_baseline(w, q, gpu_y_rows, rows):
    """The FP64 oracle's operator on a bounded sample: all sources, a subset of target rows."""
    from threadpoolctl import threadpool_limits

    from oracle import neural_field as NF
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ref = NF.apply_K(w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows=rows)
        t1 = time.perf_counter()
    import numpy as np
    err = float(np.max(np.abs(gpu_y_rows - ref)) / np.max(np.abs(ref)))
    return {"value": float(len(rows)) * w.n / (t1 - t0), "unit": "pair-interactions/s", "cores": 1,
            "kind": "oracle",
            "sample": "one operator application, %d of %d target rows x all %d sources, FP64 NumPy, 1 thread"
                      % (len(rows), w.n, w.n)}, err


def probes(P, torch, ctx):
    import ctypes
    L = P.lib()
    out = {}
    grid_threads = torch.cuda.get_device_properties(0).multi_processor_count * 8 * 256
    small = torch.empty(grid_threads * 4 + 256, dtype=torch.uint8, device="cuda")
    for name, which, size in (("fma_lane_ops", 0, 20000), ("fma_vop3_lane_ops", 6, 20000), ("exp_lane_ops", 1, 5000),
                              ("sqrt_lane_ops", 2, 5000), ("fma_exp_mix_lane_ops", 7, 5000),
                              ("mfma_bf16_flops", 5, 20000), ("mfma_f32_flops", 8, 20000),
                              ("mfma_f32_beside_fma_flops", 9, 20000), ("mfma_bf16_beside_fma_flops", 10, 20000)):
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
    import numpy as np
    import torch

    import paper_2504_13379_amd as P
    from workloads import configs as C

    if args.probes_only:
        print(json.dumps({"probes": probes(P, torch, P.Context(0))}), flush=True)
        return
    w = C.torus_exp(32768, steps=args.rk4_steps)
    q = C.area_share_weights(w.surface)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = P.Context(0, stream)
    xyz_t = torch.from_numpy(w.surface.xyz).cuda()
    q_t = torch.from_numpy(q).cuda()
    prob = P.Problem(ctx, xyz_t, q_t)
    u0_t = torch.from_numpy(w.u0.copy()).cuda()
    torch.cuda.synchronize()

    names = {"otf": P.FORM_ONTHEFLY_FP32, "w32": P.FORM_W_FP32}
    results = {}
    for nm in args.forms.split(","):
        print("bench: form %s, %d warmup + %d timed integrations of %d RK4 steps" % (nm, args.warmup, args.steps,
              args.rk4_steps), file=sys.stderr, flush=True)
        results[nm] = run_form(P, torch, prob, w, q_t, names[nm], args, u0_t)
        print("bench: form %s %.3f ms/step" % (nm, results[nm]["ms_per_step"]), file=sys.stderr, flush=True)
    best = max(results, key=lambda k: results[k]["value"])
    r = results[best]
    kern = (w.kernel_kind,) + tuple(w.kernel)
    rl = roofline(best, r, w.n, prob.npad, kern)

    forms = {}
    for nm, rr in results.items():
        rlf = roofline(nm, rr, w.n, prob.npad, kern)
        forms[nm] = {"value": rr["value"], "ms_per_step": rr["ms_per_step"], "kernel_avg_ms": rr["kernel_avg_ms"],
                     "roofline_frac": rlf["frac"]}
    if len(results) == 2:
        ua, ub = results["otf"]["u"].cpu().numpy(), results["w32"]["u"].cpu().numpy()
        forms["otf_vs_w32_rel_linf"] = float(np.max(np.abs(ua - ub)) / np.max(np.abs(ub)))

    line = {
        "metric": "kernel pair-interactions/s (RK4 integration, FP32 pair sums, FP64 state)",
        "value": r["value"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "torus R=1 r=0.4, N=32768, exp Mexican hat, B=1, RK4 dt=0.02 x %d steps"
                               % args.rk4_steps, "form": best, "n": w.n, "B": 1},
        "roofline": rl,
        "forms": forms,
    }
    if not args.no_cpu_baseline:
        rows = np.random.default_rng(7).choice(w.n, 12288, replace=False)
        y = prob.apply(P.kernel_struct(w.kernel_kind, *w.kernel), P.Firing(w.beta, float(w.theta[0])), u0_t)
        torch.cuda.synchronize()
        cb, err = cpu_baseline(w, q, y.cpu().numpy()[:, rows], rows)
        line["cpu_baseline"] = cb
        line["rel_err_vs_fp64_sampled_apply"] = err
    if not args.no_small:
        print("bench: small sphere", file=sys.stderr, flush=True)
        line["small"] = small_leg(P, torch, args)
    if args.ens_rk4_steps > 0:
        line["ensemble"] = ensemble_leg(P, torch, args)
    if args.batch_rk4_steps > 0:
        print("bench: uneven batch", file=sys.stderr, flush=True)
        line["batch"] = batch_leg(P, torch, args)
    if args.adjoint_rk4_steps > 0:
        print("bench: adjoint", file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_leg(P, torch, args)
    if args.quad_n > 0:
        print("bench: quadrature weights", file=sys.stderr, flush=True)
        line["quadrature"] = quad_leg(P, torch, args)
    if args.probes:
        line["probes"] = probes(P, torch, ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
