"""Throughput of the TENO10-AA Euler step on one MI355X.

Workload: 3D Euler on a 256^3 periodic grid (gamma = 1.4), Gaussian-random-field
state with a high-pressure blast sphere and a near-vacuum cavity, TENO10-AA
with LLF splitting and the positivity limiter, one SSP-RK3 step at CFL 0.4
per timed step (dt recomputed on the device every step).  Input is resident in
HBM before timing starts.

Prints one JSON line.  `value` is face reconstructions per second
(one face of one sweep direction, all five characteristic fields, both split
sides): 3 stages x 3 directions x 256^3 per step.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gface-recon/s (RHS) FP64 3D 256^3 TENO-AA10 fwd & fwd+adj; % of FP64/HBM roofline"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
PEAK_HBM_GBS = 8000.0


# HBM traffic of the dominant sweep, measured with rocprofv3 counters and
# calibrated against a plain copy kernel; valid only for the kernel sources
# it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep_x_3d_256_teno10.json")
KERNEL_SOURCES = ["tenoaa_stencil.h", "tenoaa_device.h", "tenoaa_sos.h", "tenoaa_kernels.hip", "tenoaa_internal.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2109_14340_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """Bytes per launch of `kernel` from the committed counter summary, or
    None if there is none for the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("kernel_class") != kernel:
        return None
    return t.get("traffic_bytes")


def cpu_baseline(n=72):
    """The oracle, single-threaded, on one step of the same recipe at n^3."""
    import numpy as np  # noqa: F401
    import oracle
    from paper_2109_14340_amd import inputs

    oracle.lib()
    U = inputs.blast_cavity_3d(n)
    g = oracle.make_grid((n, n, n), [1.0 / n] * 3, [0, 0, 0])
    t = time.perf_counter()
    oracle.step(g, U, order=10, splitting=0, positivity=1, gamma=1.4, cfl=0.4)
    el = time.perf_counter() - t
    work = 9 * n ** 3
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": work / el / 1e9, "unit": "Gface-recon/s", "cores": 1, "kind": "oracle",
            "sample": "one SSP-RK3 step (TENO10-AA, LLF, limiter, CFL 0.4) of the same recipe on a "
                      "%d^3 periodic grid: %d face reconstructions in %.2f s, one thread of %s (%d visible "
                      "cores)" % (n, work, el, model, os.cpu_count() or 0),
            "legs": cpu_legs()}


def cpu_legs():
    """The oracle on the other workloads (bounded samples), single-threaded:
    the 1D shock tube (100 steps at N = 256, TENO8-AA, outflow: the whole
    workload), one 2D right-hand side with TENO8-AA and with TENO10-AA on a
    512^2 sample of the 1024^2 recipe, and the forward-mode step derivative
    (the oracle's adjoint check) of one TENO10-AA step on a 256^2 sample of
    the 512^2 adjoint recipe."""
    import numpy as np
    import oracle
    from paper_2109_14340_amd import inputs

    out = {}
    U = inputs.shock_tube_1d(256)
    g = oracle.make_grid((256,), [1.0 / 256], [1], [1])
    t = time.perf_counter()
    for _ in range(100):
        U, _, _, _ = oracle.step(g, U, order=8, splitting=0, cfl=0.4)
    el = time.perf_counter() - t
    out["1d_256_teno8_100_steps"] = {"s": round(el, 3), "value": 3 * 257 * 100 / el / 1e9, "unit": "Gface-recon/s"}
    n = 512
    U = inputs.grf_2d(1024)[:, :, :n, :n].copy()
    g = oracle.make_grid((n, n), [1.0 / 1024] * 2, [0, 0])
    for order in (8, 10):
        t = time.perf_counter()
        oracle.rhs(g, U, order=order, splitting=0, want_flags=False)
        el = time.perf_counter() - t
        out["2d_%d_sample_rhs_teno%d" % (n, order)] = {"s": round(el, 3), "value": 2 * n * n / el / 1e9,
                                                       "unit": "Gface-recon/s"}
    n = 256
    U = inputs.grf_2d(512, jump=False)[:, :, :n, :n].copy()
    g = oracle.make_grid((n, n), [1.0 / 512] * 2, [0, 0])
    _, dt, fl3, _ = oracle.step(g, U, order=10, splitting=0, cfl=0.4, want_flags=True)
    V = np.random.default_rng(0).standard_normal(U.shape)
    t = time.perf_counter()
    oracle.step_jvp(g, U, V, dt, fl3, order=10, splitting=0)
    el = time.perf_counter() - t
    out["2d_%d_sample_step_jvp_teno10" % n] = {"s": round(el, 3), "value": 3 * 2 * n * n / el / 1e9,
                                               "unit": "Gface-recon/s"}
    return out


def gpu_legs(dev):
    """The other workloads on the GPU: the 1D shock tube (100 steps at
    N = 256, TENO8-AA, outflow) and one 2D 1024^2 right-hand side with
    TENO8-AA and with TENO10-AA (periodic)."""
    import torch

    from paper_2109_14340_amd import inputs, tenoaa

    out = {}
    grid = tenoaa.make_grid((256,), bc_lo=[tenoaa.BC_OUTFLOW], bc_hi=[tenoaa.BC_OUTFLOW])
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    U0 = torch.from_numpy(inputs.shock_tube_1d(256)).to(dev)
    ws = tenoaa.workspace(grid, sch, tenoaa.WS_STEP, dev)
    dts = torch.zeros(100, dtype=torch.float64, device=dev)
    for rep_ in range(2):
        U = U0.clone()
        dts.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(100):
            tenoaa.step(grid, sch, U, dts[k:k + 1], cfl=0.4, ws=ws)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
    out["1d_256_teno8_100_steps"] = {"ms": round(el * 1e3, 3), "value": 3 * 257 * 100 / el / 1e9,
                                     "unit": "Gface-recon/s", "note": "launch-bound: 1,542 faces per sweep"}
    n = 1024
    U = torch.from_numpy(inputs.grf_2d(n)).to(dev)
    grid = tenoaa.make_grid((n, n))
    for order in (8, 10):
        sch = tenoaa.make_scheme(order, tenoaa.LLF, 0)
        ws = tenoaa.workspace(grid, sch, tenoaa.WS_RHS, dev)
        out_t = torch.empty_like(U)
        for _ in range(2):
            tenoaa.rhs(grid, sch, U, out=out_t, ws=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            tenoaa.rhs(grid, sch, U, out=out_t, ws=ws)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / 10
        out["2d_1024_rhs_teno%d" % order] = {"ms": round(el * 1e3, 4), "value": 2 * n * n / el / 1e9,
                                              "unit": "Gface-recon/s"}
    return out


def fwd_adj_leg(shape, steps, warmup, U0, positivity):
    """Forward step plus its adjoint (tenoaa_step_vjp, which recomputes the
    stages) on one state, TENO10-AA, LLF, dt from CFL 0.4 then frozen for the
    adjoint.  With positivity 1 the limiter acts in both, its factors frozen
    in the adjoint like the other decisions."""
    import torch

    from paper_2109_14340_amd import tenoaa

    dev = U0.device
    grid = tenoaa.make_grid(shape)
    sch = tenoaa.make_scheme(10, tenoaa.LLF, positivity)
    ws = tenoaa.workspace(grid, sch, tenoaa.WS_STEP, dev)
    wsv = tenoaa.workspace(grid, sch, tenoaa.WS_STEP_VJP, dev)
    U = U0.clone()
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    bar = torch.randn(U.shape, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(14340))
    out = torch.empty_like(bar)

    def fwd():
        U.copy_(U0)
        dt.zero_()
        tenoaa.step(grid, sch, U, dt, gamma=1.4, cfl=0.4, ws=ws)

    def adj():
        tenoaa.step_vjp(grid, sch, U0, dt, bar, gamma=1.4, out=out, ws=wsv)

    # the taped pair: the step keeps its stage states and records (one
    # TENOAA_WS_STEP_TAPE workspace), the adjoint runs only the reverse sweeps
    wst = tenoaa.workspace(grid, sch, tenoaa.WS_STEP_TAPE, dev)
    dtt = torch.zeros(1, dtype=torch.float64, device=dev)
    Ut = torch.empty_like(U0)

    def fwd_tape():
        dtt.zero_()
        tenoaa.step_tape(grid, sch, U0, dtt, gamma=1.4, cfl=0.4, out=Ut, ws=wst)

    def adj_tape():
        tenoaa.step_vjp_tape(grid, sch, U0, dtt, bar, wst, gamma=1.4, out=out)

    res = {}
    for name, fn in (("fwd", fwd), ("adj", adj), ("fwd_tape", fwd_tape), ("adj_tape", adj_tape)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / steps * 1e3
    work = 3 * len(shape) * U0[0].numel()
    return {"grid": list(shape), "limiter": bool(positivity), "fwd_ms": round(res["fwd"], 3), "adj_ms": round(res["adj"], 3),
            "adj_over_fwd": round(res["adj"] / res["fwd"], 3),
            "value": round(work / ((res["fwd"] + res["adj"]) * 1e-3) / 1e9, 4), "unit": "Gface-recon/s",
            "note": "face reconstructions of the forward step / (step + step VJP time); the forward "
                    "copy of the input state is inside fwd_ms",
            "tape": {"fwd_ms": round(res["fwd_tape"], 3), "adj_ms": round(res["adj_tape"], 3),
                     "value": round(work / ((res["fwd_tape"] + res["adj_tape"]) * 1e-3) / 1e9, 4),
                     "workspace_bytes": int(wst.numel()),
                     "note": "tenoaa_step_tape (the step keeping its stage states and records) + "
                             "tenoaa_step_vjp_tape (reverse sweeps only), bit-identical to the pair above"}}


def slab_leg(U0, pieces=8, steps=5, warmup=1):
    """One GPU's share of the same workload split into `pieces` z-slabs: each
    slab is a grid n x n x n/pieces whose z sides are halo sides holding the
    neighbour slabs' 5 cells next to the cut.  A split step is: halo refresh,
    wave speeds per slab and their maximum, then per stage a halo refresh and
    tenoaa_rk3_stage on every slab.  Checked once, untimed: the slabs' step
    equals tenoaa_step on the whole grid bit for bit.  Timed: one slab's
    share of a step (speeds + three stages) with its halos in place; the halo
    exchanges and the maximum over GPUs are the communication a multi-GPU
    run adds, reported as bytes."""
    import torch

    from paper_2109_14340_amd import tenoaa

    dev = U0.device
    n = U0.shape[-1]
    nz = n // pieces
    G = 5
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    spans = [(k * nz, (k + 1) * nz) for k in range(pieces)]

    def halos(full, lo, hi):
        out = {}
        for side in (0, 1):
            idx = [(lo - r) % n if side == 0 else (hi - 1 + r) % n for r in range(1, G + 1)]
            out[(2, side)] = full[:, idx].permute(1, 0, 2, 3).reshape(1, G, 5, n * n).contiguous()
        return out

    grids = [tenoaa.make_grid((n, n, nz), [1.0 / n] * 3, [0, 0, tenoaa.BC_HALO], [0, 0, tenoaa.BC_HALO],
                              bc_values=halos(U0, lo, hi)) for lo, hi in spans]
    wss = [tenoaa.workspace(g, sch, tenoaa.WS_RHS, dev) for g in grids]

    def exchange(states):
        full = torch.cat(states, dim=1)
        for (lo, hi), g in zip(spans, grids):
            for key, v in halos(full, lo, hi).items():
                g._faces[key].copy_(v)

    def split_step(slabs, stage_states, dt):
        exchange(slabs)
        amax = torch.stack([tenoaa.wave_speeds(g, sch, u, ws=w) for g, u, w in zip(grids, slabs, wss)])
        amax = amax.max(dim=0).values.contiguous()
        dt.zero_()
        for stage in (1, 2, 3):
            if stage > 1:
                exchange(stage_states)
            for k in range(pieces):
                tenoaa.rk3_stage(grids[k], sch, stage, amax, dt, slabs[k], None if stage == 1 else stage_states[k],
                                 slabs[k] if stage == 3 else stage_states[k], ws=wss[k])

    # bitwise check of the split step against the whole grid's
    slabs = [U0[:, lo:hi].contiguous() for lo, hi in spans]
    stage_states = [torch.empty_like(u) for u in slabs]
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    split_step(slabs, stage_states, dt)
    whole = U0.clone()
    dtw = torch.zeros(1, dtype=torch.float64, device=dev)
    g_whole = tenoaa.make_grid((n, n, n))
    tenoaa.step(g_whole, sch, whole, dtw)
    equal = bool(torch.equal(torch.cat(slabs, dim=1), whole)) and float(dt.item()) == float(dtw.item())
    del whole, stage_states

    # one slab's share, timed (halos of U0 in place, the speeds of the whole step)
    g0, w0 = grids[0], wss[0]
    exchange([U0[:, lo:hi].contiguous() for lo, hi in spans])
    u = U0[:, :nz].contiguous()
    us = torch.empty_like(u)
    amax = torch.stack([tenoaa.wave_speeds(g, sch, U0[:, lo:hi].contiguous(), ws=w)
                        for g, (lo, hi), w in zip(grids, spans, wss)]).max(dim=0).values.contiguous()

    def share():
        u.copy_(U0[:, :nz])
        tenoaa.wave_speeds(g0, sch, u, ws=w0)
        dt.zero_()
        for stage in (1, 2, 3):
            tenoaa.rk3_stage(g0, sch, stage, amax, dt, u, None if stage == 1 else us, u if stage == 3 else us, ws=w0)

    for _ in range(warmup):
        share()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        share()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    if any(tenoaa.get_status(w) != 0 for w in wss):
        raise RuntimeError("non-physical state in the split step")
    work = 9 * n * n * nz
    return {"grid": [n, n, nz], "pieces": pieces, "ms_per_step": round(ms, 3),
            "value": round(work / (ms * 1e-3) / 1e9, 4), "unit": "Gface-recon/s",
            "halo_bytes_per_stage": 2 * G * 5 * n * n * 8,
            "split_step_bitwise_equal_to_whole_grid": equal,
            "note": "one slab's share of a step (wave speeds + three stages, the state copy inside); halo "
                    "exchanges and the maximum of the speeds over the slabs excluded"}


def batched_leg(nprob=512, nsteps=20, tune_cache=None, compare=True):
    """The batched workload: nprob 2D problems with n_x, n_y ~ U{64..512},
    TENO8-AA, LLF, outflow, nsteps SSP-RK3 steps each with its own dt, in one
    persistent graph launch; against the same steps launched per problem
    unless compare is False."""
    import tempfile

    import torch

    from paper_2109_14340_amd import flops, inputs, tenoaa

    sizes = inputs.batch_sizes(nprob)
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    bc = [tenoaa.BC_OUTFLOW, tenoaa.BC_OUTFLOW]
    grids = [tenoaa.make_grid((nx, ny), bc_lo=bc, bc_hi=bc) for nx, ny in sizes]
    states = [inputs.riemann_2d(nx, ny, p) for p, (nx, ny) in enumerate(sizes)]
    faces = sum((nx + 1) * ny + (ny + 1) * nx for nx, ny in sizes) * 3 * nsteps
    path = tune_cache or os.path.join(tempfile.mkdtemp(prefix="tenoaa_tune_"), "tune.jsonl")
    t0 = time.perf_counter()
    plan = tenoaa.BatchPlan(grids, sch, nsteps, tune_cache=path)
    t_plan = time.perf_counter() - t0
    packed0 = plan.pack(states)
    packed = packed0.clone()
    dtb = torch.zeros(nprob * nsteps, dtype=torch.float64, device="cuda")
    plan.run(packed, dtb)  # warm-up
    reps = 3
    times = []
    ev_ms = []
    for _ in range(reps):
        packed.copy_(packed0)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        t0 = time.perf_counter()
        ev[0].record()
        plan.run(packed, dtb)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ev_ms.append(ev[0].elapsed_time(ev[1]))
    if any(plan.status()):
        raise RuntimeError("non-physical state in the batched run")
    stats = plan.run_stats()
    t_batch = min(times)
    # the run is one graph launch (a clearing kernel and the persistent
    # kernel) on torch's current stream; its event duration is the kernel's
    kernel_ms = min(ev_ms)
    face_flops = flops.smooth_face_flops(2, 8, 0, False)
    fl_total = face_flops * faces
    achieved = fl_total / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None, "kernel": "batch_kernel",
                "kernel_avg_ms": round(kernel_ms, 3), "algorithmic_flops_per_launch": fl_total,
                "flop_model": "every reconstruction on the largest stencil (%d flop per face): a lower "
                              "bound of the work, which the deeper cascade paths raise" % face_flops}
    res = {"problems": nprob, "steps": nsteps, "cells": sum(nx * ny for nx, ny in sizes),
           "face_recons": faces, "batched_ms": round(t_batch * 1e3, 2),
           "value": round(faces / t_batch / 1e9, 4), "unit": "Gface-recon/s",
           "barrier_wait_share": round(stats["barrier_wait_share"], 4),
           "wait_per_barrier_us": round(stats["wait_per_barrier_us"], 2),
           "sweep_item_share": round(stats["sweep_share"], 4), "cell_item_share": round(stats["cell_share"], 4)}
    if not compare:
        res.update({"plan": plan.info(), "plan_create_s": round(t_plan, 3), "roofline": roofline})
        return res

    # per problem: the same steps through tenoaa_step, one problem after another;
    # a plain pass for the wall time, then a pass with per-kernel events
    wss = [tenoaa.workspace(g, sch, tenoaa.WS_STEP) for g in grids]
    dts = torch.zeros(nprob * nsteps, dtype=torch.float64, device="cuda")

    def per_problem():
        Us = [plan.unpack(packed0, p).clone() for p in range(nprob)]
        dts.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in range(nprob):
            for n in range(nsteps):
                tenoaa.step(grids[p], sch, Us[p], dts[p * nsteps + n:p * nsteps + n + 1], cfl=0.4, ws=wss[p])
        torch.cuda.synchronize()
        return Us, time.perf_counter() - t0

    per_problem()  # warm-up
    Us, t_pp = per_problem()
    tenoaa.timing_enable(True)
    per_problem()
    ksum = 0.0
    for k in range(8):
        ksum += tenoaa.timing_read(k)[1]
    tenoaa.timing_enable(False)
    same = all(torch.equal(plan.unpack(packed, p), Us[p]) for p in range(nprob)) and torch.equal(dts, dtb)
    res.update({"per_problem_wall_ms": round(t_pp * 1e3, 2), "per_problem_kernel_sum_ms": round(ksum, 2),
                "speedup_vs_wall": round(t_pp / t_batch, 3), "speedup_vs_kernel_sum": round(ksum / 1e3 / t_batch, 3),
                "bitwise_equal_to_per_problem": bool(same), "plan": plan.info(), "plan_create_s": round(t_plan, 3),
                "roofline": roofline})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwd-adj", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-slab", action="store_true")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain copy of the state (a kernel of known traffic) for counter runs")
    ap.add_argument("--only", choices=["batched", "fwd_adj"], default=None,
                    help="run one side leg alone and print its object (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2109_14340_amd import flops, inputs, tenoaa

    n = args.n
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.only == "batched":
        print(json.dumps({"batched": batched_leg(tune_cache=args.tune_cache, compare=False)}), flush=True)
        return
    if args.only == "fwd_adj":
        U3 = torch.from_numpy(inputs.grf_3d(n)).to(dev)
        print(json.dumps({"fwd_adj": {"3d": fwd_adj_leg((n, n, n), 1, 1, U3, 1)}}), flush=True)
        return
    grid = tenoaa.make_grid((n, n, n))
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    U = torch.from_numpy(inputs.grf_3d(n)).to(dev)
    ws = tenoaa.workspace(grid, sch, tenoaa.WS_STEP, dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)

    def one_step():
        dt.zero_()
        tenoaa.step(grid, sch, U, dt, gamma=1.4, cfl=0.4, ws=ws)

    if args.copy_calibration:
        # reads and writes exactly 5 * n^3 doubles
        V = torch.empty_like(U)
        torch.neg(U, out=V)
        torch.cuda.synchronize()
        del V
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # events on the stream the library runs on (torch's current stream) between
    # the steps give each step's duration; the wall clock gives the value
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k].record()
        one_step()
    evs[-1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    per_step = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps))
    if tenoaa.get_status(ws) != 0:
        raise RuntimeError("non-physical state during the benchmark")
    ms = el / args.steps * 1e3
    work = 9 * n ** 3
    value = work / (ms * 1e-3) / 1e9

    # per-kernel durations (HIP events on the library's stream) over a few steps
    tenoaa.timing_enable(True)
    ksteps = 3
    for _ in range(ksteps):
        one_step()
    per = {}
    for k, name in enumerate(["sweep_x", "sweep_y", "sweep_z", "update", "wave_speeds"]):
        cnt, tot = tenoaa.timing_read(k)
        per[name] = (cnt, tot)
    tenoaa.timing_enable(False)
    dom = max(["sweep_x", "sweep_y", "sweep_z"], key=lambda k: per[k][1])
    dom_dir = ["sweep_x", "sweep_y", "sweep_z"].index(dom)
    avg_ms = per[dom][1] / per[dom][0]

    # algorithmic flops of that sweep: path counts from the decision flags of
    # one right-hand side of the current state
    fl = torch.zeros(tenoaa.flags_size(grid), dtype=torch.uint8, device=dev)
    tenoaa.rhs(grid, sch, U, gamma=1.4, dt_limiter=float(dt.item()), flags=fl)
    nft = n ** 3
    seg = fl[dom_dir * 10 * nft:(dom_dir + 1) * 10 * nft]
    hist = torch.bincount((seg & 3).to(torch.int64), minlength=4).cpu().tolist()
    sel_counts = {5: hist[3], 4: hist[2], 3: hist[1], 0: hist[0]}
    fl_total = flops.sweep_flops(3, 10, sel_counts, nft, 0, True)
    achieved = fl_total / (avg_ms * 1e-3) / 1e12
    del fl, seg

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gface-recon/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "step_ms_median": round(per_step[len(per_step) // 2], 3),
        "step_ms_min": round(per_step[0], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D Euler %d^3 periodic, GRF + blast sphere + cavity, TENO10-AA, LLF, "
                               "positivity limiter, one SSP-RK3 step at CFL 0.4" % n,
                   "grid": [n, n, n], "order": 10, "splitting": "LLF", "limiter": True,
                   "face_recons_per_step": work},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": measured_traffic(dom),
                     "kernel": dom, "kernel_avg_ms": round(avg_ms, 4),
                     "algorithmic_flops_per_launch": fl_total,
                     "path_counts": {"S5": hist[3], "S4": hist[2], "S3": hist[1], "fallback": hist[0]},
                     "per_kernel_avg_ms": {k: round(v[1] / max(v[0], 1), 4) for k, v in per.items()}},
    }
    if not args.no_fwd_adj:
        # the 3D leg on the headline state (blast and cavity spheres, limiter on)
        U3 = torch.from_numpy(inputs.grf_3d(n)).to(dev)
        U2 = torch.from_numpy(inputs.grf_2d(512, jump=False)).to(dev)
        line["fwd_adj"] = {"3d": fwd_adj_leg((n, n, n), 3, 1, U3, 1),
                           "2d_512_periodic": fwd_adj_leg((512, 512), 20, 3, U2, 0)}
        del U3, U2
    if not args.no_slab:
        line["slab_share"] = slab_leg(torch.from_numpy(inputs.grf_3d(n)).to(dev))
    if not args.no_fwd_adj:
        line["other_workloads"] = gpu_legs(dev)
    if not args.no_batched:
        line["batched"] = batched_leg(tune_cache=args.tune_cache)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
