#!/usr/bin/env python3
"""Benchmark: wall time of one inexact Newton step of the CPR-FGMRES hot path.

One step = assemble the Jacobian and right-hand side, set up the CPR
preconditioner, solve with FGMRES(30) to a relative residual of 1e-6, and
update the state (Algorithm 1, one iteration), on the saturated black-oil
workload of 128 x 128 x 32 cells (3x3 blocks, layered lognormal
permeability with kz/kx = 0.1, inverted five-spot, 1-day step), inputs
already resident in GPU memory.  Every step restarts from the same initial
state so the timed steps do identical work.

Prints one JSON line: the step time, a roofline entry for the dominant
kernel (algorithmic bytes over the average launch duration, measured with
HIP events on the library's stream during the timed steps), and the CPU
oracle's time for the same step as a reference baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CPR-GMRES s/Newton step + GB/s at 1e-6 rel resid; plain FP64 vs mixed+learned"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak of the device

# (input, output) channels and grid level (0 = full, l = 1/2^l per axis) of
# the seven 3x3x3 convolutions of the pressure network
NET_CONVS = [(3, 16, 0), (16, 32, 1), (32, 64, 2), (64, 64, 3), (64, 64, 2), (64, 32, 1), (32, 16, 0)]


def network_flop(nx, ny, nz):
    """Algorithmic FLOP of one inference: 2 * 27 * C_in * C_out per output
    voxel of every convolution, plus the 1x1x1 head."""
    v0 = nx * ny * nz
    conv = sum(2 * 27 * ci * co * v0 // 8 ** lv for ci, co, lv in NET_CONVS)
    return conv + 2 * 16 * v0


def network_timing(nx, ny, nz, reps=50):
    """Event-timed inference of the black-oil network at one grid (batch 1)."""
    import numpy as np
    import torch
    from paper_1606_00548_amd import cprmi, train
    net = cprmi.Network(nx, ny, nz, max_batch=1)
    net.set_params(np.load(train.weights_path("black-oil")))
    x = torch.randn((1, nz, ny, nx, 3), dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.infer(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.infer(x)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    gf = network_flop(nx, ny, nz) / 1e9
    net.close()
    tflops = gf / us * 1e3          # GFLOP per microsecond -> TFLOP/s
    return {"inference_us": us, "gflop_per_inference": gf, "tflops": tflops,
            "frac_of_bf16_peak": tflops / BF16_PEAK_TFLOPS, "grid": [nx, ny, nz], "batch": 1}


def algorithmic_bytes(kclass, b, n, iterations_per_cycle, precision, levels=None):
    """Bytes the launches of one kernel class in one Newton step must move at
    minimum (every array element touched once per launch, FP64), and the
    number of those launches.  iterations_per_cycle: Arnoldi steps of each
    restart cycle; levels: cell counts of the multigrid levels."""
    s = 8
    its = sum(iterations_per_cycle)
    if kclass == "spmv":
        # 7 b x b blocks + x + y per cell; once per cycle also the true
        # residual, which reads the right-hand side as well
        per = (7 * b * b + 2 * b) * s * n
        return its * per + len(iterations_per_cycle) * (per + b * s * n), its + len(iterations_per_cycle)
    if kclass == "orth":
        tot, launches = 0, 0
        for k in iterations_per_cycle:
            for j in range(k):
                nv = j + 1
                # dots: V (nv) + w; update+dots: V + w read + w write;
                # update+norm: V + w read + w write
                tot += ((nv + 1) + (nv + 2) + (nv + 2)) * b * n * s
                launches += 3
        return tot, launches
    if kclass == "smooth":
        # red-black Gauss-Seidel half-sweeps on the levels smoothed by
        # multi-block kernels (those above the first level of <= 4096 cells):
        # black pre-sweep 11 values per black cell (7 stencil, r, x, res, red x),
        # black post-sweep 10 + coarse correction n/8, red sweep 10 (the
        # zero-guess red sweeps ride with the decoupling on the fine level and
        # with the restriction on the others)
        down = next((l for l, nl in enumerate(levels) if nl <= 4096), len(levels) - 1)
        per, launches = 0, 0
        for l in range(down):
            nl = levels[l]
            per += (44 + 41 + 40) * nl
            launches += 3
        return its * per, its * launches
    if kclass == "ilu":
        # stage-2 residual and red-black block ILU(0) sweeps, per cell of a
        # colour: red forward b^2 + 9b values, black 7b^2 + 5b, red backward
        # 7b^2 + 3b + 1, plus the pressure correction dp once per sweep
        nh = n // 2
        per = nh * s * ((b * b + 9 * b) + (7 * b * b + 5 * b) + (7 * b * b + 3 * b + 1)) + 2 * n * s
        return its * per, 3 * its
    raise ValueError(kclass)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--kernel", default="spmv", choices=["spmv", "orth"],
                    help="kernel class reported in the roofline entry")
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--ny", type=int, default=128)
    ap.add_argument("--nz", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP64 / mixed / mixed+learned comparison runs")
    ap.add_argument("--oracle-configs", action="store_true",
                    help="time only the CPU oracle on the other configurations (oil-water 32x32x8: a "
                         "whole Newton step; channelised 256x256x64: assembly, setup and a sample "
                         "of FGMRES iterations) and print one JSON line")
    ap.add_argument("--network-only", action="store_true",
                    help="time only the pressure network's inference on the workload grid")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.network_only:
        print(json.dumps({"network": network_timing(args.nx, args.ny, args.nz, reps=max(args.steps, 1) * 10)}))
        return
    if args.oracle_configs:
        print(json.dumps({"oracle_configs": oracle_configs()}))
        return

    import numpy as np
    import torch
    from paper_1606_00548_amd import cprmi, synth

    case = synth.black_oil_layered(args.nx, args.ny, args.nz)
    n = args.nx * args.ny * args.nz
    b = 3
    solver = cprmi.Solver.from_case(case)
    x_old = torch.as_tensor(case["x_old"]).cuda().contiguous()
    x0 = torch.as_tensor(case["x"]).cuda().contiguous()
    x = x0.clone()
    opts = cprmi.default_options(precision=args.precision)

    step_times = []   # host wall time of each timed step, per call of timed()

    def timed(o, kernel=None, krylov="fgmres"):
        """Warm-up, then exactly args.steps Newton steps between two syncs."""
        def step():
            x.copy_(x0)
            dx, st = cprmi.newton_step(solver, x_old, x, case["dt"], o, krylov=krylov)
            return st
        for _ in range(args.warmup):
            step()
        if kernel:
            solver.profile_kernel(kernel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts, marks = [], [t0]
        for _ in range(args.steps):
            sts.append(step())
            marks.append(time.perf_counter())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step_times.append([b - a for a, b in zip(marks[:-1], marks[1:])])
        prof = solver.profile_read() if kernel else (0, 0.0)
        if kernel:
            solver.profile_kernel(None)
        if not all(st["status"] == 0 and st["true_rel"] <= 1e-6 for st in sts):
            print("a timed solve did not reach the 1e-6 true relative residual", file=sys.stderr)
            sys.exit(1)
        return (t1 - t0) / args.steps, sts, prof

    sec_per_step, stats, (launches, kernel_ms) = timed(opts, args.kernel)
    median_ms = 1e3 * float(np.median(step_times[-1]))

    # the other forms of the preconditioner on the same workload
    variants = {}
    if not args.no_variants:
        from paper_1606_00548_amd import train
        wfile = train.weights_path("black-oil")
        forms = [("fp64", dict(precision="fp64"), "fgmres"), ("mixed", dict(precision="mixed"), "fgmres")]
        if os.path.exists(wfile):
            solver.attach_network(np.load(wfile))
            forms.append(("mixed+learned", dict(precision="mixed", learned=1), "fgmres"))
        forms.append(("bicgstab fp64", dict(precision="fp64"), "bicgstab"))
        if os.path.exists(wfile):
            forms.append(("bicgstab mixed+learned", dict(precision="mixed", learned=1), "bicgstab"))
        # ABF decoupling and the F-P-F composition (CPR-FPF)
        forms.append(("abf fp64", dict(precision="fp64", decoupling="abf"), "fgmres"))
        forms.append(("fpf fp64", dict(precision="fp64", composition="fpf"), "fgmres"))
        forms.append(("fpf mixed", dict(precision="mixed", composition="fpf"), "fgmres"))
        if os.path.exists(wfile):
            forms.append(("fpf mixed+learned", dict(precision="mixed", composition="fpf", learned=1), "fgmres"))
            forms.append(("bicgstab fpf mixed+learned", dict(precision="mixed", composition="fpf", learned=1),
                          "bicgstab"))
        # a tuned cycle: more smoothing sweeps per level, V(pre, post), and an
        # over-correction x += alpha P e with alpha = 1.25
        tuned = dict(mg_pre=2, mg_post=2)
        forms.append(("fp64 V(2,2)", dict(precision="fp64", **tuned), "fgmres"))
        forms.append(("mixed V(2,2)", dict(precision="mixed", **tuned), "fgmres"))
        tuned["mg_alpha"] = 1.25
        forms.append(("fp64 V(2,2) alpha 1.25", dict(precision="fp64", **tuned), "fgmres"))
        forms.append(("mixed V(2,2) alpha 1.25", dict(precision="mixed", **tuned), "fgmres"))
        if os.path.exists(wfile):
            forms.append(("mixed+learned V(2,2) alpha 1.25", dict(precision="mixed", learned=1, **tuned), "fgmres"))
        for name, kw, kry in forms:
            sp, sts, _ = timed(cprmi.default_options(**kw), krylov=kry)
            variants[name] = {"s_per_step": sp, "krylov": kry, "krylov_iterations": sts[-1]["iterations"],
                              "true_rel": sts[-1]["true_rel"], "speedup_vs_fp64": None,
                              "nn_accepted": sts[-1]["nn_accepted"]}
        for v in variants.values():
            v["speedup_vs_fp64"] = variants["fp64"]["s_per_step"] / v["s_per_step"]
        solver.attach_network(None)

    # one whole backward-Euler step of the same workload (Algorithm 1 with
    # the first forcing term of eq. (14), time-step cuts, variable switching)
    time_step, simulation = {}, {}
    if not args.no_variants:
        from paper_1606_00548_amd import train
        wfile = train.weights_path("black-oil")
        forms = [("fp64", dict(precision="fp64"))]
        if os.path.exists(wfile):
            solver.attach_network(np.load(wfile))
            forms.append(("mixed+learned", dict(precision="mixed", learned=1)))
        tuned = dict(mg_pre=2, mg_post=2, mg_alpha=1.25)
        forms += [("fp64 V(2,2) alpha 1.25", dict(precision="fp64", **tuned)),
                  ("mixed V(2,2) alpha 1.25", dict(precision="mixed", **tuned))]
        xts = torch.empty_like(x0)
        for name, kw in forms:
            lo = cprmi.default_options(**kw)
            solver.time_step(x_old, case["dt"], options=lo, x=xts)        # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, tst = solver.time_step(x_old, case["dt"], options=lo, x=xts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            time_step[name] = {"s": t1 - t0, "converged": bool(tst["converged"]), "cuts": tst["cuts"],
                               "dt_taken_days": tst["dt_taken"], "newton_iterations": tst["newton_iterations"],
                               "linear_iterations": tst["history"]["linear_iterations"],
                               "total_newton": tst["total_newton"], "total_linear": tst["total_linear"],
                               "undersaturated_cells": int((xts[2] < 0).sum())}
            # the same day with step growth from 0.01 day (cpr_simulate)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sst = solver.simulate(x_old, case["dt"], 0.01, case["dt"], options=lo, x=xts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            simulation[name] = {"s": t1 - t0, "completed": bool(sst["completed"]), "steps": sst["steps"],
                                "cuts": sst["cuts"], "total_newton": sst["total_newton"],
                                "total_linear": sst["total_linear"], "dts_days": sst["dts"],
                                "undersaturated_cells": int((xts[2] < 0).sum())}
        solver.attach_network(None)

    # per-phase breakdown of one more (untimed) step
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    x.copy_(x0)
    ev[0].record()
    rhs = solver.assemble(x_old, x, case["dt"])
    ev[1].record()
    solver.setup(opts)
    ev[2].record()
    dx, st = solver.solve(rhs)
    ev[3].record()
    solver.newton_update(x, dx)
    ev[4].record()
    torch.cuda.synchronize()
    phases = {k: ev[i].elapsed_time(ev[i + 1]) for i, k in
              enumerate(["assemble", "setup", "solve", "update"])}
    # restart-cycle lengths of the timed solves (identical every step)
    its, cycles = st["iterations"], st["cycles"]
    per_cycle = [30] * (cycles - 1) + [its - 30 * (cycles - 1)] if cycles else []
    alg_bytes, alg_launches = algorithmic_bytes(args.kernel, b, n, per_cycle, args.precision)  # spmv / orth
    avg_ms = kernel_ms / max(launches, 1)
    achieved = (alg_bytes / alg_launches) / (avg_ms * 1e-3) / 1e9 if launches else None
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"{args.kernel}_traffic.json")
    if os.path.exists(tfile):
        info = json.load(open(tfile))
        if info.get("workload_cells") == n and info.get("source_sha") == _kernel_sha(args.kernel):
            traffic = info.get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": args.kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": traffic, "launches_sampled": launches,
                "avg_launch_us": avg_ms * 1e3,
                "algorithmic_bytes_per_launch": alg_bytes / max(alg_launches, 1)}
    if launches != alg_launches * args.steps:
        roofline["note"] = f"sampled {launches} launches, expected {alg_launches * args.steps}"

    # achieved bandwidth of each bandwidth-bound kernel class (FP64 form)
    levels = []
    while solver.mg_level_shape(len(levels)) is not None:
        levels.append(int(np.prod(solver.mg_level_shape(len(levels)))))
    classes = {}
    for cls in ("spmv", "orth", "smooth", "ilu"):
        _, _, (nl, ms) = timed(cprmi.default_options(precision="fp64"), cls)
        ab, al = algorithmic_bytes(cls, b, n, per_cycle, "fp64", levels)
        gbs = ab * args.steps / (ms * 1e-3) / 1e9 if ms > 0 else None
        classes[cls] = {"launches_per_step": nl / args.steps, "expected_launches_per_step": al,
                        "ms_per_step": ms / args.steps, "avg_launch_us": 1e3 * ms / max(nl, 1),
                        "algorithmic_bytes_per_step": ab, "GBps": gbs,
                        "frac": gbs / HBM_PEAK_GBS if gbs else None}

    # measured HBM bandwidth on this device: STREAM triad a = b + 3 c over
    # 3 x 1 GiB FP64 arrays (torch elementwise kernel), best of 5
    ta = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    tb = torch.ones_like(ta)
    tc = torch.ones_like(ta)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.add(tb, tc, alpha=3.0, out=ta)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        best = t if best is None else min(best, t)
    triad_gbs = 3 * ta.numel() * 8 / best / 1e9
    # and a device-to-device copy of 1 GiB (the runtime's copy kernel), best of 5
    bestc = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ta.copy_(tb)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        bestc = t if bestc is None else min(bestc, t)
    copy_gbs = 2 * ta.numel() * 8 / bestc / 1e9
    del ta, tb, tc
    roofline["measured_triad_GBps"] = triad_gbs
    roofline["measured_copy_GBps"] = copy_gbs
    roofline["frac_of_measured_triad"] = (achieved / triad_gbs) if achieved else None
    for v in classes.values():
        v["frac_of_measured_triad"] = v["GBps"] / triad_gbs if v["GBps"] else None
    # the four bandwidth-bound classes together over the whole solve phase
    class_bytes = sum(v["algorithmic_bytes_per_step"] for v in classes.values())
    solve_gbps = class_bytes / (phases["solve"] * 1e-3) / 1e9

    network = network_timing(args.nx, args.ny, args.nz)
    configs = other_configs() if not args.no_variants else {}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case)
        # the oracle moves the same algorithmic bytes for the step
        cpu["GBps"] = class_bytes / cpu["value"] / 1e9
    out = {
        "metric": METRIC, "value": sec_per_step, "unit": "s/Newton step", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"black-oil layered {args.nx}x{args.ny}x{args.nz} "
                               f"({n} cells, 3x3 blocks), one Newton step, FGMRES(30) to 1e-6",
                   "cells": n, "block": b, "precision": args.precision, "restart": 30, "rtol": 1e-6,
                   "preconditioner": "quasi-IMPES CPR, P-then-F, multigrid V(1,1), alpha 1, coarsest <= 512 "
                                     "cells, red-black block ILU(0)"},
        "median_ms_per_step": median_ms,
        "fgmres_iterations": its, "restart_cycles": cycles, "true_rel": st["true_rel"],
        "solve_class_bytes_GBps": solve_gbps, "network": network,
        "phases_ms": phases, "roofline": roofline, "kernel_classes": classes, "cpu_baseline": cpu,
        "variants": variants, "time_step": time_step, "simulation": simulation, "other_configs": configs,
    }
    print(json.dumps(out))


def _kernel_sha(kclass):
    import hashlib
    f = {"spmv": "spmv.hip", "orth": "krylov.hip"}[kclass]
    p = os.path.join(ROOT, "paper_1606_00548_amd", "csrc", f)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def other_configs(steps=2):
    """One Newton step of the small oil-water system (32x32x8, latency
    regime) and of the first system of the channelised 256x256x64 black-oil
    10-day step (bandwidth regime), FP64 and mixed precision, with the
    default V(1,1) cycle and with the tuned V(2,2), alpha 1.25 one; each
    timed step restarts from the same state."""
    import numpy as np
    import torch
    from paper_1606_00548_amd import cprmi, synth
    out = {}
    for name, make in (("oil-water 32x32x8", lambda: synth.oil_water_lognormal()),
                       ("black-oil channelised 256x256x64, first system of the 10-day step",
                        lambda: synth.black_oil_channelised())):
        case = make()
        s = cprmi.Solver.from_case(case)
        x_old = torch.as_tensor(case["x_old"]).cuda().contiguous()
        x0 = torch.as_tensor(case["x"]).cuda().contiguous()
        x = x0.clone()
        res = {"cells": int(np.prod(case["x"].shape[1:])), "block": int(case["x"].shape[0])}
        forms = (("fp64", dict(precision="fp64")), ("mixed", dict(precision="mixed")),
                 ("fp64 V(2,2) alpha 1.25", dict(precision="fp64", mg_pre=2, mg_post=2, mg_alpha=1.25)),
                 ("mixed V(2,2) alpha 1.25", dict(precision="mixed", mg_pre=2, mg_post=2, mg_alpha=1.25)))
        for prec, kw in forms:
            o = cprmi.default_options(**kw)

            def step():
                x.copy_(x0)
                _, st = cprmi.newton_step(s, x_old, x, case["dt"], o)
                return st
            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = [step() for _ in range(steps)]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ok = all(st["status"] == 0 and st["true_rel"] <= 1e-6 for st in sts)
            res[prec] = {"ms_per_step": 1e3 * (t1 - t0) / steps, "iterations": sts[-1]["iterations"],
                         "true_rel": sts[-1]["true_rel"], "reached_1e-6": ok}
        s.close()
        del x_old, x0, x
        torch.cuda.empty_cache()
        out[name] = res
    return out


def cpu_baseline(case):
    """The FP64 oracle's time for the same Newton step (single thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import newton
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, _, st, _ = newton.newton_step(case["grid"], case["fluid"], case["perm"], case["poro"],
                                         case["wells"], case["x_old"], case["x"], case["dt"])
        t1 = time.perf_counter()
    return {"value": t1 - t0, "unit": "s/Newton step", "cores": 1, "kind": "oracle",
            "sample": "one full Newton step (assemble, CPR setup, FGMRES(30) to 1e-6, update) "
                      "of the same workload, numpy/scipy single-threaded",
            "iterations": st["iterations"]}


def oracle_configs(sample_iterations=10):
    """The FP64 oracle, single-threaded, on the other configurations: the
    whole Newton step of the oil-water 32x32x8 system; for the channelised
    256x256x64 system (whose step takes about a hundred FGMRES iterations)
    the assembly, the CPR setup and the first `sample_iterations` FGMRES
    iterations, timed separately and reported as measured."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cpr, krylov, model, newton
    from paper_1606_00548_amd import synth
    out = {}
    with threadpool_limits(limits=1):
        case = synth.oil_water_lognormal()
        t0 = time.perf_counter()
        _, _, st, _ = newton.newton_step(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                                         case["x_old"], case["x"], case["dt"])
        out["oil-water 32x32x8"] = {"s_per_newton_step": time.perf_counter() - t0,
                                    "iterations": st["iterations"], "cores": 1}
        case = synth.black_oil_channelised()
        t0 = time.perf_counter()
        R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                              case["x_old"], case["x"], case["dt"])
        t1 = time.perf_counter()
        pc = cpr.cpr_setup(J)
        t2 = time.perf_counter()
        _, st = krylov.fgmres(lambda v: cpr.block_spmv(J, v), lambda v: cpr.cpr_apply(pc, v), -R,
                              rtol=0.0, max_iter=sample_iterations)
        t3 = time.perf_counter()
        out["black-oil channelised 256x256x64"] = {
            "assemble_s": t1 - t0, "setup_s": t2 - t1, "fgmres_iterations_sampled": st["iterations"],
            "s_per_fgmres_iteration": (t3 - t2) / st["iterations"], "cores": 1,
            "cells": int(np.prod(case["x"].shape[1:]))}
    return out


if __name__ == "__main__":
    main()
