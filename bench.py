#!/usr/bin/env python3
"""Benchmark: wall time of one inexact Newton step of the CPR-FGMRES hot path.

One step = assemble the Jacobian and right-hand side, set up the CPR
preconditioner, solve with FGMRES(30) to a relative residual of 1e-6, and
update the state (Algorithm 1, one iteration).  Every form on the line uses
the same CPR: quasi-IMPES decoupling, an aggregation multigrid V(2,2) cycle
with its coarse correction scaled by 1.25 for the pressure, red-black block
ILU(0); the library's default V(1,1) cycle is reported beside it.  The default workload is the
largest single-GPU one: saturated black oil on a 512 x 512 x 128 grid
(33.5 M cells, 3x3 blocks, a 17 GB FP64 Jacobian), lognormal permeability
with sigma 1.5 correlated over (4, 4, 1) cells, kz = 0.1 kx, 25 BHP wells on
a 5 x 5 lattice, a 1-day step; inputs resident in GPU memory, every step
restarting from the same state so the timed steps do identical work.

Prints one JSON line: the plain FP64 step time (value), the same step with
the FP32 preconditioner and with the FP32 preconditioner plus the learned
pressure stage (variants, each with its distance to the FP64 solution), a
roofline entry for the dominant kernel (the block SpMV: algorithmic bytes
over its average launch duration, sampled with HIP events on the library's
stream in a separate pass of identical steps), the achieved bandwidth of
each kernel class, and the CPU oracle's time for a bounded sample of the
same workload, scaled to one whole Newton step.
"""
import argparse
import json
import os
import platform
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

# multigrid cycle of every form on the headline line: two red-black
# Gauss-Seidel sweeps before and after the coarse correction, which is scaled
# by 1.25 (the library default is V(1,1) with alpha 1; both are reported)
CYCLE = dict(mg_pre=2, mg_post=2, mg_alpha=1.25)

# workload name -> (synth generator, default shape)
WORKLOADS = {
    "lattice": ("black_oil_lattice", (512, 512, 128)),
    "layered": ("black_oil_layered", (128, 128, 32)),
    "channelised": ("black_oil_channelised", (256, 256, 64)),
    "oil-water": ("oil_water_lognormal", (32, 32, 8)),
}


def make_case(workload, nx=None, ny=None, nz=None):
    from paper_1606_00548_amd import synth
    gen, (dnx, dny, dnz) = WORKLOADS[workload]
    return getattr(synth, gen)(nx or dnx, ny or dny, nz or dnz)


def network_flop(nx, ny, nz):
    """Algorithmic FLOP of one inference: 2 * 27 * C_in * C_out per output
    voxel of every convolution, plus the 1x1x1 head."""
    v0 = nx * ny * nz
    conv = sum(2 * 27 * ci * co * v0 // 8 ** lv for ci, co, lv in NET_CONVS)
    return conv + 2 * 16 * v0


def network_timing(nx, ny, nz, reps=20):
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
    del x
    torch.cuda.empty_cache()
    tflops = gf / us * 1e3          # GFLOP per microsecond -> TFLOP/s
    return {"inference_us": us, "gflop_per_inference": gf, "tflops": tflops,
            "frac_of_bf16_peak": tflops / BF16_PEAK_TFLOPS, "grid": [nx, ny, nz], "batch": 1}


def algorithmic_bytes(kclass, b, n, iterations_per_cycle, precision, levels=None, orth="dcgs2", pre=1, post=1):
    """Bytes the launches of one kernel class in one Newton step must move at
    minimum (every array element touched once per launch, FP64), and the
    number of those launches.  iterations_per_cycle: Arnoldi steps of each
    restart cycle; levels: cell counts of the multigrid levels; orth: the
    FGMRES orthogonalisation (delayed CGS2 or CGS2); pre / post: sweeps of
    the V(pre, post) cycle."""
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
                if orth == "cgs2":
                    # nv = j + 1 vectors; dots: V + w; update+dots: V + w read
                    # + w write; update+norm: V + w read + w write
                    nv = j + 1
                    tot += ((nv + 1) + (nv + 2) + (nv + 2)) * b * n * s
                    launches += 3
                else:
                    # delayed CGS2, j final vectors before uh: dots read V,
                    # uh, w; update reads V, uh, w and writes v_j and u
                    tot += ((j + 2) + (j + 4)) * b * n * s
                    launches += 2
        return tot, launches
    if kclass == "smooth":
        # red-black Gauss-Seidel half-sweeps on the levels smoothed by
        # multi-block kernels (those above the first level of <= 4096 cells):
        # black pre-sweep 11 values per black cell (7 stencil, r, x, res, red x),
        # black post-sweep 10 + coarse correction n/8, red sweep 10 (the
        # zero-guess red sweep of the first pre-sweep rides with the
        # decoupling on the fine level and with the restriction on the
        # others); each further pre-sweep is red + black pre, each further
        # post-sweep black pre + red
        down = next((l for l, nl in enumerate(levels) if nl <= 4096), len(levels) - 1)
        per, launches = 0, 0
        for l in range(down):
            nl = levels[l]
            per += (44 + 41 + 40 + (pre - 1 + post - 1) * (40 + 44)) * nl
            launches += 3 + 2 * (pre - 1 + post - 1)
        return its * per, its * launches
    if kclass == "ilu":
        # stage-2 residual and red-black block ILU(0) sweeps, per cell of a
        # colour: red forward b^2 + 9b values, black 7b^2 + 5b, red backward
        # 7b^2 + 3b + 1, plus the pressure correction dp once per sweep
        nh = n // 2
        per = nh * s * ((b * b + 9 * b) + (7 * b * b + 5 * b) + (7 * b * b + 3 * b + 1)) + 2 * n * s
        return its * per, 3 * its
    raise ValueError(kclass)


def cycle_lengths(st, restart=30):
    its, cycles = st["iterations"], st["cycles"]
    return [restart] * (cycles - 1) + [its - restart * (cycles - 1)] if cycles else []


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# ------------------------------------------------------------------ CPU oracle

def _oracle_window(args):
    """One full Newton step of the FP64 oracle on a window of a workload,
    single-threaded, phase by phase (runs in a worker process)."""
    sub, = args
    from threadpoolctl import threadpool_limits

    from oracle import cpr, krylov, model, newton
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        R, J = model.assemble(sub["grid"], sub["fluid"], sub["perm"], sub["poro"], sub["wells"],
                              sub["x_old"], sub["x"], sub["dt"])
        t1 = time.perf_counter()
        pc = cpr.cpr_setup(J, pre=CYCLE["mg_pre"], post=CYCLE["mg_post"])
        t2 = time.perf_counter()
        dx, st = krylov.fgmres(lambda v: cpr.block_spmv(J, v),
                               lambda v: cpr.cpr_apply(pc, v, alpha=CYCLE["mg_alpha"]), -R)
        t3 = time.perf_counter()
        newton.newton_update(sub["x"], dx, float(sub["fluid"]["pvt"][0][0]) if sub["fluid"]["model"] == 3 else None)
        t4 = time.perf_counter()
    return {"cells": int(sub["x"][0].size), "assemble_s": t1 - t0, "setup_s": t2 - t1, "solve_s": t3 - t2,
            "update_s": t4 - t3, "iterations": int(st["iterations"]), "converged": bool(st["converged"])}


def _windows(case, wn, count):
    """Sub-cases: wn = (nx, ny, nz) windows of the workload centred on its
    first `count` wells (top layers), wells clipped to the window."""
    g = case["grid"]
    out = []
    for w in case["wells"][:count]:
        i0 = min(max(w["i"] - wn[0] // 2, 0), g["nx"] - wn[0])
        j0 = min(max(w["j"] - wn[1] // 2, 0), g["ny"] - wn[1])
        win = (slice(0, wn[2]), slice(j0, j0 + wn[1]), slice(i0, i0 + wn[0]))
        wells = [dict(v, i=v["i"] - i0, j=v["j"] - j0, k0=0, k1=wn[2] - 1) for v in case["wells"]
                 if i0 <= v["i"] < i0 + wn[0] and j0 <= v["j"] < j0 + wn[1]]
        out.append({"grid": dict(g, nx=wn[0], ny=wn[1], nz=wn[2]), "fluid": case["fluid"],
                    "perm": case["perm"][(slice(None),) + win].copy(), "poro": case["poro"][win].copy(),
                    "wells": wells, "x_old": case["x_old"][(slice(None),) + win].copy(),
                    "x": case["x"][(slice(None),) + win].copy(), "dt": case["dt"]})
    return out


def cpu_baseline_sample(case, procs):
    """The oracle on a bounded sample of the workload: `procs` windows of
    128 x 128 x 16 cells (or the whole grid if it is smaller), each a full
    Newton step in its own single-threaded process, all at once on the
    host's cores.  Runs before anything touches the GPU."""
    import multiprocessing as mp
    g = case["grid"]
    wn = (min(128, g["nx"]), min(128, g["ny"]), min(16, g["nz"]))
    whole = wn == (g["nx"], g["ny"], g["nz"])
    subs = _windows(case, wn, 1 if whole else procs)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(len(subs)) as pool:
        res = pool.map(_oracle_window, [(s,) for s in subs])
    wall = time.perf_counter() - t0
    return {"windows": res, "window": list(wn), "whole_grid": whole, "processes": len(subs), "wall_s": wall}


def cpu_baseline_value(sample, n, gpu_iterations, class_bytes):
    """Scale the sampled oracle rates to one Newton step of the whole grid
    on the cores the sample ran on: per-cell assembly, setup and update
    times, and the per-cell time of one FGMRES iteration times the
    iterations the full system takes (the GPU's FP64 count; the oracle
    follows the same path), per core as measured with all windows running at
    once, divided by the number of those cores (the windows are independent,
    so p cores take the cells of p windows in the time one core takes one)."""
    ws = sample["windows"]
    cells = sum(w["cells"] for w in ws)
    fixed = sum(w["assemble_s"] + w["setup_s"] + w["update_s"] for w in ws) / cells
    per_it = sum(w["solve_s"] for w in ws) / sum(w["cells"] * w["iterations"] for w in ws)
    single = fixed * n + per_it * n * gpu_iterations
    value = single / sample["processes"]
    return {
        "value": value, "unit": "s/Newton step", "cores": sample["processes"], "kind": "oracle",
        "sample": (f"{sample['processes']} window(s) of {'x'.join(map(str, sample['window']))} cells of the "
                   f"same workload{' (the whole grid)' if sample['whole_grid'] else ', centred on wells'}, one full "
                   "Newton step each (assemble, CPR setup, FGMRES(30) with the V(2,2), alpha 1.25 cycle to "
                   "1e-6, update) in a single-threaded "
                   "numpy process per window, all running at once; value = (measured per-cell assembly/setup/"
                   f"update time x {n} cells + measured per-cell-per-iteration FGMRES time x {n} cells x "
                   f"{gpu_iterations} iterations (the whole system's FP64 count)) / {sample['processes']} "
                   "processes (per-core times measured with all of them running)"),
        "single_core_value": single,
        "sample_wall_s": sample["wall_s"], "window_iterations": [w["iterations"] for w in ws],
        "windows_converged": all(w["converged"] for w in ws),
        "host": {"nproc": os.cpu_count(), "cpu_model": _cpu_model()},
        "GBps": class_bytes / value / 1e9 if class_bytes else None,
    }


# ------------------------------------------------------------------ GPU runs

class Stepper:
    """Times whole Newton steps of one solver and state."""

    def __init__(self, solver, case):
        import torch
        self.torch = torch
        self.s = solver
        self.case = case
        self.x_old = torch.as_tensor(case["x_old"]).cuda().contiguous()
        self.x0 = torch.as_tensor(case["x"]).cuda().contiguous()
        self.x = self.x0.clone()

    def step(self, o, krylov="fgmres"):
        from paper_1606_00548_amd import cprmi
        self.x.copy_(self.x0)
        return cprmi.newton_step(self.s, self.x_old, self.x, self.case["dt"], o, krylov=krylov)

    def timed(self, o, steps, warmup, krylov="fgmres", kclass=None):
        """Warm-up, then exactly `steps` Newton steps between two syncs.
        Returns (s per step, per-step host times, stats, dx of the last step,
        sampled launches, sampled ms)."""
        torch = self.torch
        for _ in range(warmup):
            self.step(o, krylov)
        if kclass:
            self.s.profile_kernel(kclass)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts, marks, dx = [], [t0], None
        for _ in range(steps):
            dx, st = self.step(o, krylov)
            sts.append(st)
            marks.append(time.perf_counter())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = self.s.profile_read() if kclass else (0, 0.0)
        if kclass:
            self.s.profile_kernel(None)
        if not all(st["status"] == 0 and st["true_rel"] <= 1e-6 for st in sts):
            print("a timed solve did not reach the 1e-6 true relative residual", file=sys.stderr)
            sys.exit(1)
        return (t1 - t0) / steps, [b - a for a, b in zip(marks[:-1], marks[1:])], sts, dx, prof

    def phases(self, o):
        """Device time of each phase of one Newton step from the library's
        phase timers (HIP events on its stream), milliseconds."""
        torch = self.torch
        self.s.set_timing(True)
        self.x.copy_(self.x0)
        rhs = self.s.assemble(self.x_old, self.x, self.case["dt"])
        self.s.setup(o)
        dx, st = self.s.solve(rhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.s.newton_update(self.x, dx)
        torch.cuda.synchronize()
        upd = (time.perf_counter() - t0) * 1e3
        self.s.set_timing(False)
        out = {"assemble": st["ms_assemble"], "setup": st["ms_setup"], "solve": st["ms_solve"],
               "update (host-timed)": upd, "solve: preconditioner": st["ms_precond"], "solve: spmv": st["ms_spmv"],
               "solve: orthogonalisation": st["ms_orth"]}
        return out, st


def measured_bandwidth():
    """STREAM triad a = b + 3 c over 3 x 1 GiB FP64 arrays and a 1 GiB
    device copy (torch kernels), best of 5 each, in GB/s."""
    import torch
    ta = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    tb = torch.ones_like(ta)
    tc = torch.ones_like(ta)

    def best(fn):
        b = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3
            b = t if b is None else min(b, t)
        return b
    triad = 3 * ta.numel() * 8 / best(lambda: torch.add(tb, tc, alpha=3.0, out=ta)) / 1e9
    copy = 2 * ta.numel() * 8 / best(lambda: ta.copy_(tb)) / 1e9
    del ta, tb, tc
    torch.cuda.empty_cache()
    return triad, copy


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def newton_iterations_mixed_vs_fp64(s, case, iters=10, dt0=0.01, newton_tol=1e-3):
    """The first `iters` Newton iterations of the workload's time stepping
    (Algorithm 1 with every system solved to 1e-6; steps from dt0 days,
    doubling after each converged step, as the simulation's) along two
    paths, plain FP64 CPR and the FP32 preconditioner.  Both paths take the
    same step lengths and, within a step, as many iterations as the FP64
    path needs to reach ||F(x_l)|| < newton_tol ||F(x_0)||.  Per iteration:
    the nonlinear residual of each path, the FGMRES iterations, the relative
    difference of the mixed correction from the FP64 one on the same
    (FP64-path) state, and the relative difference of the two paths' states
    after the update."""
    import torch
    from paper_1606_00548_amd import cprmi
    o64 = cprmi.default_options(precision="fp64")
    om = cprmi.default_options(precision="mixed")
    old64 = torch.as_tensor(case["x_old"]).cuda()
    oldm = old64.clone()
    x64, xm = old64.clone(), oldm.clone()
    rows = []
    dt, step, f0 = dt0, 1, None
    while len(rows) < iters:
        rhs = s.assemble(old64, x64, dt)
        f64 = float(torch.linalg.vector_norm(rhs))
        f0 = f64 if f0 is None else f0
        if f64 < newton_tol * f0:
            # the step converged: both paths start the next one from it
            old64, oldm = x64.clone(), xm.clone()
            dt, step, f0 = min(2 * dt, case["dt"]), step + 1, None
            continue
        s.setup(o64)
        dx64, st64 = s.solve(rhs)
        s.setup(om)
        dxs, sts = s.solve(rhs)
        same = _rel(dxs, dx64)
        rhm = s.assemble(oldm, xm, dt)
        s.setup(om)
        dxm, stm = s.solve(rhm)
        s.newton_update(x64, dx64)
        s.newton_update(xm, dxm)
        torch.cuda.synchronize()
        rows.append({"iteration": len(rows) + 1, "time_step": step, "dt_days": dt, "residual_fp64": f64,
                     "residual_mixed": float(torch.linalg.vector_norm(rhm)),
                     "fgmres_fp64": st64["iterations"], "fgmres_mixed": stm["iterations"],
                     "dx_rel_diff_same_state": same, "state_rel_diff_after": _rel(xm, x64),
                     "true_rel_fp64": st64["true_rel"], "true_rel_mixed": stm["true_rel"]})
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lattice", choices=sorted(WORKLOADS))
    ap.add_argument("--nx", type=int)
    ap.add_argument("--ny", type=int)
    ap.add_argument("--nz", type=int)
    ap.add_argument("--variant-steps", type=int, default=3,
                    help="timed steps of each comparison form (at most --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed / mixed+learned / tuned-cycle comparison runs")
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--kernel-only", choices=["spmv", "ilu", "orth"],
                    help="for counter runs, printing one JSON line: 'spmv' assembles once, then launches only "
                         "the SpMV 20 times and copies the state vector once (calibration); 'ilu' sets up the "
                         "V(2,2) cycle with each ILU order in FP64 and FP32, applies each form 10 times and "
                         "copies the state vector once; 'orth' runs one FGMRES(30) cycle of 30 steps (FP64, rtol 0) "
                         "and the same copy")
    ap.add_argument("--network-only", action="store_true",
                    help="time only the pressure network's inference on the workload grid")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    gen, dshape = WORKLOADS[args.workload]
    nx, ny, nz = args.nx or dshape[0], args.ny or dshape[1], args.nz or dshape[2]
    if args.network_only:
        print(json.dumps({"network": network_timing(nx, ny, nz, reps=max(args.steps, 1) * 10)}))
        return

    case = make_case(args.workload, nx, ny, nz)
    n = nx * ny * nz
    b = int(case["x"].shape[0])
    # the CPU sample runs first, before this process initialises the GPU
    sample = None
    if not args.no_cpu_baseline and not args.kernel_only:
        sample = cpu_baseline_sample(case, procs=min(16, os.cpu_count() or 1))

    import numpy as np
    import torch
    from paper_1606_00548_amd import cprmi, train

    solver = cprmi.Solver.from_case(case)
    run = Stepper(solver, case)
    if args.kernel_only:
        print(json.dumps(kernel_only(run, args.kernel_only, n, b)))
        return
    fp64 = cprmi.default_options(precision="fp64", **CYCLE)

    # headline: plain FP64 CPR, no per-launch events inside the timed steps
    sec, host_times, sts, dx64, _ = run.timed(fp64, args.steps, args.warmup)
    st = sts[-1]
    per_cycle = cycle_lengths(st)

    # the comparison asked for by the metric, on the same workload
    variants = {"fp64": {"s_per_step": sec, "krylov_iterations": st["iterations"], "true_rel": st["true_rel"],
                         "speedup_vs_fp64": 1.0, "rel_diff_vs_fp64": 0.0, "nn_accepted": 0}}
    wfile = train.weights_path("black-oil")
    if not args.no_variants:
        vs = min(args.variant_steps, args.steps)
        learned = os.path.exists(wfile) and b == 3
        auto_level = solver.nn_level()      # the learned stage's level chosen by the last setup
        forms = [("mixed", dict(precision="mixed", **CYCLE))]
        if learned:
            forms.append(("mixed+learned", dict(precision="mixed", learned=1, **CYCLE)))
            forms.append(("mixed+learned fine level", dict(precision="mixed", learned=1, nn_level=0, **CYCLE)))
            forms.append(("fp64+learned", dict(precision="fp64", learned=1, **CYCLE)))
        forms += [("fp64 CGS2", dict(precision="fp64", orth="cgs2", **CYCLE)),
                  ("fp64 tiled ILU", dict(precision="fp64", ilu_order="tiles", **CYCLE)),
                  ("mixed tiled ILU", dict(precision="mixed", ilu_order="tiles", **CYCLE))]
        if learned:
            forms.append(("mixed+learned tiled ILU", dict(precision="mixed", learned=1, ilu_order="tiles", **CYCLE)))
        forms += [("fp64 V(1,1) alpha 1", dict(precision="fp64")),
                  ("mixed V(1,1) alpha 1", dict(precision="mixed"))]
        if learned:
            forms.append(("mixed+learned V(1,1) alpha 1", dict(precision="mixed", learned=1)))
        for name, kw in forms:
            net_file = None
            if kw.get("learned"):
                # the network trained for the level the stage acts on, if shipped
                net_file = train.weights_for_level("black-oil", kw.get("nn_level", auto_level))
                solver.attach_network(np.load(net_file))
            sp, _, vsts, dxv, _ = run.timed(cprmi.default_options(**kw), vs, 1)
            variants[name] = {"s_per_step": sp, "krylov_iterations": vsts[-1]["iterations"],
                              "true_rel": vsts[-1]["true_rel"], "speedup_vs_fp64": sec / sp,
                              "rel_diff_vs_fp64": _rel(dxv, dx64), "nn_accepted": vsts[-1]["nn_accepted"],
                              "fp64_fallback_after_cycle": vsts[-1].get("fp64_fallback", 0)}
            if kw.get("learned"):
                variants[name]["nn_level"] = solver.nn_level()
                variants[name]["network"] = os.path.basename(net_file)
        solver.attach_network(None)

    phases, _ = run.phases(fp64)

    # achieved bandwidth of each bandwidth-bound kernel class (FP64 form),
    # HIP events around every launch of the class, one class per pass
    levels = []
    while solver.mg_level_shape(len(levels)) is not None:
        levels.append(int(np.prod(solver.mg_level_shape(len(levels)))))
    ks = min(2, args.steps)
    classes = {}
    for cls in ("spmv", "orth", "smooth", "ilu"):
        _, _, _, _, (nl, ms) = run.timed(fp64, ks, 0, kclass=cls)
        ab, al = algorithmic_bytes(cls, b, n, per_cycle, "fp64", levels, pre=CYCLE["mg_pre"], post=CYCLE["mg_post"])
        gbs = ab * ks / (ms * 1e-3) / 1e9 if ms > 0 else None
        classes[cls] = {"launches_per_step": nl / ks, "expected_launches_per_step": al,
                        "ms_per_step": ms / ks, "avg_launch_us": 1e3 * ms / max(nl, 1),
                        "algorithmic_bytes_per_step": ab, "GBps": gbs,
                        "frac": gbs / HBM_PEAK_GBS if gbs else None}
    sp = classes["spmv"]
    ab, al = algorithmic_bytes("spmv", b, n, per_cycle, "fp64")
    avg_ms = sp["ms_per_step"] / max(sp["launches_per_step"], 1)
    achieved = (ab / al) / (avg_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "spmv_traffic.json")
    if os.path.exists(tfile):
        info = json.load(open(tfile))
        if info.get("workload_cells") == n and info.get("source_sha") == _kernel_sha("spmv"):
            traffic = info.get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": "spmv_kernel<3>" if (b == 3 and n > (1 << 20)) else "spmv",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic, "launches_sampled": int(sp["launches_per_step"] * ks),
                "avg_launch_us": avg_ms * 1e3, "algorithmic_bytes_per_launch": ab / al,
                "timing": f"HIP events around every SpMV launch on the library's stream during {ks} extra "
                          "FP64 Newton steps identical to the timed ones"}
    triad, copy = measured_bandwidth()
    roofline.update(measured_triad_GBps=triad, measured_copy_GBps=copy, frac_of_measured_triad=achieved / triad)
    for v in classes.values():
        v["frac_of_measured_triad"] = v["GBps"] / triad if v["GBps"] else None
    class_bytes = sum(v["algorithmic_bytes_per_step"] for v in classes.values())
    solve_gbps = class_bytes / (phases["solve"] * 1e-3) / 1e9
    run = None
    solver.close()
    torch.cuda.empty_cache()

    network = network_timing(nx, ny, nz) if (b == 3 and nx % 8 == 0 and ny % 8 == 0 and nz % 8 == 0) else None
    configs = other_configs() if not (args.no_variants or args.no_other_configs) else {}

    cpu = cpu_baseline_value(sample, n, st["iterations"], class_bytes) if sample else None
    out = {
        "metric": METRIC, "value": sec, "unit": "s/Newton step", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{case['name']} ({n} cells, {b}x{b} blocks), one Newton step, FGMRES(30) to 1e-6, "
                               "plain FP64 CPR",
                   "cells": n, "block": b, "precision": "fp64", "restart": 30, "rtol": 1e-6, "dt_days": case["dt"],
                   "preconditioner": "quasi-IMPES CPR, P-then-F, aggregation multigrid V(2,2) with red-black "
                                     "Gauss-Seidel, coarse correction scaled by 1.25, coarsest <= 512 cells, "
                                     "red-black block ILU(0)"},
        "median_ms_per_step": 1e3 * float(np.median(host_times)),
        "fgmres_iterations": st["iterations"], "restart_cycles": st["cycles"], "true_rel": st["true_rel"],
        "phases_ms": phases, "solve_class_bytes_GBps": solve_gbps, "roofline": roofline,
        "kernel_classes": classes, "cpu_baseline": cpu, "variants": variants, "network": network,
        "other_configs": configs,
    }
    print(json.dumps(out))


def kernel_only(run, kclass, n, b):
    """Assemble once, then 20 SpMV launches and one copy of the state
    vector (the calibration transfer for the memory counters); or, for
    'ilu', ten CPR applications of each of the four forms (red-black and
    tiled ILU order, FP64 and FP32) with the benchmark's cycle, then the
    same calibration copy; for 'orth', one full FGMRES(30) cycle in FP64
    (rtol 0) and the copy."""
    import torch
    s = run.s
    rhs = s.assemble(run.x_old, run.x, run.case["dt"])
    if kclass == "orth":
        s.setup(precision="fp64", rtol=0.0, max_iter=30, **CYCLE)
        _, st = s.solve(rhs)
        torch.cuda.synchronize()
        cp = torch.empty_like(rhs)
        cp.copy_(rhs)
        torch.cuda.synchronize()
        return {"kernel": kclass, "arnoldi_steps": st["iterations"], "cells": n, "copy_bytes": rhs.numel() * 8,
                "source_sha": _kernel_sha(kclass)}
    if kclass == "ilu":
        v = rhs / torch.linalg.vector_norm(rhs)
        z = torch.empty_like(v)
        forms = [(p, o) for p in ("fp64", "mixed") for o in ("red-black", "tiles")]
        for prec, order in forms:
            s.setup(precision=prec, ilu_order=order, **CYCLE)
            for _ in range(10):
                s.precond(v, z)
            torch.cuda.synchronize()
        cp = torch.empty_like(rhs)
        cp.copy_(rhs)
        torch.cuda.synchronize()
        return {"kernel": kclass, "forms": [f"{p} {o}" for p, o in forms], "applications": 10, "cells": n,
                "copy_bytes": rhs.numel() * 8, "source_sha": _kernel_sha(kclass)}
    xin = torch.randn_like(rhs)
    y = torch.empty_like(rhs)
    for _ in range(20):
        s.spmv(xin, y)
    cp = torch.empty_like(rhs)
    cp.copy_(rhs)
    torch.cuda.synchronize()
    return {"kernel": kclass, "launches": 20, "cells": n, "copy_bytes": rhs.numel() * 8,
            "source_sha": _kernel_sha(kclass)}


def _kernel_sha(kclass):
    import hashlib
    f = {"spmv": "spmv.hip", "orth": "krylov.hip", "ilu": "apply.hip"}[kclass]
    p = os.path.join(ROOT, "paper_1606_00548_amd", "csrc", f)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def other_configs(steps=2):
    """The other workloads, each timed per Newton step from the same state
    with the same cycle as the headline (and the library's default V(1,1)
    beside it): the layered 128x128x32 black oil (FP64, mixed, mixed +
    learned; plus one whole backward-Euler day by time stepping), the
    oil-water 32x32x8 system (latency regime) and the first system of the
    channelised 256x256x64 black-oil 10-day step."""
    import numpy as np
    import torch
    from paper_1606_00548_amd import cprmi, synth, train
    out = {}
    wfile = train.weights_path("black-oil")
    for name, make, learned in (
            ("black-oil layered 128x128x32", lambda: synth.black_oil_layered(), True),
            ("oil-water 32x32x8", lambda: synth.oil_water_lognormal(), False),
            ("black-oil channelised 256x256x64, first system of the 10-day step",
             lambda: synth.black_oil_channelised(), False)):
        case = make()
        s = cprmi.Solver.from_case(case)
        run = Stepper(s, case)
        res = {"cells": int(np.prod(case["x"].shape[1:])), "block": int(case["x"].shape[0])}
        forms = [("fp64", dict(precision="fp64", **CYCLE)), ("mixed", dict(precision="mixed", **CYCLE)),
                 ("fp64 tiled ILU", dict(precision="fp64", ilu_order="tiles", **CYCLE)),
                 ("mixed tiled ILU", dict(precision="mixed", ilu_order="tiles", **CYCLE)),
                 ("fp64 V(1,1) alpha 1", dict(precision="fp64")),
                 ("mixed V(1,1) alpha 1", dict(precision="mixed"))]
        if learned and os.path.exists(wfile):
            s.attach_network(np.load(wfile))
            forms.insert(2, ("mixed+learned", dict(precision="mixed", learned=1, **CYCLE)))
        dx64 = None
        for prec, kw in forms:
            sp, _, sts, dx, _ = run.timed(cprmi.default_options(**kw), steps, 1)
            if prec == "fp64":
                dx64 = dx.clone()
            res[prec] = {"ms_per_step": 1e3 * sp, "iterations": sts[-1]["iterations"],
                         "true_rel": sts[-1]["true_rel"], "rel_diff_vs_fp64": _rel(dx, dx64)}
        if learned and os.path.exists(wfile):
            # one backward-Euler day: a single 1-day step (with its cuts) and
            # the same day by time stepping from 0.01 day with growth
            for prec, kw in (("fp64", dict(precision="fp64", **CYCLE)),
                             ("fp64 tiled ILU", dict(precision="fp64", ilu_order="tiles", **CYCLE)),
                             ("mixed+learned", dict(precision="mixed", learned=1, **CYCLE))):
                lo = cprmi.default_options(**kw)
                xts = torch.empty_like(run.x0)
                s.time_step(run.x_old, case["dt"], options=lo, x=xts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, tst = s.time_step(run.x_old, case["dt"], options=lo, x=xts)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, sst = s.simulate(run.x_old, case["dt"], 0.01, case["dt"], options=lo, x=xts)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                res[f"time_step {prec}"] = {"s": t1 - t0, "cuts": tst["cuts"], "total_newton": tst["total_newton"],
                                            "total_linear": tst["total_linear"], "converged": bool(tst["converged"])}
                res[f"simulation {prec}"] = {"s": t2 - t1, "steps": sst["steps"], "cuts": sst["cuts"],
                                             "total_newton": sst["total_newton"], "total_linear": sst["total_linear"],
                                             "completed": bool(sst["completed"])}
        if name.startswith("black-oil channelised"):
            try:
                res["newton_iterations_mixed_vs_fp64"] = newton_iterations_mixed_vs_fp64(s, case)
            except cprmi.CPRError as e:
                res["newton_iterations_mixed_vs_fp64"] = {"error": str(e)}
        s.attach_network(None)
        run = None
        s.close()
        torch.cuda.empty_cache()
        out[name] = res
    return out


if __name__ == "__main__":
    main()
