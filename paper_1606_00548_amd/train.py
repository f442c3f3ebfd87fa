"""Training data, training and evaluation of the pressure-correction network.

All arithmetic runs in libcprmi.so; this module only orchestrates calls and
keeps tensors in GPU memory.

Data: for each synthetic system of a reservoir family (oil-water or black
oil) the solver assembles its Newton system, sets up CPR and runs a fixed
number of FGMRES iterations; for each Krylov vector v_j it runs the
pressure stage alone to get the residual the multigrid cycle leaves,
r' = r~_p - A_p dp_mg, and the network input for it.  The
target is the exact remaining correction A_p^-1 r', obtained with the same
library by solving the pressure system to 1e-10 (A_p embedded as the
pressure block of a two-unknown system whose second unknown is decoupled
by an identity block), divided by the feature scale s.  The network learns
only the direction of that correction: the loss is 1 - cos^2(N(input), t),
and inside the solver the step length comes from the residual-minimising
alpha = <A_p d, r'> / |A_p d|^2 for d = N(input), judged against plain CPR.

With --level l the same is done for the learned stage inside the cycle on
multigrid level l: r' is the residual the cycle leaves on that level after
its post-smoothing, the features are those of the level (block means of
ln k and ln lambda_t), and the target solves with the level's operator.
"""
import argparse
import json
import os
import time

import numpy as np
import torch

from . import cprmi, synth

WEIGHT_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")

# Training and evaluation systems per reservoir family: generator, training
# grid, evaluation generator and grid, first evaluation seed.
FAMILIES = {
    "oil-water": {"train": synth.oil_water_training, "shape": (64, 64, 32),
                  "eval": synth.oil_water_eval, "eval_shape": (128, 128, 64), "seed0": 5000, "eval_seed0": 6000},
    "black-oil": {"train": synth.black_oil_training, "shape": (64, 64, 32),
                  "eval": synth.black_oil_layered, "eval_shape": (128, 128, 32), "seed0": 7000, "eval_seed0": 2000},
}
# A network for a coarse multigrid level: trained on level-l residuals of
# larger systems (level 2 of 256 x 256 x 64 is 64 x 64 x 16) with fields
# around the lattice workload's, evaluated where that level is the automatic
# choice (level 2 of the 512 x 512 x 128 lattice, a seed outside training).
LEVEL_TRAINING = {"black-oil": {"train": synth.black_oil_lattice_training, "shape": (256, 256, 64), "seed0": 5100,
                                "eval": synth.black_oil_lattice, "eval_shape": (512, 512, 128), "eval_seed0": 5000}}


def weights_path(family, level=0):
    """Shipped parameters of the network trained for a family, on the fine
    pressure residual (level 0) or on the residual the multigrid cycle
    leaves on level `level` (see harvest)."""
    tag = "" if level == 0 else f"_level{level}"
    return os.path.join(WEIGHT_DIR, f"pressure_unet_{family.replace('-', '_')}{tag}.npy")


def weights_for_level(family, level):
    """The parameters to attach for a learned stage on `level`: the network
    trained for that level if one is shipped, else the fine-level one."""
    p = weights_path(family, level)
    return p if os.path.exists(p) else weights_path(family)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


class PressureTarget:
    """Solves A e = r' for the exact remaining pressure correction, A a
    scalar 7-point operator on an nx x ny x nz grid (the fine pressure matrix
    or a multigrid level's operator)."""

    def __init__(self, nx, ny, nz):
        shape = (nz, ny, nx)
        perm = np.ones((3,) + shape)
        self.s = cprmi.Solver(synth.grid_of(nx, ny, nz), synth.OIL_WATER, perm, np.full(shape, 0.2), [])
        self.shape = self.s.shape

    def load(self, Ap):
        J2 = torch.zeros((7, 2, 2) + self.shape, dtype=torch.float64, device="cuda")
        J2[:, 0, 0] = Ap
        J2[0, 1, 1] = 1.0
        self.s.import_jacobian(J2.contiguous())
        self.s.setup(rtol=1e-10, max_iter=600)

    def solve(self, rprime):
        rhs = torch.zeros((2,) + self.shape, dtype=torch.float64, device="cuda")
        rhs[0] = rprime
        dx, st = self.s.solve(rhs.contiguous())
        return dx[0].clone(), st


def harvest(case, per_system, cycle=None, level=0):
    """(features [k, nz, ny, nx, 3] float32, targets [k, nz, ny, nx] float32)
    for the first k = per_system (<= 30) Krylov vectors of the system.
    cycle: multigrid options (mg_pre, mg_post, mg_alpha) of the pressure
    stage whose residuals are harvested (default V(1,1), alpha 1).  level:
    0 for the fine residual after the cycle, l >= 1 for the residual the
    cycle leaves on multigrid level l after its post-smoothing (features and
    targets then live on that level's grid)."""
    s = cprmi.Solver.from_case(case)
    rhs = s.assemble(_dev(case["x_old"]), _dev(case["x"]), case["dt"])
    s.setup(rtol=0.0, max_iter=min(per_system, 30), nn_level=level, **(cycle or {}))
    _, st = s.solve(rhs)
    k = min(per_system, st["iterations"], 30)
    nz, ny, nx = s.mg_level_shape(level)
    tgt = PressureTarget(nx, ny, nz)
    tgt.load(s.export_mg_level(level))
    feats, targets = [], []
    for j in range(k):
        v = s.export_krylov(j)
        rp, _ = s.pressure_stage(v)
        f, scale = s.features(rp)
        if not scale > 0:
            continue
        e, tst = tgt.solve(rp)
        feats.append(f)
        targets.append(cprmi.make_target(e, scale))
    s.close()
    tgt.s.close()
    return torch.stack(feats), torch.stack(targets)


def make_dataset(n_systems, per_system, shape=(64, 64, 32), seed0=5000, log=print, family="oil-water",
                 cycle=None, level=0, gen=None):
    nx, ny, nz = shape
    gen = gen or FAMILIES[family]["train"]
    X, T = [], []
    t0 = time.time()
    for i in range(n_systems):
        case = gen(nx, ny, nz, seed=seed0 + i)
        f, t = harvest(case, per_system, cycle, level)
        X.append(f)
        T.append(t)
        if log and (i + 1) % max(1, n_systems // 10) == 0:
            log(f"[data] {i + 1}/{n_systems} systems, {sum(x.shape[0] for x in X)} pairs, "
                f"{time.time() - t0:.1f} s")
    return torch.cat(X).contiguous(), torch.cat(T).contiguous()


def _sha256(path):
    import hashlib
    h = hashlib.sha256()
    with open(path, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()


def save_checkpoint(path, state, meta):
    """Write a training checkpoint: `state` (parameters theta, Adam moments
    m and v, adam_step, the finished epoch, the shuffling generator's state
    and the loss history) as one .npz of plain arrays (nothing pickled), and
    beside it <path>.json with the training configuration `meta` and the
    file's SHA-256."""
    assert path.endswith(".npz")
    np.savez(path, theta=state["theta"], m=state["m"], v=state["v"], adam_step=np.int64(state["adam_step"]),
             epoch=np.int64(state["epoch"]), rng_state=np.array(json.dumps(state["rng_state"])),
             history=np.array(json.dumps(state["history"])))
    with open(path[:-4] + ".json", "w") as f:
        json.dump(dict(meta, epoch=int(state["epoch"]), sha256=_sha256(path)), f, indent=1)


def load_checkpoint(path):
    """Read a checkpoint written by save_checkpoint after checking its
    SHA-256 against the one recorded beside it (ValueError if they differ)."""
    with open(path[:-4] + ".json") as f:
        meta = json.load(f)
    if _sha256(path) != meta["sha256"]:
        raise ValueError(f"{path}: SHA-256 does not match {path[:-4]}.json")
    with np.load(path, allow_pickle=False) as z:
        return {"theta": z["theta"], "m": z["m"], "v": z["v"], "adam_step": int(z["adam_step"]),
                "epoch": int(z["epoch"]), "rng_state": json.loads(str(z["rng_state"])),
                "history": json.loads(str(z["history"])), "meta": meta}


def train(X, T, epochs, batch=4, lr=1e-3, seed=0, val_frac=0.1, init_seed=1, log=print,
          checkpoint=None, resume=None):
    """Adam on the normalised MSE; returns (parameters, history).
    checkpoint: .npz path rewritten after every epoch (save_checkpoint);
    resume: a checkpoint of a run with the same data and arguments to
    continue from its last finished epoch -- parameters, Adam moments and
    step count, and the shuffling generator are restored, so the resumed run
    reproduces the uninterrupted one."""
    n = X.shape[0]
    nz, ny, nx = X.shape[1:4]
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    nval = max(1, int(round(val_frac * n)))
    val, tr = order[:nval], order[nval:]
    net = cprmi.Network(nx, ny, nz, max_batch=batch)
    net.set_params(synth.nn_initial_weights(init_seed))
    hist = []
    start = 0
    if resume:
        ck = load_checkpoint(resume)
        net.set_params(ck["theta"])
        net.set_adam(ck["m"], ck["v"], ck["adam_step"])
        rng.bit_generator.state = ck["rng_state"]
        hist, start = ck["history"], ck["epoch"]
        if log:
            log(f"[train] resumed after epoch {start} from {resume}")
    meta = {"samples": int(n), "grid": [nx, ny, nz], "epochs": epochs, "batch": batch, "lr": lr, "seed": seed,
            "val_frac": val_frac, "init_seed": init_seed}
    t0 = time.time()
    for ep in range(start, epochs):
        perm = rng.permutation(tr)
        losses = []
        for q in range(0, len(perm) - batch + 1, batch):
            idx = torch.as_tensor(perm[q:q + batch], device="cuda")
            losses.append(net.train_step(X[idx].contiguous(), T[idx].contiguous(), lr))
        vl = validation_loss(net, X, T, val, batch)
        hist.append({"epoch": ep + 1, "train_loss": float(np.mean(losses)), "val_loss": vl,
                     "seconds": time.time() - t0})
        if log:
            log(f"[train] epoch {ep + 1}: train {np.mean(losses):.4f}, validation {vl:.4f}, "
                f"{time.time() - t0:.1f} s")
        if checkpoint:
            m, v, k = net.get_adam()
            save_checkpoint(checkpoint, {"theta": net.get_params(), "m": m, "v": v, "adam_step": k,
                                         "epoch": ep + 1, "rng_state": rng.bit_generator.state,
                                         "history": hist}, meta)
    theta = net.get_params()
    net.close()
    return theta, hist


def validation_loss(net, X, T, idx, batch):
    """Mean normalised MSE over the validation samples (one sample per call,
    so every sample weighs the same)."""
    tot = []
    for q in idx:
        sel = torch.as_tensor([q], device="cuda")
        tot.append(net.eval_loss(X[sel].contiguous(), T[sel].contiguous()))
    return float(np.mean(tot))


def evaluate(theta, seeds, shape=(128, 128, 64), control_seed=99, log=print, family="oil-water",
             precision="fp64", cycle=None, level=0, gen=None):
    """FGMRES iterations and solve time to 1e-6 on evaluation systems: plain
    CPR, CPR with the trained network, CPR with a random-init network (all
    with the multigrid options `cycle`, the learned stage on `level`)."""
    nx, ny, nz = shape
    gen = gen or FAMILIES[family]["eval"]
    rows = []
    for sd in seeds:
        case = gen(nx, ny, nz, seed=sd)
        s = cprmi.Solver.from_case(case)
        rhs = s.assemble(_dev(case["x_old"]), _dev(case["x"]), case["dt"])
        row = {"seed": sd}
        for name, th in (("plain", None), ("learned", theta),
                         ("random", synth.nn_initial_weights(control_seed))):
            if th is not None:
                s.attach_network(th)
            s.setup(learned=0 if th is None else 1, precision=precision, nn_level=level, **(cycle or {}))
            s.solve(rhs)                       # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = s.solve(rhs)
            torch.cuda.synchronize()
            row[name] = {"iterations": st["iterations"], "seconds": time.perf_counter() - t0,
                         "true_rel": st["true_rel"], "accepted": st["nn_accepted"],
                         "rejected": st["nn_rejected"]}
        s.close()
        rows.append(row)
        if log:
            log(f"[eval] seed {sd}: " + ", ".join(
                f"{k} {row[k]['iterations']} its {1e3 * row[k]['seconds']:.2f} ms "
                f"(acc {row[k]['accepted']})" for k in ("plain", "learned", "random")))
    return rows


def main():
    ap = argparse.ArgumentParser(description="train and evaluate the pressure-correction network")
    ap.add_argument("--family", default="black-oil", choices=sorted(FAMILIES))
    ap.add_argument("--systems", type=int, default=100)
    ap.add_argument("--per-system", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-seeds", type=int, default=8)
    ap.add_argument("--out", default=None, help="parameter file (default: the family's shipped file)")
    ap.add_argument("--report", default=None)
    ap.add_argument("--checkpoint", default=None, help="training checkpoint (.npz) rewritten every epoch")
    ap.add_argument("--resume", default=None, help="checkpoint (.npz) to continue training from")
    ap.add_argument("--mg-pre", type=int, default=1, help="pre-smoothing sweeps of the cycle trained for")
    ap.add_argument("--mg-post", type=int, default=1, help="post-smoothing sweeps of the cycle trained for")
    ap.add_argument("--mg-alpha", type=float, default=1.0, help="coarse-correction scaling of that cycle")
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the parameters in --out (default: the shipped file) without training")
    ap.add_argument("--level", type=int, default=0,
                    help="multigrid level whose residuals the network is trained on (0: the fine residual)")
    args = ap.parse_args()
    fam = dict(FAMILIES[args.family])
    if args.level > 0:
        fam.update(LEVEL_TRAINING[args.family])
    out = args.out or weights_path(args.family, args.level)
    cycle = {"mg_pre": args.mg_pre, "mg_post": args.mg_post, "mg_alpha": args.mg_alpha}
    eval_kw = dict(family=args.family, cycle=cycle, level=args.level, gen=fam["eval"],
                   log=lambda m: print(m, flush=True))
    if args.eval_only:
        theta = np.load(out)
        ex, ey, ez = fam["eval_shape"]
        rows = []
        for prec in ("fp64", "mixed"):
            rows += [dict(r, precision=prec) for r in evaluate(
                theta, [fam["eval_seed0"] + i for i in range(args.eval_seeds)], shape=(ex, ey, ez),
                precision=prec, **eval_kw)]
        if args.report:
            with open(args.report, "w") as f:
                json.dump({"family": args.family, "weights": os.path.basename(out), "cycle": cycle,
                           "level": args.level, "eval": rows}, f, indent=1)
        return
    X, T = make_dataset(args.systems, args.per_system, fam["shape"], fam["seed0"], family=args.family,
                        log=lambda m: print(m, flush=True), cycle=cycle, level=args.level, gen=fam["train"])
    pairs = int(X.shape[0])
    print(f"[data] {pairs} pairs", flush=True)
    theta, hist = train(X, T, args.epochs, lr=args.lr, log=lambda m: print(m, flush=True),
                        checkpoint=args.checkpoint, resume=args.resume)
    del X, T
    torch.cuda.empty_cache()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.save(out, theta)
    nx, ny, nz = fam["shape"]
    where = ("the pressure residuals after the multigrid cycle" if args.level == 0 else
             f"the residuals the multigrid cycle leaves on level {args.level} after its post-smoothing")
    meta = {
        "family": args.family,
        "network": "3-D U-Net, channels (16, 32, 64, 64), one 3x3x3 convolution per level and path, ReLU, "
                   "avg-pool / nearest-upsample, additive skips, 1x1x1 head",
        "parameters": int(theta.size),
        "dtype": "float32 master (BF16 in the convolutions)",
        "data": f"{args.systems} {args.family} systems {nx}x{ny}x{nz} ({fam['train'].__module__}."
                f"{fam['train'].__name__} seeds {fam['seed0']}-{fam['seed0'] + args.systems - 1}), "
                f"{where} for the first {args.per_system} Krylov vectors of each; targets A^-1 r' / "
                f"rms(D^-1 r') from a 1e-10 solve with that level's operator A",
        "level": args.level,
        "pairs": pairs, "epochs": args.epochs, "batch": 4,
        "optimizer": f"Adam lr {args.lr:g} (0.9, 0.999, 1e-8)", "init_seed": 1, "shuffle_seed": 0,
        "loss": "direction loss 1 - cos^2(N(x), t)", "cycle": cycle, "history": hist,
    }
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    ex, ey, ez = fam["eval_shape"]
    rows = []
    for prec in ("fp64", "mixed"):
        rows += [dict(r, precision=prec) for r in evaluate(
            theta, [fam["eval_seed0"] + i for i in range(args.eval_seeds)], shape=(ex, ey, ez),
            precision=prec, **eval_kw)]
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"family": args.family, "cycle": cycle, "level": args.level, "history": hist, "eval": rows},
                      f, indent=1)


if __name__ == "__main__":
    main()
