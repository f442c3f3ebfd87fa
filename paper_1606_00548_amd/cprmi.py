"""Python binding of the C ABI in include/cprmi.h (ctypes; marshalling only).

Every array is a torch tensor on the GPU (float64, contiguous, natural cell
order [b][nz][ny][nx]); torch provides device memory and the HIP stream, and
all arithmetic happens in libcprmi.so.  Importing this module loads torch
first so that the library binds to the HIP runtime torch already mapped.
The library must have been built (`python -m paper_1606_00548_amd.build`);
without it every entry point raises.
"""
import ctypes
import json
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcprmi.so")
_lib = None

CPR_OK, CPR_NOT_CONVERGED = 0, 1
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESINGULAR", -5: "ENONFINITE",
          -6: "EBREAKDOWN"}
PREC = {"fp64": 0, "mixed": 1}
DECOUPLING = {"qimpes": 0, "abf": 1}
COMPOSITION = {"two-stage": 0, "fpf": 1}
ORTH = {"dcgs2": 0, "cgs2": 1}
ILU_ORDER = {"red-black": 0, "tiles": 1}


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("top", ctypes.c_double)]


class Fluid(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("p_ref", ctypes.c_double),
                ("rho_w_ref", ctypes.c_double), ("rho_o_ref", ctypes.c_double),
                ("rho_o_sc", ctypes.c_double), ("rho_g_sc", ctypes.c_double),
                ("c_w", ctypes.c_double), ("c_o", ctypes.c_double), ("c_r", ctypes.c_double),
                ("mu_w", ctypes.c_double), ("mu_o", ctypes.c_double),
                ("s_wc", ctypes.c_double), ("s_or", ctypes.c_double), ("sg_den", ctypes.c_double),
                ("n_pvt", ctypes.c_int), ("pvt", ctypes.POINTER(ctypes.c_double))]


class Well(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int), ("j", ctypes.c_int), ("k0", ctypes.c_int), ("k1", ctypes.c_int),
                ("kind", ctypes.c_int), ("bhp", ctypes.c_double), ("rw", ctypes.c_double),
                ("skin", ctypes.c_double), ("control", ctypes.c_int), ("rate", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("learned", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double), ("mg_coarsest", ctypes.c_int),
                ("mg_alpha", ctypes.c_double), ("decoupling", ctypes.c_int), ("composition", ctypes.c_int),
                ("x0", ctypes.c_int), ("mg_pre", ctypes.c_int), ("mg_post", ctypes.c_int),
                ("stall_ratio", ctypes.c_double), ("orth", ctypes.c_int), ("nn_level", ctypes.c_int),
                ("ilu_order", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("cycles", ctypes.c_int), ("converged", ctypes.c_int),
                ("mg_levels", ctypes.c_int), ("qimpes_fallback", ctypes.c_int),
                ("nn_accepted", ctypes.c_int), ("nn_rejected", ctypes.c_int),
                ("bnorm", ctypes.c_double), ("est_rel", ctypes.c_double),
                ("true_rel", ctypes.c_double), ("fp64_fallback", ctypes.c_int),
                ("ms_assemble", ctypes.c_double), ("ms_setup", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("ms_precond", ctypes.c_double), ("ms_spmv", ctypes.c_double), ("ms_orth", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


NEWTON_HIST = 64
FORCING = {"fixed": 0, "ew1": 1, "ew2": 2, "ew3": 3}
KRYLOV = {"fgmres": 0, "bicgstab": 1}


class NewtonOptions(ctypes.Structure):
    _fields_ = [("forcing", ctypes.c_int), ("krylov", ctypes.c_int), ("max_newton", ctypes.c_int),
                ("max_cuts", ctypes.c_int), ("newton_tol", ctypes.c_double), ("theta0", ctypes.c_double),
                ("theta_min", ctypes.c_double), ("theta_max", ctypes.c_double), ("gamma", ctypes.c_double),
                ("beta", ctypes.c_double)]


class NewtonStats(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("cuts", ctypes.c_int), ("newton_iterations", ctypes.c_int),
                ("linear_iterations", ctypes.c_int), ("total_newton", ctypes.c_int),
                ("total_linear", ctypes.c_int), ("dt_taken", ctypes.c_double),
                ("theta", ctypes.c_double * NEWTON_HIST), ("lin_its", ctypes.c_int * NEWTON_HIST),
                ("bnorm", ctypes.c_double * (NEWTON_HIST + 1))]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_[:7]}
        k = min(self.newton_iterations, NEWTON_HIST)
        d["history"] = {"theta": list(self.theta[:k]), "linear_iterations": list(self.lin_its[:k]),
                        "bnorm": list(self.bnorm[:k + 1])}
        return d


SIM_HIST = 256


class SimStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int), ("steps", ctypes.c_int), ("cuts", ctypes.c_int),
                ("total_newton", ctypes.c_int), ("total_linear", ctypes.c_int), ("t_reached", ctypes.c_double),
                ("dts", ctypes.c_double * SIM_HIST), ("seconds", ctypes.c_double),
                ("step_newton", ctypes.c_int * SIM_HIST), ("step_linear", ctypes.c_int * SIM_HIST),
                ("step_cuts", ctypes.c_int * SIM_HIST), ("step_seconds", ctypes.c_double * SIM_HIST)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_[:6]}
        k = min(self.steps, SIM_HIST)
        d["dts"] = list(self.dts[:k])
        d["seconds"] = self.seconds
        for f in ("step_newton", "step_linear", "step_cuts", "step_seconds"):
            d[f] = list(getattr(self, f)[:k])
        return d


def paper_table(stats):
    """The columns of the paper's result tables (Sec. 4) for a simulate()
    run: steps, Newton iterations, linear-solver iterations, linear
    iterations per Newton iteration, wall time and wall time per Newton
    iteration (seconds)."""
    newton = stats["total_newton"]
    return {"steps": stats["steps"], "newton": newton, "solver": stats["total_linear"],
            "avg_solver": stats["total_linear"] / newton if newton else None,
            "time_s": stats["seconds"], "avg_time_s": stats["seconds"] / newton if newton else None}


def write_jsonl(path, stats):
    """One JSON line per accepted time step of a simulate() run (time,
    step size, Newton and linear iterations, cuts, wall time), then one line
    with the run's paper_table() columns."""
    t = 0.0
    with open(path, "w") as f:
        for i, dt in enumerate(stats["dts"]):
            t += dt
            f.write(json.dumps({"step": i + 1, "t_days": t, "dt_days": dt, "newton": stats["step_newton"][i],
                                "solver": stats["step_linear"][i], "cuts": stats["step_cuts"][i],
                                "seconds": stats["step_seconds"][i]}) + "\n")
        f.write(json.dumps(dict(paper_table(stats), completed=bool(stats["completed"]),
                                t_reached_days=stats["t_reached"])) + "\n")


EXPORTS = ["cpr_default_options", "cpr_create", "cpr_destroy", "cpr_last_error", "cpr_block_size",
           "cpr_num_cells", "assemble_jacobian", "cpr_import_jacobian", "cpr_export_jacobian",
           "cpr_setup", "cpr_gmres_solve", "cpr_newton_update", "cpr_spmv", "cpr_precond_apply",
           "cpr_export_qimpes", "cpr_mg_level_shape", "cpr_nn_level", "cpr_export_mg_level", "cpr_export_ilu",
           "cpr_profile_kernel", "cpr_profile_read", "cpr_set_timing", "cpr_nn_num_params", "cpr_nn_create",
           "cpr_nn_destroy", "cpr_nn_last_error", "cpr_nn_set_params", "cpr_nn_get_params",
           "cpr_nn_forward", "cpr_nn_backward", "cpr_nn_train_step", "cpr_nn_attach",
           "cpr_pressure_stage", "cpr_nn_features", "cpr_export_krylov", "cpr_nn_eval_loss",
           "cpr_nn_make_target", "cpr_nn_infer", "cpr_bicgstab_solve", "cpr_default_newton_options",
           "cpr_time_step", "cpr_simulate", "cpr_num_unknowns", "cpr_set_allocator", "cpr_nn_get_adam",
           "cpr_nn_set_adam", "cpr_spmv_noalloc", "cpr_spmv_noalloc_max_unknowns"]
KCLASS = {"spmv": 0, "orth": 1, "smooth": 2, "ilu": 3, "assemble": 4}


def load():
    """Load libcprmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with python -m paper_1606_00548_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.cpr_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.cpr_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fluid), P, P, ctypes.POINTER(Well),
                               ctypes.c_int, P, ctypes.POINTER(P)]
    lib.cpr_destroy.argtypes = [P]
    lib.cpr_last_error.argtypes = [P]
    lib.cpr_last_error.restype = ctypes.c_char_p
    lib.cpr_block_size.argtypes = [P]
    lib.cpr_num_cells.argtypes = [P]
    lib.cpr_num_cells.restype = ctypes.c_longlong
    lib.cpr_num_unknowns.argtypes = [P]
    lib.cpr_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
    lib.cpr_num_unknowns.restype = ctypes.c_longlong
    lib.assemble_jacobian.argtypes = [P, P, P, ctypes.c_double, P]
    lib.cpr_import_jacobian.argtypes = [P, P]
    lib.cpr_export_jacobian.argtypes = [P, P]
    lib.cpr_setup.argtypes = [P, ctypes.POINTER(Options)]
    lib.cpr_gmres_solve.argtypes = [P, P, P, ctypes.POINTER(Stats)]
    lib.cpr_bicgstab_solve.argtypes = [P, P, P, ctypes.POINTER(Stats)]
    lib.cpr_default_newton_options.argtypes = [ctypes.POINTER(NewtonOptions)]
    lib.cpr_simulate.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(Options), ctypes.POINTER(NewtonOptions), ctypes.POINTER(SimStats)]
    lib.cpr_time_step.argtypes = [P, P, P, ctypes.c_double, ctypes.POINTER(Options),
                                  ctypes.POINTER(NewtonOptions), ctypes.POINTER(NewtonStats)]
    lib.cpr_newton_update.argtypes = [P, P, P]
    lib.cpr_spmv.argtypes = [P, P, P]
    lib.cpr_precond_apply.argtypes = [P, P, P]
    lib.cpr_spmv_noalloc.argtypes = [P, P, P]
    lib.cpr_spmv_noalloc_max_unknowns.restype = ctypes.c_longlong
    lib.cpr_export_qimpes.argtypes = [P, P]
    lib.cpr_mg_level_shape.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.cpr_export_mg_level.argtypes = [P, ctypes.c_int, P]
    lib.cpr_nn_level.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.cpr_export_ilu.argtypes = [P, P]
    lib.cpr_profile_kernel.argtypes = [P, ctypes.c_int]
    lib.cpr_set_timing.argtypes = [P, ctypes.c_int]
    lib.cpr_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    lib.cpr_nn_num_params.restype = ctypes.c_longlong
    lib.cpr_nn_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.POINTER(P)]
    lib.cpr_nn_destroy.argtypes = [P]
    lib.cpr_nn_last_error.argtypes = [P]
    lib.cpr_nn_last_error.restype = ctypes.c_char_p
    lib.cpr_nn_set_params.argtypes = [P, P]
    lib.cpr_nn_get_params.argtypes = [P, P]
    lib.cpr_nn_get_adam.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_longlong)]
    lib.cpr_nn_set_adam.argtypes = [P, P, P, ctypes.c_longlong]
    lib.cpr_nn_forward.argtypes = [P, P, ctypes.c_int, P]
    lib.cpr_nn_infer.argtypes = [P, P, P]
    lib.cpr_nn_backward.argtypes = [P, P, P]
    lib.cpr_nn_train_step.argtypes = [P, P, P, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]
    lib.cpr_nn_attach.argtypes = [P, P]
    lib.cpr_pressure_stage.argtypes = [P, P, P, P]
    lib.cpr_nn_features.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_double)]
    lib.cpr_export_krylov.argtypes = [P, ctypes.c_int, P]
    lib.cpr_nn_eval_loss.argtypes = [P, P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    lib.cpr_nn_make_target.argtypes = [P, ctypes.c_longlong, ctypes.c_double, P, P]
    _lib = lib
    return lib


class CPRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t, dtype=torch.float64):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _fptr(t):
    return _ptr(t, torch.float32)


class Network:
    """The pressure-correction network (training and inference on the GPU)."""

    def __init__(self, nx, ny, nz, max_batch=1, stream=None):
        self.lib = load()
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.cpr_nn_create(nx, ny, nz, max_batch, ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h))
        self.h = h
        if rc != 0:
            msg = self.lib.cpr_nn_last_error(h).decode() if h.value else ""
            self.lib.cpr_nn_destroy(h)
            self.h = None
            raise CPRError(rc, msg)
        self.P = int(self.lib.cpr_nn_num_params())

    def _check(self, rc):
        if rc != 0:
            raise CPRError(rc, self.lib.cpr_nn_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.cpr_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == self.P
        self._check(self.lib.cpr_nn_set_params(self.h, th.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        th = np.empty(self.P, dtype=np.float32)
        self._check(self.lib.cpr_nn_get_params(self.h, th.ctypes.data_as(ctypes.c_void_p)))
        return th

    def get_adam(self):
        """(first moment, second moment, Adam steps taken)."""
        m = np.empty(self.P, dtype=np.float32)
        v = np.empty(self.P, dtype=np.float32)
        k = ctypes.c_longlong()
        self._check(self.lib.cpr_nn_get_adam(self.h, m.ctypes.data_as(ctypes.c_void_p),
                                             v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(k)))
        return m, v, int(k.value)

    def set_adam(self, m, v, step):
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        assert m.size == self.P and v.size == self.P
        self._check(self.lib.cpr_nn_set_adam(self.h, m.ctypes.data_as(ctypes.c_void_p),
                                             v.ctypes.data_as(ctypes.c_void_p), int(step)))

    def forward(self, x):
        """x: float32 CUDA tensor [B, nz, ny, nx, 3] -> y [B, nz, ny, nx]."""
        B = x.shape[0]
        y = torch.empty((B,) + self.shape, dtype=torch.float32, device="cuda")
        self._check(self.lib.cpr_nn_forward(self.h, _fptr(x), B, _fptr(y)))
        return y

    def infer(self, x):
        """Inference form for one sample: x [1, nz, ny, nx, 3] -> y [1, nz, ny, nx]."""
        assert x.shape[0] == 1
        y = torch.empty((1,) + self.shape, dtype=torch.float32, device="cuda")
        self._check(self.lib.cpr_nn_infer(self.h, _fptr(x), _fptr(y)))
        return y

    def backward(self, dy):
        g = torch.empty(self.P, dtype=torch.float32, device="cuda")
        self._check(self.lib.cpr_nn_backward(self.h, _fptr(dy), _fptr(g)))
        return g

    def eval_loss(self, x, t):
        loss = ctypes.c_float()
        self._check(self.lib.cpr_nn_eval_loss(self.h, _fptr(x), _fptr(t), x.shape[0], ctypes.byref(loss)))
        return float(loss.value)

    def train_step(self, x, t, lr=1e-3):
        loss = ctypes.c_float()
        self._check(self.lib.cpr_nn_train_step(self.h, _fptr(x), _fptr(t), x.shape[0], float(lr),
                                               ctypes.byref(loss)))
        return float(loss.value)


def default_options(**kw):
    o = Options()
    load().cpr_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PREC[v]
        if k == "decoupling" and isinstance(v, str):
            v = DECOUPLING[v]
        if k == "composition" and isinstance(v, str):
            v = COMPOSITION[v]
        if k == "orth" and isinstance(v, str):
            v = ORTH[v]
        if k == "ilu_order" and isinstance(v, str):
            v = ILU_ORDER[v]
        setattr(o, k, v)
    return o


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
# Every registered callback pair stays alive for the life of the process:
# contexts created under it return their memory through it when destroyed.
_allocators = []


def set_allocator(alloc=None, free=None):
    """Route the library's device memory through alloc(nbytes) -> int and
    free(ptr) (cpr_set_allocator); no arguments restore hipMalloc/hipFree.
    Contexts keep the allocator they were created with."""
    lib = load()
    if alloc is None:
        rc = lib.cpr_set_allocator(_ALLOC_FN(), _FREE_FN(), None)
    else:
        cb = (_ALLOC_FN(lambda n, user: alloc(n) or None), _FREE_FN(lambda p, user: free(p)))
        _allocators.append(cb)
        rc = lib.cpr_set_allocator(cb[0], cb[1], None)
    if rc != 0:
        raise CPRError(rc, "cpr_set_allocator")


def use_torch_allocator():
    """Let torch's caching allocator supply the library's device memory."""
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                  lambda p: torch.cuda.caching_allocator_delete(p))


def default_newton_options(**kw):
    o = NewtonOptions()
    load().cpr_default_newton_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "forcing" and isinstance(v, str):
            v = FORCING[v]
        if k == "krylov" and isinstance(v, str):
            v = KRYLOV[v]
        setattr(o, k, v)
    return o


class Solver:
    """One C-ABI context: grid, rock, fluid and wells of a reservoir model."""

    def __init__(self, grid, fluid, perm, poro, wells, stream=None):
        lib = load()
        self.lib = lib
        self.grid = grid
        self.b = {1: 1, 2: 2, 3: 3}[fluid["model"]]
        self.shape = (grid["nz"], grid["ny"], grid["nx"])
        g = Grid(grid["nx"], grid["ny"], grid["nz"], grid["dx"], grid["dy"], grid["dz"], grid["top"])
        f = Fluid()
        f.model = fluid["model"]
        for key in ["p_ref", "rho_w_ref", "rho_o_ref", "rho_o_sc", "rho_g_sc", "c_w", "c_o", "c_r",
                    "mu_w", "mu_o", "s_wc", "s_or", "sg_den"]:
            setattr(f, key, float(fluid.get(key, 0.0)))
        self._pvt = None
        if fluid["model"] == 3:
            self._pvt = np.ascontiguousarray(fluid["pvt"], dtype=np.float64)
            f.n_pvt = self._pvt.shape[1]
            f.pvt = self._pvt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ws = (Well * max(1, len(wells)))()
        for q, w in enumerate(wells):
            rate = w.get("control", "bhp") == "rate"
            ws[q] = Well(w["i"], w["j"], w["k0"], w["k1"], 0 if w["kind"] == "inj" else 1,
                         w["bhp"], w["rw"], w["skin"], 1 if rate else 0, float(w.get("rate", 0.0)))
        # rate-controlled wells append their BHPs to every vector
        self.nrate = sum(1 for w in wells if w.get("control", "bhp") == "rate")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        perm_t = torch.as_tensor(np.asarray(perm, dtype=np.float64)).cuda().contiguous() \
            if not isinstance(perm, torch.Tensor) else perm
        poro_t = torch.as_tensor(np.asarray(poro, dtype=np.float64)).cuda().contiguous() \
            if not isinstance(poro, torch.Tensor) else poro
        ctx = ctypes.c_void_p()
        with torch.cuda.stream(self.stream):
            rc = lib.cpr_create(ctypes.byref(g), ctypes.byref(f), _ptr(perm_t), _ptr(poro_t), ws,
                                len(wells), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        self.ctx = ctx
        if rc != 0:
            msg = lib.cpr_last_error(ctx).decode() if ctx.value else ""
            lib.cpr_destroy(ctx)
            self.ctx = None
            raise CPRError(rc, msg)

    @classmethod
    def from_case(cls, case, stream=None):
        return cls(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"], stream)

    def _check(self, rc, allow=(0,)):
        if rc not in allow:
            raise CPRError(rc, self.lib.cpr_last_error(self.ctx).decode())
        return rc

    def vector(self):
        """A zero state / right-hand-side vector: shaped [b, nz, ny, nx], or
        flat [b n + rate wells] when rate-controlled wells add BHPs."""
        if self.nrate:
            return torch.zeros(self.b * int(np.prod(self.shape)) + self.nrate, dtype=torch.float64, device="cuda")
        return torch.zeros((self.b,) + self.shape, dtype=torch.float64, device="cuda")

    def unknowns(self):
        return int(self.lib.cpr_num_unknowns(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.cpr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the three calls of the hot path and the Newton update
    def assemble(self, x_old, x, dt_days, rhs=None):
        rhs = self.vector() if rhs is None else rhs
        self._check(self.lib.assemble_jacobian(self.ctx, _ptr(x_old), _ptr(x), float(dt_days), _ptr(rhs)))
        return rhs

    def setup(self, options=None, **kw):
        o = options if options is not None else default_options(**kw)
        self._check(self.lib.cpr_setup(self.ctx, ctypes.byref(o)))

    def solve(self, rhs, dx=None):
        dx = self.vector() if dx is None else dx
        st = Stats()
        rc = self._check(self.lib.cpr_gmres_solve(self.ctx, _ptr(rhs), _ptr(dx), ctypes.byref(st)),
                         allow=(0, 1))
        d = st.as_dict()
        d["status"] = rc
        return dx, d

    def bicgstab(self, rhs, dx=None):
        """BiCGSTAB with the same CPR preconditioner; returns (dx, stats)."""
        dx = self.vector() if dx is None else dx
        st = Stats()
        rc = self._check(self.lib.cpr_bicgstab_solve(self.ctx, _ptr(rhs), _ptr(dx), ctypes.byref(st)),
                         allow=(0, 1))
        d = st.as_dict()
        d["status"] = rc
        return dx, d

    def time_step(self, x_old, dt_days, options=None, newton=None, x=None):
        """One inexact Newton time step from x_old (Algorithm 1 with
        time-step cuts); returns (x, stats).  options: linear-solver
        options (cpr_options_t); newton: NewtonOptions or a dict of its
        fields."""
        x = self.vector() if x is None else x
        lo = options if options is not None else default_options()
        no = newton if isinstance(newton, NewtonOptions) else default_newton_options(**(newton or {}))
        st = NewtonStats()
        rc = self._check(self.lib.cpr_time_step(self.ctx, _ptr(x_old), _ptr(x), float(dt_days),
                                                ctypes.byref(lo), ctypes.byref(no), ctypes.byref(st)),
                         allow=(0, 1))
        d = st.as_dict()
        d["status"] = rc
        return x, d

    def simulate(self, x0, t_end, dt0, dt_max, growth=2.0, options=None, newton=None, x=None, log=None):
        """Time stepping over [0, t_end] days from x0 (cpr_simulate);
        returns (x, stats).  log: path of a JSON-lines record of the run
        (write_jsonl)."""
        x = self.vector() if x is None else x
        lo = options if options is not None else default_options()
        no = newton if isinstance(newton, NewtonOptions) else default_newton_options(**(newton or {}))
        st = SimStats()
        rc = self._check(self.lib.cpr_simulate(self.ctx, _ptr(x0), _ptr(x), float(t_end), float(dt0),
                                               float(dt_max), float(growth), ctypes.byref(lo), ctypes.byref(no),
                                               ctypes.byref(st)), allow=(0, 1))
        d = st.as_dict()
        d["status"] = rc
        if log:
            write_jsonl(log, d)
        return x, d

    def newton_update(self, x, dx):
        self._check(self.lib.cpr_newton_update(self.ctx, _ptr(x), _ptr(dx)))
        return x

    # -- single operations and setup products, for verification
    def spmv(self, x, y=None):
        y = self.vector() if y is None else y
        self._check(self.lib.cpr_spmv(self.ctx, _ptr(x), _ptr(y)))
        return y

    def spmv_noalloc(self, x, y):
        """y = A x like spmv(), staged through the library's static device
        buffer (cpr_spmv_noalloc: the call allocates nothing; y must be
        given)."""
        self._check(self.lib.cpr_spmv_noalloc(self.ctx, _ptr(x), _ptr(y)))
        return y

    def precond(self, v, z=None):
        z = self.vector() if z is None else z
        self._check(self.lib.cpr_precond_apply(self.ctx, _ptr(v), _ptr(z)))
        return z

    def export_jacobian(self):
        J = torch.empty((7, self.b, self.b) + self.shape, dtype=torch.float64, device="cuda")
        self._check(self.lib.cpr_export_jacobian(self.ctx, _ptr(J)))
        return J

    def import_jacobian(self, J):
        J = J if isinstance(J, torch.Tensor) else torch.as_tensor(np.ascontiguousarray(J)).cuda()
        self._check(self.lib.cpr_import_jacobian(self.ctx, _ptr(J.contiguous())))
        torch.cuda.synchronize()

    def export_qimpes(self):
        w = self.vector()
        self._check(self.lib.cpr_export_qimpes(self.ctx, _ptr(w)))
        return w

    def mg_level_shape(self, level):
        nx, ny, nz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rc = self.lib.cpr_mg_level_shape(self.ctx, level, ctypes.byref(nx), ctypes.byref(ny),
                                         ctypes.byref(nz))
        if rc != 0:
            return None
        return (nz.value, ny.value, nx.value)

    def nn_level(self):
        """Multigrid level of the learned stage under the last setup's options."""
        lv = ctypes.c_int()
        self._check(self.lib.cpr_nn_level(self.ctx, ctypes.byref(lv)))
        return lv.value

    def export_mg_level(self, level):
        shape = self.mg_level_shape(level)
        a = torch.empty((7,) + shape, dtype=torch.float64, device="cuda")
        self._check(self.lib.cpr_export_mg_level(self.ctx, level, _ptr(a)))
        return a

    def profile_kernel(self, kclass):
        """Sample every launch of one kernel class with HIP events (None: off)."""
        k = -1 if kclass is None else KCLASS[kclass]
        self._check(self.lib.cpr_profile_kernel(self.ctx, k))

    def set_timing(self, on=True):
        """Phase timers: solves then report ms_assemble, ms_setup, ms_solve,
        ms_precond, ms_spmv and ms_orth in their stats."""
        self._check(self.lib.cpr_set_timing(self.ctx, 1 if on else 0))

    def profile_read(self):
        """(launches, total milliseconds) sampled since the last read; syncs."""
        n, ms = ctypes.c_int(), ctypes.c_double()
        self._check(self.lib.cpr_profile_read(self.ctx, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def attach_network(self, theta):
        """Give the solver trained network parameters (None detaches)."""
        if theta is None:
            self._check(self.lib.cpr_nn_attach(self.ctx, None))
            return
        th = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(self.lib.cpr_nn_attach(self.ctx, th.ctypes.data_as(ctypes.c_void_p)))

    def pressure_stage(self, v, level=None):
        """(r', dp_mg) of the pressure stage applied to v [b, nz, ny, nx]; on
        the multigrid level of the learned stage under the last setup's
        options (nn_level(); `level`, if given, must equal it): the residual
        the cycle leaves there and that level's correction, in its natural
        order."""
        lv = self.nn_level()
        if level is not None and level != lv:
            raise ValueError(f"level {level} is not the learned stage's level {lv}")
        level = lv
        shape = self.shape if level == 0 else self.mg_level_shape(level)
        rp = torch.empty(shape, dtype=torch.float64, device="cuda")
        dp = torch.empty(shape, dtype=torch.float64, device="cuda")
        self._check(self.lib.cpr_pressure_stage(self.ctx, _ptr(v), _ptr(rp), _ptr(dp)))
        return rp, dp

    def features(self, rprime):
        """Network input [nz, ny, nx, 3] for a pressure residual (on the
        level options.nn_level of the last setup), and its scale."""
        f = torch.empty(tuple(rprime.shape) + (3,), dtype=torch.float32, device="cuda")
        sc = ctypes.c_double()
        self._check(self.lib.cpr_nn_features(self.ctx, _ptr(rprime), _fptr(f), ctypes.byref(sc)))
        return f, sc.value

    def export_krylov(self, j):
        v = self.vector()
        self._check(self.lib.cpr_export_krylov(self.ctx, j, _ptr(v)))
        return v

    def export_ilu(self):
        d = torch.empty((self.b, self.b) + self.shape, dtype=torch.float64, device="cuda")
        self._check(self.lib.cpr_export_ilu(self.ctx, _ptr(d)))
        return d


def make_target(e, scale):
    """FP32 training target e / scale computed on the GPU (e: float64 tensor)."""
    t = torch.empty(e.shape, dtype=torch.float32, device="cuda")
    rc = load().cpr_nn_make_target(_ptr(e.contiguous()), e.numel(), float(scale), _fptr(t),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise CPRError(rc, "cpr_nn_make_target")
    return t


def newton_step(solver, x_old, x, dt_days, options=None, krylov="fgmres", **kw):
    """One inexact Newton iteration (Algorithm 1): assemble A and b = -F(x),
    set up CPR, solve with FGMRES (or BiCGSTAB), update x in place.  Returns
    (dx, stats)."""
    rhs = solver.assemble(x_old, x, dt_days)
    solver.setup(options, **kw)
    dx, st = solver.bicgstab(rhs) if krylov == "bicgstab" else solver.solve(rhs)
    solver.newton_update(x, dx)
    return dx, st
