"""Pins of the oracle's FGMRES with delayed reorthogonalisation (DCGS2):
in exact arithmetic it builds the basis of classical Gram-Schmidt twice, so
on well-conditioned systems its iterates must equal the CGS2 iterates to
rounding (same iteration counts, fixed paths across a restart), the vectors
it hands the preconditioner must be orthonormal to rounding, and it must
solve dense systems like LAPACK.  One step is also checked against its defining
identities on an input far from orthogonal to the basis, where the
reorthogonalisation is not a rounding-level correction.  Mistakes planted in
a copy of the oracle (a sign flipped or a term dropped in the projections,
the Pythagorean norm replaced by the unprojected one, the reorthogonalisation
left out) fail these pins."""
import os
import types

import numpy as np
import pytest

from oracle import cpr, krylov, model
from paper_1606_00548_amd import synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "krylov.py")


def _dense(n=60, seed=3):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    d = np.diag(A).copy()
    return A, b, (lambda v: A @ v), (lambda v: v / d)


def _cpr_system():
    case = synth.black_oil_layered(8, 6, 4, seed=41)
    x = synth.random_state_perturbation(case, 42)
    R, J = model.assemble(case["grid"], case["fluid"], case["perm"], case["poro"], case["wells"],
                          case["x_old"], x, case["dt"])
    pc = cpr.cpr_setup(J)
    return -R, (lambda v: cpr.block_spmv(J, v)), (lambda v: cpr.cpr_apply(pc, v))


def pin_equals_cgs2(kr):
    A, b, mv, M = _dense()
    for kw in (dict(), dict(restart=10, rtol=1e-10), dict(rtol=0.0, max_iter=25, restart=12)):
        x1, s1 = kr.fgmres(mv, M, b, orth="dcgs2", **kw)
        x2, s2 = kr.fgmres(mv, M, b, orth="cgs2", **kw)
        if s1["iterations"] != s2["iterations"]:
            return f"dense {kw}: {s1['iterations']} != {s2['iterations']} iterations"
        if np.linalg.norm(x1 - x2) > 1e-10 * np.linalg.norm(x2):
            return f"dense {kw}: iterates differ by {np.linalg.norm(x1 - x2) / np.linalg.norm(x2):.1e}"
    b, mv, M = _cpr_system()
    for kw in (dict(), dict(rtol=0.0, max_iter=45)):
        x1, s1 = kr.fgmres(mv, M, b, orth="dcgs2", **kw)
        x2, s2 = kr.fgmres(mv, M, b, orth="cgs2", **kw)
        if s1["iterations"] != s2["iterations"] or np.linalg.norm(x1 - x2) > 1e-10 * np.linalg.norm(x2):
            return f"cpr {kw}: {s1['iterations']} / {s2['iterations']} iterations"
    return None


def pin_preconditioner_inputs_orthonormal(kr):
    A, b, mv, M = _dense(n=80, seed=5)
    Q = []
    kr.fgmres(mv, M, b, restart=40, rtol=1e-12, max_iter=40, record=lambda j, q, z: Q.append(q.copy()))
    Q = np.array(Q).T
    err = np.abs(Q.T @ Q - np.eye(Q.shape[1])).max()
    return None if err <= 1e-12 else f"preconditioner inputs lose orthogonality: {err:.1e}"


def pin_dense_solve(kr):
    A, b, mv, M = _dense(n=30, seed=7)
    x, st = kr.fgmres(mv, M, b, restart=30, rtol=1e-13)
    ref = np.linalg.solve(A, b)
    if not (st["converged"] and st["iterations"] <= 30):
        return f"dense 30x30: {st['iterations']} iterations"
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    return None if err <= 1e-10 else f"dense 30x30 error {err:.1e}"


def pin_step_identities(kr):
    """One step with a far from orthogonal input (|a| ~ 0.5): v orthonormal
    to V, uh = V a + beta v (the previous column's correction), w = V c +
    g v + u with u orthogonal to V and v -- definitions that hold in exact
    arithmetic whatever the input."""
    rng = np.random.default_rng(11)
    n, j = 200, 7
    V, _ = np.linalg.qr(rng.standard_normal((n, j)))
    V = [V[:, i].copy() for i in range(j)]
    uh = rng.standard_normal(n)
    uh = uh / np.linalg.norm(uh) + 0.3 * V[2] - 0.4 * V[5]
    uh = uh / np.linalg.norm(uh)
    w = rng.standard_normal(n) + 2.0 * V[0]
    v, a, beta, c, g, u = kr.dcgs2_step(V, uh, w)
    Vm = np.array(V).T
    checks = {
        "|v| = 1": abs(np.linalg.norm(v) - 1.0),
        "V^T v = 0": np.abs(Vm.T @ v).max(),
        "uh = V a + beta v": np.linalg.norm(uh - Vm @ a - beta * v),
        "w = V c + g v + u": np.linalg.norm(w - Vm @ c - g * v - u) / np.linalg.norm(w),
        "V^T u = 0, v^T u = 0": max(np.abs(Vm.T @ u).max(), abs(v @ u)) / np.linalg.norm(w),
    }
    bad = {k: f"{e:.1e}" for k, e in checks.items() if not e <= 1e-13}
    return None if not bad else f"step identities fail: {bad}"


PINS = (pin_equals_cgs2, pin_preconditioner_inputs_orthonormal, pin_dense_solve, pin_step_identities)


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_dcgs2_pins(pin):
    msg = pin(krylov)
    assert msg is None, msg


MUTANTS = {
    "sign of the new vector's projection": [
        ("    g = (d - float(np.dot(a, c))) / bj", "    g = (d + float(np.dot(a, c))) / bj")],
    "norm without the projection": [("    b2 = e - float(np.dot(a, a))", "    b2 = e")],
    "new vector not reorthogonalised": [("        v = v - a[i] * V[i]", "        pass")],
    "projection onto the new vector dropped": [("    u = u - g * v\n", "")],
    "projection coefficients from the unreorthogonalised vector": [
        ("    g = (d - float(np.dot(a, c))) / bj", "    g = d")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_dcgs2_mistake_fails_a_pin(name):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"planted edit no longer matches the oracle: {old!r}"
        src = src.replace(old, new)
    mod = types.ModuleType("krylov_mutant")
    exec(compile(src, "krylov_mutant", "exec"), mod.__dict__)
    failures = [m for m in (pin(mod) for pin in PINS) if m is not None]
    assert failures, f"planted mistake '{name}' passed every DCGS2 pin"
