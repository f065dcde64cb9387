"""Newton step on the incremental potential with block-Jacobi PCG (oracle).

TEST INFRASTRUCTURE ONLY.  Follows:
* Eq. 2 / Eq. 3: x(t+dt) = argmin E_BE(x), v(t+dt) = (x(t+dt) - x(t))/dt, with
  x_tilde = x(t) + dt v(t) + dt^2 g.
* Sec. 7.2 (linear solve): 3x3 block-diagonal preconditioned CG with a forcing
  sequence; the forcing term is eta_k = min(0.5, sqrt(r_k / r_0)) (the paper
  only names the technique; this is the reading used here), zero initial guess.
* Sec. 5.2 (three evaluation levels): energy only in the line search, energy
  and gradient for convergence, full Hessian for the Newton system.
* Sec. 7 (benchmark protocol): a step that needs too many Newton iterations or
  whose line search does not descend is restarted with half the time step; the
  step grows back after a few successes (read here as 3).

Line search: backtracking from alpha = 1, halving while
E(x + alpha dx) > E(x) + 1e-4 alpha g.dx + 1e-12 |E(x)|, at most 30 times
(the paper names no line-search rule; this reading adds to Armijo's test the
rounding of the float64 energy sum, so that close to the minimiser, where the
energy no longer resolves the decrease, the full Newton step is taken).
Convergence: ||g_free||_2 <= rtol * ||g_free(x(t))||_2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import assembly
from .elements import x_tilde as predict


@dataclass
class StepParams:
    dt: float = 0.01
    gravity: tuple = (0.0, 0.0, -9.81)
    newton_rtol: float = 1e-6
    max_newton: int = 100
    max_pcg: int = 500
    project: bool | str = False        # True: nearest PSD; "filter": see assembly
    ls_max: int = 30
    armijo_c: float = 1e-4
    energy_round: float = 1e-12       # relative rounding allowance of E comparisons
    max_halvings: int = 8
    regrow_after: int = 3


def diag_inverse(row_ptr, col_idx, vals, contact_blocks=None):
    """Inverses of the 3x3 diagonal blocks (block-Jacobi preconditioner),
    contact diagonal blocks included."""
    N = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    d = np.nonzero(rows == col_idx)[0]
    D = vals[d].copy()
    for (i, j), b in (contact_blocks or {}).items():
        if i == j:
            D[i] += b
    return np.linalg.inv(D)


def pcg(A, Dinv, b, rtol, max_iter):
    """Preconditioned CG on A x = b from x = 0; stop at ||r|| <= rtol ||b||.

    A is a scipy sparse matrix (3N x 3N), Dinv the (N,3,3) block inverses.
    Returns (x, iterations, converged).
    """
    N = Dinv.shape[0]

    def prec(r):
        return np.einsum("nij,nj->ni", Dinv, r.reshape(N, 3)).ravel()

    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, True
    z = prec(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * bnorm:
            return x, it, True
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter, False


def newton_solve(scene, x_t, v_t, dt, prm: StepParams, solver="pcg", record=None):
    """One implicit-Euler step at fixed dt.  Returns (ok, x, report dict).
    Lagged rotations (fixed co-rotational, ARAP) are taken at x(t)."""
    xt = predict(x_t, v_t, dt, prm.gravity)
    x = x_t.copy()
    rp, ci = assembly.pattern_fast(scene)
    rep = dict(newton_iters=0, pcg_iters=0, ls_backtracks=0, residual0=0.0, residual=0.0,
               energy=0.0, status="ok")
    r0 = None
    for it in range(prm.max_newton + 1):
        asm = assembly.assemble(scene, x, xt, dt, project=prm.project, row_ptr=rp, col_idx=ci,
                                x_lag=x_t)
        g = asm["g"]
        r = float(np.linalg.norm(g))
        if r0 is None:
            r0 = r
            rep["residual0"] = r0
        rep["residual"] = r
        rep["energy"] = asm["E"]
        if r <= prm.newton_rtol * r0:
            return True, x, rep
        if it == prm.max_newton:
            break
        A = assembly.to_scipy(rp, ci, asm["vals"], asm["contact_blocks"])
        b = -g.ravel()
        if solver == "direct":
            dx = spla.spsolve(A.tocsc(), b)
            n_cg = 0
        else:
            eta = min(0.5, np.sqrt(r / r0))
            Dinv = diag_inverse(rp, ci, asm["vals"], asm["contact_blocks"])
            dx, n_cg, _ = pcg(A, Dinv, b, eta, prm.max_pcg)
        rep["pcg_iters"] += n_cg
        if record is not None:
            record.append(dict(x=x.copy(), g=g.copy(), dx=dx.reshape(-1, 3).copy(),
                               vals=asm["vals"].copy(), E=asm["E"]))
        dx = dx.reshape(-1, 3)
        gd = float(np.sum(g * dx))
        if not gd < 0.0:
            rep["status"] = "line_search"
            return False, x, rep
        E0 = asm["E"]
        alpha = 1.0
        ok = False
        for _ in range(prm.ls_max + 1):
            Et = assembly.energy(scene, x + alpha * dx, xt, dt, x_lag=x_t)
            if Et <= E0 + prm.armijo_c * alpha * gd + prm.energy_round * abs(E0):
                ok = True
                break
            alpha *= 0.5
            rep["ls_backtracks"] += 1
        if not ok:
            rep["status"] = "line_search"
            return False, x, rep
        x = x + alpha * dx
        rep["newton_iters"] += 1
    rep["status"] = "not_converged"
    return False, x, rep


class Stepper:
    """Time stepping with dt halving on failure and regrowth after successes.

    With max_halvings == 0 there is no step control: every step is taken at
    exactly prm.dt and the reduced step and success count are left alone, so a
    given dt sequence can be replayed."""

    def __init__(self, scene, prm: StepParams, solver="pcg"):
        self.scene = scene
        self.prm = prm
        self.solver = solver
        self.dt_cur = prm.dt
        self.successes = 0

    def step(self, x_t, v_t):
        control = self.prm.max_halvings > 0
        dt = self.dt_cur if control else self.prm.dt
        halvings = 0
        while True:
            ok, x, rep = newton_solve(self.scene, x_t, v_t, dt, self.prm, self.solver)
            if ok:
                break
            if halvings == self.prm.max_halvings:
                rep["dt_halvings"] = halvings
                rep["dt_used"] = dt
                return x_t, v_t, rep
            dt *= 0.5
            halvings += 1
        v = (x - x_t) / dt
        if not control:
            pass
        elif halvings:
            self.dt_cur = dt
            self.successes = 0
        else:
            self.successes += 1
            if self.successes >= self.prm.regrow_after and self.dt_cur < self.prm.dt:
                self.dt_cur = min(2.0 * self.dt_cur, self.prm.dt)
                self.successes = 0
        rep["dt_halvings"] = halvings
        rep["dt_used"] = dt
        return x, v, rep
