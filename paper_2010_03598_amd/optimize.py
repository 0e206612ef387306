"""Host L-BFGS driver around the GPU gradient (the update step of Algorithm 1).

The paper feeds its gradient to an L-BFGS routine (Nocedal's limited-memory
BFGS) whose step length satisfies the Wolfe conditions, and stops at a target
infidelity or when the infidelity changes by less than ten machine epsilons
between iterations (Sec. III.B).  `lbfgs` is that driver for any smooth
objective given as (value, gradient); `optimize_controls` minimises the
infidelity I = 1 - F of a chain with the gradients of this library (the
centred variant by default, the paper's choice).

The quasi-Newton direction uses the two-loop recursion (Nocedal & Wright,
Numerical Optimization, 2nd ed., Algorithm 7.4) with the scaling
gamma = s'y / y'y of the latest pair; the step length comes from a bracketing
line search with bisection zoom for the strong Wolfe conditions (ibid.,
Algorithms 3.5 and 3.6).  The vectors are short (one entry per slice), so
this runs on the host in FP64.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Tuple

import numpy as np

FunGrad = Callable[[np.ndarray], Tuple[float, np.ndarray]]


@dataclasses.dataclass
class LbfgsResult:
    x: np.ndarray
    f: float
    g: np.ndarray
    iterations: int
    evaluations: int
    reason: str
    history: List[float]          # objective after every iteration (history[0] = start)


def _wolfe_search(fg: FunGrad, x: np.ndarray, f0: float, g0: np.ndarray, p: np.ndarray,
                  c1: float, c2: float, max_eval: int, a_max: float = 1e6):
    """Step a along p with f(x+ap) <= f0 + c1 a g0'p and |g(x+ap)'p| <= c2 |g0'p|.
    Returns (a, f, g, evaluations); a = 0 when no acceptable step was found."""
    d0 = float(g0 @ p)
    evals = 0
    a_prev, f_prev = 0.0, f0
    a = 1.0
    lo = hi = None
    f_lo = g_lo = None
    while evals < max_eval:
        f, g = fg(x + a * p)
        evals += 1
        d = float(g @ p)
        if f > f0 + c1 * a * d0 or (evals > 1 and f >= f_prev):
            lo, hi, f_lo = a_prev, a, f_prev
            break
        if abs(d) <= -c2 * d0:
            return a, f, g, evals
        if d >= 0:
            lo, hi, f_lo = a, a_prev, f
            break
        a_prev, f_prev = a, f
        a = min(2.0 * a, a_max)
    else:
        return 0.0, f0, g0, evals
    # zoom between lo (sufficient decrease holds) and hi, by bisection
    while evals < max_eval:
        a = 0.5 * (lo + hi)
        f, g = fg(x + a * p)
        evals += 1
        d = float(g @ p)
        if f > f0 + c1 * a * d0 or f >= f_lo:
            hi = a
        else:
            if abs(d) <= -c2 * d0:
                return a, f, g, evals
            if d * (hi - lo) >= 0:
                hi = lo
            lo, f_lo = a, f
        if abs(hi - lo) < 1e-12 * max(1.0, abs(lo)):
            break
    if lo and lo > 0.0:
        f, g = fg(x + lo * p)
        evals += 1
        if f <= f0 + c1 * lo * d0:
            return lo, f, g, evals
    return 0.0, f0, g0, evals


def lbfgs(fg: FunGrad, x0, history: int = 10, max_iter: int = 200, f_target: float = -np.inf,
          df_min: float = 10.0 * np.finfo(float).eps, g_tol: float = 0.0, c1: float = 1e-4,
          c2: float = 0.9, max_ls: int = 30,
          callback: Optional[Callable[[int, np.ndarray, float], None]] = None) -> LbfgsResult:
    """Minimise f with gradient g = grad f.  Stops when f <= f_target, when f
    changes by less than df_min in an iteration, when max|g| <= g_tol, when no
    step satisfies the Wolfe conditions, or after max_iter iterations."""
    x = np.array(x0, dtype=np.float64)
    f, g = fg(x)
    evals = 1
    S: List[np.ndarray] = []
    Y: List[np.ndarray] = []
    hist = [f]
    reason = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        if f <= f_target:
            reason, it = "f_target", it - 1
            break
        if np.max(np.abs(g)) <= g_tol:
            reason, it = "g_tol", it - 1
            break
        # two-loop recursion
        q = g.copy()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            rho = 1.0 / float(y @ s)
            a = rho * float(s @ q)
            q -= a * y
            alphas.append((rho, a, s, y))
        gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1]) if S else 1.0 / max(1.0, np.linalg.norm(g))
        r = gamma * q
        for rho, a, s, y in reversed(alphas):
            b = rho * float(y @ r)
            r += (a - b) * s
        p = -r
        if float(g @ p) >= 0.0:          # not a descent direction: restart
            S.clear()
            Y.clear()
            p = -g / max(1.0, np.linalg.norm(g))
        step, f_new, g_new, ne = _wolfe_search(fg, x, f, g, p, c1, c2, max_ls)
        evals += ne
        if step == 0.0:
            reason, it = "line_search", it - 1
            break
        s = step * p
        y = g_new - g
        x = x + s
        df = f - f_new
        f, g = f_new, g_new
        hist.append(f)
        if float(s @ y) > 1e-12 * float(y @ y):
            S.append(s)
            Y.append(y)
            if len(S) > history:
                S.pop(0)
                Y.pop(0)
        if callback is not None:
            callback(it, x, f)
        if abs(df) < df_min:
            reason = "df_min"
            break
    return LbfgsResult(x=x, f=f, g=g, iterations=it, evaluations=evals, reason=reason,
                       history=hist)


def optimize_controls(h, u0, dt: float, k, psi0, target, ckpt_every: int = 0,
                      gradient: str = "centred", I_target: float = 1e-2, max_iter: int = 200,
                      history: int = 10, nodes: int = 4, callback=None) -> LbfgsResult:
    """Minimise the infidelity I(u) = 1 - F(u) over the controls with L-BFGS,
    every evaluation one GPU gradient (`gradient`: "zeroth", "centred",
    "first_order" or "quadrature" with `nodes` Gauss-Legendre nodes).  Stops at
    I <= I_target or when I changes by less than ten machine epsilons."""
    import torch

    from .api import Workspace, grape_gradient, new_states

    dev = psi0.device
    N = int(np.asarray(u0).size)
    ws = Workspace(h, k, psi0.dtype, dev, extended=gradient in ("first_order", "quadrature"))
    states = new_states(h, N, ckpt_every, psi0.dtype, dev)
    u_dev = torch.empty(N, dtype=torch.float64, device=dev)
    opts = {"zeroth": {}, "centred": {"centred": True}, "first_order": {"first_order": True},
            "quadrature": {"nodes": nodes}}[gradient]

    def fg(u):
        u_dev.copy_(torch.from_numpy(np.ascontiguousarray(u)))
        r = grape_gradient(h, u_dev, dt, k, psi0, target, ckpt_every=ckpt_every, states=states,
                           workspace=ws, **opts)
        return 1.0 - float(r.F.cpu()), -r.grad.cpu().numpy()

    return lbfgs(fg, np.asarray(u0, dtype=np.float64), history=history, max_iter=max_iter,
                 f_target=I_target, callback=callback)


__all__ = ["lbfgs", "optimize_controls", "LbfgsResult"]
