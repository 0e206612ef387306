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


class GradientEvaluator:
    """One GPU gradient evaluation per call, u given on the host.

    All buffers (controls, states, workspace, F, beta, gradient) are allocated
    once.  With `graph`, the first call runs eagerly, the second records the
    whole evaluation (every Krylov call, bracket and reduction: thousands of
    launches) into one HIP graph on a side stream, and later calls copy u into
    the static control buffer and replay the graph.  The kernels read u from
    device memory, so the graph stays valid for any controls; nothing in the
    evaluation records a memset.  `basis` (a ReducedBasis) runs the
    evaluation in the fixed-excitation, even-parity basis."""

    VARIANTS = ("zeroth", "centred", "first_order", "quadrature")

    def __init__(self, h, N: int, dt: float, k, psi0, target, ckpt_every: int = 0,
                 gradient: str = "centred", nodes: int = 4, basis=None, graph: bool = False):
        import torch

        from .api import Workspace, new_states
        if gradient not in self.VARIANTS:
            raise ValueError(f"gradient must be one of {self.VARIANTS}")
        self.torch = torch
        dev = psi0.device
        self.N = int(N)
        extended = gradient in ("first_order", "quadrature")
        # the closure below holds these buffers, not the evaluator, so that a
        # dropped evaluator is freed at once rather than by the cycle collector
        u = self.u = torch.zeros(self.N, dtype=torch.float64, device=dev)
        F = self.F = torch.empty((), dtype=torch.float64, device=dev)
        beta = self.beta = torch.empty(2, dtype=torch.float64, device=dev)
        grad = self.grad = torch.empty(self.N, dtype=torch.float64, device=dev)
        if basis is None:
            from . import api
            ws = Workspace(h, k, psi0.dtype, dev, extended=extended)
            states = new_states(h, self.N, ckpt_every, psi0.dtype, dev)
            opts = {"zeroth": {}, "centred": {"centred": True},
                    "first_order": {"first_order": True}, "quadrature": {"nodes": nodes}}[gradient]

            def run():
                api.grape_gradient(h, u, dt, k, psi0, target, ckpt_every=ckpt_every,
                                   states=states, workspace=ws, F=F, beta=beta, grad=grad,
                                   **opts)
        else:
            from . import reduced
            ws = reduced.ReducedWorkspace(basis, k, psi0.dtype, dev, extended=extended)
            states = reduced.pe_states(basis, self.N, ckpt_every, psi0.dtype, dev)

            def run():
                reduced.grape_gradient_pe(h, basis, u, dt, k, psi0, target,
                                          ckpt_every=ckpt_every, variant=gradient,
                                          nodes=nodes if gradient == "quadrature" else 0,
                                          states=states, workspace=ws, F=F, beta=beta,
                                          grad=grad)
        self._keep = (ws, states)
        self._run = run
        self.graph = graph
        self._g = None
        self.calls = 0

    def _capture(self):
        from ._graph import capture_guard
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with capture_guard(), torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self._run()
        torch.cuda.current_stream().wait_stream(s)
        self._g = g

    def __call__(self, u):
        torch = self.torch
        self.u.copy_(torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64)))
        if self.graph and self.calls >= 1:
            if self._g is None:
                self._capture()
            self._g.replay()
        else:
            self._run()
        self.calls += 1
        torch.cuda.synchronize()
        return float(self.F.cpu()), self.grad.cpu().numpy().copy()


def optimize_controls(h, u0, dt: float, k, psi0, target, ckpt_every: int = 0,
                      gradient: str = "centred", I_target: float = 1e-2, max_iter: int = 200,
                      history: int = 10, nodes: int = 4, callback=None, basis=None,
                      graph: bool = False) -> LbfgsResult:
    """Minimise the infidelity I(u) = 1 - F(u) over the controls with L-BFGS,
    every evaluation one GPU gradient (`gradient`: "zeroth", "centred",
    "first_order" or "quadrature" with `nodes` Gauss-Legendre nodes).  Stops at
    I <= I_target or when I changes by less than ten machine epsilons.
    `basis` runs in a ReducedBasis (vectors of its dimension); `graph` replays
    each evaluation from a captured HIP graph."""
    ev = GradientEvaluator(h, int(np.asarray(u0).size), dt, k, psi0, target, ckpt_every,
                           gradient, nodes, basis, graph)

    def fg(u):
        F, g = ev(u)
        return 1.0 - F, -g

    res = lbfgs(fg, np.asarray(u0, dtype=np.float64), history=history, max_iter=max_iter,
                f_target=I_target, callback=callback)
    return res


__all__ = ["lbfgs", "optimize_controls", "LbfgsResult", "GradientEvaluator"]
