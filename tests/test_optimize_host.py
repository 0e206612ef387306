"""The host L-BFGS driver on objectives with known minima (no GPU)."""

import os

import numpy as np
import pytest
import scipy.optimize as so

from paper_2010_03598_amd import _lib, optimize


def rosen(x):
    return float(so.rosen(x)), so.rosen_der(x)


@pytest.mark.parametrize("n", [2, 10])
def test_rosenbrock_minimum(n):
    x0 = np.full(n, -1.2)
    x0[1::2] = 1.0
    r = optimize.lbfgs(rosen, x0, max_iter=500, df_min=0.0, g_tol=1e-9)
    assert r.reason in ("g_tol", "line_search")
    assert np.abs(r.x - 1.0).max() < 1e-6
    ref = so.minimize(rosen, x0, jac=True, method="L-BFGS-B", options={"gtol": 1e-10})
    assert np.abs(r.x - ref.x).max() < 1e-5
    assert all(b <= a + 1e-15 for a, b in zip(r.history, r.history[1:]))


def test_quadratic_solves_linear_system():
    rng = np.random.default_rng(0)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    b = rng.standard_normal(n)
    fg = lambda x: (0.5 * float(x @ A @ x) - float(b @ x), A @ x - b)
    r = optimize.lbfgs(fg, np.zeros(n), max_iter=200, df_min=0.0, g_tol=1e-12)
    assert np.abs(r.x - np.linalg.solve(A, b)).max() < 1e-9


def test_line_search_meets_strong_wolfe():
    fg = lambda x: (float(np.sum(np.cosh(x - 0.3)) + x @ x), np.sinh(x - 0.3) + 2.0 * x)
    x = np.array([2.0, -1.5, 0.7])
    f0, g0 = fg(x)
    p = -g0
    for c1, c2 in [(1e-4, 0.9), (1e-4, 0.1)]:
        a, f, g, _ = optimize._wolfe_search(fg, x, f0, g0, p, c1, c2, 40)
        assert a > 0
        assert f <= f0 + c1 * a * float(g0 @ p)
        assert abs(float(g @ p)) <= c2 * abs(float(g0 @ p))


def test_stops_at_target_and_on_stagnation():
    fg = lambda x: (float(x @ x), 2.0 * x)
    r = optimize.lbfgs(fg, np.ones(5), f_target=1e-3)
    assert r.reason == "f_target" and r.f <= 1e-3
    r = optimize.lbfgs(lambda x: (1.0, np.zeros_like(x)), np.ones(3), g_tol=-1.0)
    assert r.reason in ("line_search", "df_min")


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libkgrape.so not built")
def test_evaluator_is_freed_without_the_cycle_collector():
    """A dropped GradientEvaluator releases its buffers (and any captured graph) by
    reference counting alone: a collection by the cycle collector could otherwise
    free device memory in the middle of a later graph capture.  (The buffers are
    host tensors here; nothing runs.)"""
    import gc
    import weakref

    import torch

    import paper_2010_03598_amd as kg
    psi0 = torch.zeros(64, dtype=torch.complex128)
    ev = optimize.GradientEvaluator(kg.XXZ(6), 5, 0.1, kg.Krylov(8), psi0, psi0, ckpt_every=2,
                                    gradient="centred", graph=True)
    ref = weakref.ref(ev)
    was = gc.isenabled()
    gc.disable()
    try:
        del ev
        assert ref() is None
    finally:
        if was:
            gc.enable()
