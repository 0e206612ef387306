"""Write the oracle's expected values for the GPU parity tests that are too
large to run the oracle inside a test (L=16 ascent, L=20 and L=24 chains).

Calls only the oracle and the seeded input generators:

    python tests/golden/make_golden.py [adjoint_short adjoint_short_plain adjoint_full
                                        large_short large_ckpt
                                        ascent batched batched_planned]

Each JSON file records the workload, the oracle settings and the values.
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import dimension, exact, grape, krylov, model  # noqa: E402


def sample_rows(D, seed=123):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(32), D - 1 - np.arange(32),
                                     rng.integers(0, D, 128)])).astype(np.int64)


def cplx(z):
    return [float(np.real(z)), float(np.imag(z))]


def chain_record(c):
    return {"L": c.L, "J": c.J, "Delta": c.Delta, "hc_kind": c.hc_kind, "hc_sites": c.hc_sites,
            "N": c.N, "dt": c.dt, "m": c.m}


def gradient_case(name, c, exact_slices=(), reorth=True):
    t0 = time.time()
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    r = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, reorth, krylov.default_tol())
    rows = sample_rows(1 << c.L)
    out = {"workload": name, "chain": chain_record(c), "reorth": reorth,
           "oracle": "grape.gradient (Lanczos, " +
                     ("full re-orthonormalisation" if reorth else "plain three-term window") +
                     ", FP64)",
           "F": r.F, "beta": cplx(r.beta), "grad": r.grad.tolist(),
           "m_eff_fwd": r.m_eff_fwd.tolist(), "psi_N_rows": rows.tolist(),
           "psi_N_re": np.real(r.psi_N[rows]).tolist(), "psi_N_im": np.imag(r.psi_N[rows]).tolist()}
    if exact_slices:
        _, gq = exact.exact_gradient_quadrature(ch, c.u, c.psi0, c.target, c.dt, c.m,
                                                slices=list(exact_slices), nodes=8)
        out["exact_grad_slices"] = [int(j) for j in exact_slices]
        out["exact_grad"] = [float(gq[j]) for j in exact_slices]
        out["exact_method"] = "Gauss-Legendre (8 nodes) quadrature of the natural gradient per slice"
    out["oracle_seconds"] = time.time() - t0
    return out


def adjoint_short():
    c = workloads.adjoint(N=8)
    return gradient_case("adjoint L=20 with N=8 (seed 2)", c, exact_slices=range(8))


def adjoint_short_plain():
    c = workloads.adjoint(N=8)
    return gradient_case("adjoint L=20 with N=8 (seed 2), plain Lanczos", c, reorth=False)


def adjoint_full():
    c = workloads.adjoint()
    return gradient_case("adjoint L=20 with all N=400 slices (seed 2)", c)


def large_ckpt():
    c = workloads.large(N=LARGE_CKPT_N)
    return gradient_case(f"large L=24 with N={LARGE_CKPT_N} (seed 4)", c)


LARGE_CKPT_N = 6


def large_short():
    c = workloads.large(N=2)
    return gradient_case("large L=24 with N=2 (seed 4)", c)


def ascent():
    c = workloads.ascent()
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    u = c.u.copy()
    Fs, gs = [], []
    t0 = time.time()
    for it in range(workloads.ASCENT_STEPS):
        r = grape.gradient(ch, u, c.psi0, c.target, c.dt, c.m, True, krylov.default_tol())
        Fs.append(r.F)
        gs.append(r.grad.tolist())
        u = grape.ascent_update(u, r.grad, workloads.ASCENT_ETA)
        print(f"ascent iteration {it}: F={r.F:.12e}", flush=True)
    return {"workload": "ascent L=16 (seed 1)", "chain": chain_record(c), "reorth": True,
            "eta": workloads.ASCENT_ETA, "steps": workloads.ASCENT_STEPS,
            "update": "u <- u + eta g / max|g|", "F": Fs, "grad": gs,
            "u_final": u.tolist(), "oracle_seconds": time.time() - t0}


BATCH_M = 12


def batched():
    """The 64-chain batched workload (seed 3) with a fixed Krylov dimension, using the
    complex64 breakdown policy (the batched form keeps complex64 vectors)."""
    import dataclasses
    recs = []
    t0 = time.time()
    for i, c in enumerate(workloads.batched()):
        c = dataclasses.replace(c, m=BATCH_M)
        ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
        r = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, True,
                           krylov.default_tol(krylov.EPS_C64))
        recs.append({"chain": chain_record(c), "F": r.F, "beta": cplx(r.beta),
                     "grad": r.grad.tolist()})
        print(f"batched chain {i}: L={c.L} N={c.N} F={r.F:.6e}", flush=True)
    return {"workload": "batched: 64 chains (seed 3)", "m": BATCH_M, "reorth": True,
            "oracle": "grape.gradient per chain, complex64 breakdown tolerance",
            "chains": recs, "oracle_seconds": time.time() - t0}


def batched_planned():
    """The 64-chain batched workload (seed 3) with the Krylov dimension of each chain
    chosen from the a-priori bound (oracle.dimension: accuracy 1e-8 per sweep, m in
    8..24), the dimensions the batched form's planner must also choose."""
    import dataclasses
    recs = []
    t0 = time.time()
    for i, c in enumerate(workloads.batched()):
        m = dimension.krylov_dimension(c.L, c.J, c.Delta, bin(c.hc_sites).count("1"),
                                       float(np.max(np.abs(c.u))), c.dt, c.N)
        c = dataclasses.replace(c, m=m)
        ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
        r = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, True,
                           krylov.default_tol(krylov.EPS_C64))
        recs.append({"chain": chain_record(c), "F": r.F, "beta": cplx(r.beta),
                     "grad": r.grad.tolist()})
        print(f"batched chain {i}: L={c.L} N={c.N} m={m} F={r.F:.6e}", flush=True)
    return {"workload": "batched: 64 chains (seed 3), Krylov dimension per chain from "
                        "oracle.dimension.krylov_dimension (tol 1e-8, m in 8..24)",
            "reorth": True, "oracle": "grape.gradient per chain, complex64 breakdown tolerance",
            "chains": recs, "oracle_seconds": time.time() - t0}


CASES = {"adjoint_short": adjoint_short, "adjoint_short_plain": adjoint_short_plain,
         "adjoint_full": adjoint_full,
         "large_short": large_short, "large_ckpt": large_ckpt, "ascent": ascent,
         "batched": batched, "batched_planned": batched_planned}


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        t = time.time()
        rec = CASES[n]()
        with open(os.path.join(HERE, f"{n}.json"), "w") as fh:
            json.dump(rec, fh)
        print(f"{n}: written in {time.time() - t:.0f} s", flush=True)
