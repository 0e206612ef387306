"""Benchmark of the K-GRAPE hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the adjoint form's chain): open XXZ chain L=20 (D = 1,048,576),
J=1, Delta=1, control S^x on site 1, N=400 slices, dt=0.05, Krylov m=20 with
full re-orthogonalisation, random-phase psi0 and target, controls U(-1,1)
(seed 2), sqrt(N) checkpointing every 20 slices.  One step = one GRAPE
gradient evaluation: forward sweep, overlap, segment recomputation, backward
sweep and the N gradient brackets, all on the GPU.  The headline value is
gradient evaluations per second of the mixed-precision path (complex64
vectors, FP64 scalars); the FP64 path (complex128) is timed beside it on the
same inputs and the error of mixed vs FP64 is reported.

Prints ONE JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GRAPE gradient evals/sec and H·v GB/s at L=20; mixed vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_inputs(c, dtype, torch):
    dev = torch.device("cuda:0")
    u = torch.tensor(c.u, dtype=torch.float64, device=dev)
    psi0 = torch.tensor(c.psi0, dtype=dtype, device=dev)
    f = torch.tensor(c.target, dtype=dtype, device=dev)
    return u, psi0, f


def time_gradients(kg, torch, c, dtype, ckpt, steps, warmup, profile_every=0):
    """One step = one gradient evaluation of the autograd form: F = fidelity(u)
    (grape_forward, keeping sqrt(N) checkpoints) and F.backward() (the adjoint
    sweep recomputing the segments and forming dF/du)."""
    h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    k = kg.Krylov(c.m, reorth=True)
    u, psi0, f = gpu_inputs(c, dtype, torch)
    ws = kg.Workspace(h, k, dtype)
    out = {}
    # the forward's state buffer comes from torch's caching allocator: one of
    # the same size is allocated and released here, outside any timed region
    spare = kg.new_states(h, c.N, ckpt, dtype)
    del spare

    def step():
        uu = u.detach().requires_grad_(True)
        F = kg.fidelity(uu, h, c.dt, k, psi0, f, ckpt, ws)
        F.backward()
        out["F"], out["grad"] = F.detach(), uu.grad

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{warmup} done")
    prof = None
    if profile_every:
        # events are created here, outside the timed region; inside it only the
        # sampled launches record events (about 2 * 40 * 1200 / profile_every
        # launches per gradient evaluation)
        prof = kg.profile(sample_every=profile_every,
                          max_launches=max(1024, steps * 120000 // profile_every))
        prof.__enter__()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if prof is not None:
        prof.__exit__(None, None, None)
    log(f"timed {steps} steps ({dtype}) in {t1 - t0:.3f} s")
    return ((t1 - t0) / steps, float(out["F"].cpu()), out["grad"].cpu().numpy(),
            (prof.result if prof else None))


def time_hv(kg, torch, L, dtype, reps=50):
    """Device time per H v launch: `reps` launches captured in one HIP graph and
    replayed between two events, so host-side call overhead does not enter."""
    from paper_2010_03598_amd._graph import capture_guard
    h = kg.XXZ(L, 1.0, 0.5)
    D = 1 << L
    g = torch.Generator(device="cuda")
    g.manual_seed(L)
    v = torch.randn(D, dtype=dtype, device="cuda", generator=g)
    w = torch.empty_like(v)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            kg.xxz_apply(h, 0.3, v, out=w)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with capture_guard(), torch.cuda.graph(graph):
        for _ in range(reps):
            kg.xxz_apply(h, 0.3, v, out=w)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        e0.record()
        graph.replay()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3 / reps)
    nbytes = 2 * D * v.element_size()          # v read once, w written once
    return {"L": L, "dtype": str(dtype).replace("torch.", ""), "us_per_launch": best * 1e6,
            "algorithmic_GBps": nbytes / best / 1e9, "frac_of_peak": nbytes / best / 1e9 / HBM_PEAK_GBS,
            "launches": reps, "timing": "HIP graph of the launches, best of 3 replays"}


def time_copy(torch, mib=1024, reps=10):
    """Measured HBM bandwidth of a plain device copy (torch's copy kernel) of
    `mib` MiB, larger than the Infinity Cache: bytes read plus bytes written per
    second over `reps` back-to-back copies between two events (each copy takes
    well over 100 us, so launch overhead does not enter); the reference the H v
    fractions are also stated against."""
    n = mib << 20
    src = torch.empty(n // 16, dtype=torch.complex128, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3 / reps)
    del src, dst
    return {"bytes_per_copy": 2 * n, "GBps": 2 * n / best / 1e9,
            "frac_of_peak": 2 * n / best / 1e9 / HBM_PEAK_GBS,
            "timing": f"{mib} MiB read and written, {reps} copies between two events, best of 3"}


def time_large(kg, torch, workloads, with_fp64=True, plain=True):
    """The large form: L=24 (D = 16,777,216), N=500 slices of dt=0.05, m=24
    with full re-orthogonalisation, checkpoints every 22 slices.  One gradient
    evaluation in complex64 + FP64 scalars (kernels sampled with HIP events)
    and one in complex128, each after a two-slice warm-up through the same
    workspace, and the error of the first against the second; with `plain`,
    one more complex64 evaluation with plain Lanczos (three-term window, no
    re-orthogonalisation) and its error against both."""
    c = workloads.large()
    ckpt = workloads.LARGE_CKPT_EVERY
    h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    res = {}
    legs = [(torch.complex64, True)] + ([(torch.complex128, True)] if with_fp64 else [])
    legs += [(torch.complex64, False)] if plain else []
    for dtype, reorth in legs:
        k = kg.Krylov(c.m, reorth=reorth)
        u, psi0, f = gpu_inputs(c, dtype, torch)
        ws = kg.Workspace(h, k, dtype)
        kg.grape_gradient(h, u[:2].contiguous(), c.dt, k, psi0, f, workspace=ws)
        states = kg.new_states(h, c.N, ckpt, dtype)
        torch.cuda.synchronize()
        prof = kg.profile(sample_every=16, max_launches=20000) \
            if (dtype == torch.complex64 and reorth) else None
        if prof:
            prof.__enter__()
        t0 = time.perf_counter()
        r = kg.grape_gradient(h, u, c.dt, k, psi0, f, ckpt_every=ckpt, states=states, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if prof:
            prof.__exit__(None, None, None)
        res[(dtype, reorth)] = (t1 - t0, float(r.F.cpu()), r.grad.cpu().numpy(),
                                prof.result if prof else None)
        log(f"large form: one gradient ({dtype}, reorth={reorth}) in {t1 - t0:.2f} s")
        del ws, states, r, u, psi0, f
        torch.cuda.empty_cache()
    sec64, F64, g64, prof = res[(torch.complex64, True)]
    sec128, F128, g128, _ = res.get((torch.complex128, True), (float("nan"), None, None, None))
    out_plain = None
    if plain:
        secp, Fp, gp, _ = res[(torch.complex64, False)]
        out_plain = {"seconds": secp, "gradient_evals_per_s": 1.0 / secp,
                     "precision": "complex64 vectors, FP64 scalars, plain Lanczos",
                     "vs_full_reorth_c64": {"F_rel": abs(Fp - F64) / abs(F64),
                                            "grad_rel_l2": rel_l2(gp, g64)},
                     "vs_full_reorth_c128": None if F128 is None else {
                         "F_rel": abs(Fp - F128) / abs(F128), "grad_rel_l2": rel_l2(gp, g128)}}
    return {"study": "large form: one gradient evaluation",
            "workload": f"open XXZ L={c.L} (D={c.D}), J=1, Delta={c.Delta}, Hc=Sx site 1, N={c.N}, "
                        f"dt={c.dt}, m={c.m} full reorth, ckpt every {ckpt}, seed 4",
            "c64": {"seconds": sec64, "gradient_evals_per_s": 1.0 / sec64,
                    "precision": "complex64 vectors, FP64 scalars"},
            "c128": None if F128 is None else {"seconds": sec128,
                                                "gradient_evals_per_s": 1.0 / sec128},
            "mixed_vs_fp64_error": None if F128 is None else {
                "F_rel": abs(F64 - F128) / abs(F128),
                "grad_rel_l2": float(np.linalg.norm(g64 - g128) / np.linalg.norm(g128)),
                "grad_rel_inf": float(np.abs(g64 - g128).max() / np.abs(g128).max()),
                "F_fp64": F128},
            "plain_lanczos_c64": out_plain,
            "kernels_c64": {kk: {"launches_timed": v["launches"],
                                 "avg_us": v["ms"] / v["launches"] * 1e3,
                                 "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
                            for kk, v in prof.items() if v["launches"]},
            "peak_GBps": HBM_PEAK_GBS}


def m_eff_histogram(kg, torch, c, n_slices=40):
    """Krylov dimensions reached by the forward propagations of the first
    `n_slices` slices of the workload (complex64, the timed configuration),
    through krylov_expv with its m_eff output: {m_eff: count}."""
    h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    k = kg.Krylov(c.m, reorth=True)
    u, psi, _ = gpu_inputs(c, torch.complex64, torch)
    ws = kg.Workspace(h, k, torch.complex64)
    me = torch.zeros(n_slices, dtype=torch.int32, device="cuda")
    for j in range(n_slices):
        psi = kg.krylov_expv(h, float(c.u[j]), c.dt, psi, k, workspace=ws, m_eff=me[j:j + 1])
    vals, counts = np.unique(me.cpu().numpy(), return_counts=True)
    return {"sample": f"forward propagations of slices 1..{n_slices}, complex64",
            "histogram": {str(int(v)): int(n) for v, n in zip(vals, counts)}}


def time_variants(kg, torch, workloads, nodes=(2, 4), n_columns=4):
    """The gradient variants and operator control on the adjoint workload
    (L=20, N=400, m=20, checkpoints every 20, complex64 + FP64 scalars): one
    evaluation each, after a warm-up evaluation with the same buffers, of the
    zeroth-order, centred and first-order gradients, the quadrature gradient
    with each node count, and the operator-control gradient on `n_columns`
    random columns."""
    c = workloads.adjoint()
    ckpt = workloads.ADJOINT_CKPT_EVERY
    dtype = torch.complex64
    h = kg.XXZ(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    k = kg.Krylov(c.m, reorth=True)
    u, psi0, f = gpu_inputs(c, dtype, torch)
    ws = kg.Workspace(h, k, dtype, extended=True)
    states = kg.new_states(h, c.N, ckpt, dtype)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    rows = {}
    cases = [("zeroth_order", {}), ("centred", {"centred": True}),
             ("first_order", {"first_order": True})]
    cases += [(f"quadrature_{n}", {"nodes": n}) for n in nodes]
    kept = {}
    for name, kw in cases:
        sec, r = timed(lambda: kg.grape_gradient(h, u, c.dt, k, psi0, f, ckpt_every=ckpt,
                                                 states=states, workspace=ws, **kw))
        rows[name] = {"seconds": sec, "gradient_evals_per_s": 1.0 / sec}
        if name == "zeroth_order":
            kept["full"] = (float(r.F.cpu()), r.grad.cpu().numpy())
        log(f"variants: {name} in {sec:.3f} s")
    # plain Lanczos (three-term window, no re-orthogonalisation): time and its
    # difference from the fully re-orthogonalised gradient, both complex64, and
    # from the complex128 one
    kp = kg.Krylov(c.m, reorth=False)
    sec, r = timed(lambda: kg.grape_gradient(h, u, c.dt, kp, psi0, f, ckpt_every=ckpt,
                                             states=states, workspace=ws))
    Fp, gp = float(r.F.cpu()), r.grad.cpu().numpy()
    F0, g0 = kept["full"]
    u128, psi128, f128 = gpu_inputs(c, torch.complex128, torch)
    r128 = kg.grape_gradient(h, u128, c.dt, k, psi128, f128, ckpt_every=ckpt)
    F128, g128 = float(r128.F.cpu()), r128.grad.cpu().numpy()
    del r128
    rows["zeroth_order_plain_lanczos"] = {
        "seconds": sec, "gradient_evals_per_s": 1.0 / sec,
        "vs_full_reorth_c64": {"F_rel": abs(Fp - F0) / abs(F0), "grad_rel_l2": rel_l2(gp, g0)},
        "vs_full_reorth_c128": {"F_rel": abs(Fp - F128) / abs(F128),
                                "grad_rel_l2": rel_l2(gp, g128)},
        "full_reorth_c64_vs_c128": {"F_rel": abs(F0 - F128) / abs(F128),
                                    "grad_rel_l2": rel_l2(g0, g128)}}
    log(f"variants: plain Lanczos in {sec:.3f} s")
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    cols = torch.randn((n_columns, h.D), dtype=dtype, device="cuda", generator=g)
    cols /= torch.linalg.vector_norm(cols, dim=1, keepdim=True)
    tgts = torch.roll(cols, 1, dims=0).contiguous()
    cstates = torch.empty(0)

    def columns():
        nonlocal cstates
        r = kg.grape_gradient_columns(h, u, c.dt, k, cols, tgts, ckpt_every=ckpt,
                                      states=cstates if cstates.numel() else None, workspace=ws)
        cstates = r.states
        return r

    sec, _ = timed(columns)
    rows[f"columns_{n_columns}"] = {"seconds": sec, "gradient_evals_per_s": 1.0 / sec}
    log(f"variants: {n_columns} columns in {sec:.3f} s")
    base = rows["zeroth_order"]["seconds"]
    for v in rows.values():
        v["relative_to_zeroth_order"] = v["seconds"] / base
    return {"study": "gradient variants and operator control, one evaluation each",
            "workload": f"open XXZ L={c.L}, N={c.N}, dt={c.dt}, m={c.m} full reorth, "
                        f"ckpt every {ckpt}; columns: {n_columns} random normalised columns, "
                        "targets the same columns rolled by one, seed 11",
            "precision": "complex64 vectors, FP64 scalars", "rows": rows}


def time_pe(kg, torch, workloads, steps=2, reps=20):
    """The reduced basis on the transport task at L=25, K=12 (2,600,612
    amplitudes), N=200 slices of dt=0.1, m=10: centred gradients (the paper's
    production variant) in complex64 + FP64 scalars, timed over `steps`
    evaluations with sampled kernel timing, one FP64 evaluation for the error,
    and the gather H v alone in a HIP graph."""
    import numpy as np
    from paper_2010_03598_amd._graph import capture_guard
    t = workloads.pe_large()
    B = kg.ReducedBasis(t.L, t.K)
    tab = kg.pe_tables_host(t.L, t.K)
    h = kg.XXZ(t.L, t.J, t.Delta, kg.KG_HC_SZ, t.hc_sites)
    k = kg.Krylov(t.m)
    ckpt = 14
    u = torch.tensor(t.u, dtype=torch.float64, device="cuda")

    def unit(state):
        e = np.zeros(B.dim, dtype=np.complex128)
        rev = int(format(state, f"0{t.L}b")[::-1], 2)
        e[int(np.searchsorted(tab["reps"], min(state, rev)))] = 1.0
        return e

    e1, eD = unit(t.e1_state), unit(t.eD_state)
    res = {}
    for dtype, n in ((torch.complex64, steps), (torch.complex128, 1)):
        psi0 = torch.tensor(e1, dtype=dtype, device="cuda")
        f = torch.tensor(eD, dtype=dtype, device="cuda")
        ws = kg.ReducedWorkspace(B, k, dtype)
        states = kg.pe_states(B, t.N, ckpt, dtype)
        run = lambda: kg.grape_gradient_pe(h, B, u, t.dt, k, psi0, f, ckpt_every=ckpt,
                                           variant="centred", states=states, workspace=ws)
        r = run()
        torch.cuda.synchronize()
        prof = kg.profile(sample_every=8, max_launches=max(1024, n * 20000)) \
            if dtype == torch.complex64 else None
        if prof:
            prof.__enter__()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            r = run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if prof:
            prof.__exit__(None, None, None)
        res[dtype] = ((t1 - t0) / n, float(r.F.cpu()), r.grad.cpu().numpy(),
                      prof.result if prof else None)
        log(f"reduced basis: {n} centred gradients ({dtype}) in {t1 - t0:.3f} s")
        del ws, states
    sec, F64, g64, prof = res[torch.complex64]
    _, F128, g128, _ = res[torch.complex128]
    # the gather H v alone
    x = torch.tensor(workloads.random_state(np.random.default_rng(3), B.dim), dtype=torch.complex64,
                     device="cuda")
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            kg.xxz_pe_apply(h, B, 0.3, x, out=y)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with capture_guard(), torch.cuda.graph(graph):
        for _ in range(reps):
            kg.xxz_pe_apply(h, B, 0.3, x, out=y)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        e0.record()
        graph.replay()
        e1_.record()
        e1_.synchronize()
        best = min(best, e0.elapsed_time(e1_) * 1e-3 / reps)
    # x read, y written, the labels read, and the neighbour slots the slices
    # use (the labels' ranks instead when the basis has no neighbour table)
    if "slot_counts" in tab:
        hv_bytes = B.dim * (2 * x.element_size() + 4) + 256 * int(tab["slot_counts"].sum())
    else:
        hv_bytes = B.dim * (2 * x.element_size() + 8)
    kern = {c: {"launches_timed": v["launches"], "avg_us": v["ms"] / v["launches"] * 1e3,
                "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
            for c, v in prof.items() if v["launches"]}
    return {"metric": "reduced-basis centred gradient evals/s", "value": 1.0 / sec,
            "unit": "gradient evals/s", "ms_per_step": sec * 1e3, "steps": steps,
            "workload": f"e_1 -> e_D transport, L={t.L}, K={t.K}, dim={B.dim}, N={t.N}, "
                        f"dt={t.dt}, m={t.m} full reorth, ckpt every {ckpt}, seed 6",
            "precision": "complex64 vectors, FP64 scalars",
            "mixed_vs_fp64_error": {"F_rel": abs(F64 - F128) / abs(F128),
                                    "grad_rel_l2": float(np.linalg.norm(g64 - g128) /
                                                         np.linalg.norm(g128)),
                                    "F_fp64": F128},
            "fp64_ms_per_step": res[torch.complex128][0] * 1e3,
            "kernels": kern,
            "hv_pe": {"us_per_launch": best * 1e6, "algorithmic_bytes": hv_bytes,
                      "algorithmic_GBps": hv_bytes / best / 1e9,
                      "frac_of_peak": hv_bytes / best / 1e9 / HBM_PEAK_GBS,
                      "gather": "neighbour table" if "slot_counts" in tab else "ranks formed",
                      "timing": "HIP graph of the launches, best of 3 replays"}}


def fig2b(kg, torch, workloads, sizes, max_iter=300):
    """Run-time study of the transfer task (Fig. 2): for each (L, K), L-BFGS on
    centred GPU gradients in the reduced basis (complex128, each evaluation
    replayed from a captured HIP graph) from controls U(-1, 1) with M = 4D
    slices, dt = 0.5, m = 10 to I <= 1e-2.  Reports the total run time R, the
    iterations, and the elementary run time R~ = R / (iterations * M)."""
    import numpy as np
    from paper_2010_03598_amd import optimize
    rows = []
    for L, K in sizes:
        dim = kg.pe_dim(L, K)
        t = workloads.pe_task(L, K, 4 * dim, seed=5)
        B = kg.ReducedBasis(L, K)
        tab = kg.pe_tables_host(L, K)

        def unit(state):
            e = np.zeros(dim, dtype=np.complex128)
            rev = int(format(state, f"0{L}b")[::-1], 2)
            e[int(np.searchsorted(tab["reps"], min(state, rev)))] = 1.0
            return e

        psi0 = torch.tensor(unit(t.e1_state), device="cuda")
        f = torch.tensor(unit(t.eD_state), device="cuda")
        h = kg.XXZ(L, t.J, t.Delta, kg.KG_HC_SZ, t.hc_sites)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = optimize.optimize_controls(h, t.u, t.dt, kg.Krylov(t.m), psi0, f, I_target=1e-2,
                                         max_iter=max_iter, basis=B, graph=True)
        R = time.perf_counter() - t0
        row = {"L": L, "K": K, "D": dim, "M": t.N, "iterations": res.iterations,
               "evaluations": res.evaluations, "reason": res.reason, "I_final": res.f,
               "R_s": R, "R_tilde_us": R / max(res.iterations, 1) / t.N * 1e6,
               "s_per_evaluation": R / res.evaluations}
        log(json.dumps(row))
        rows.append(row)
    return rows


def batched_algorithmic_bytes(chains, ms):
    """Bytes the batched launch must move (complex64 vectors, 8 B per amplitude):
    per chain, 2N-1 Krylov calls (store-all: no recomputation), each with one
    tile pass per Lanczos step -- step 0 reads the input and writes y_0 and w'_0;
    a later step reads w'_{k-1} (its H v), u_{k-1}, y_{k-1} and the window
    before u_k and writes u_k, y_k and w'_k (the last step only u_k) -- and the
    combination reading m vectors and writing one; N brackets and the overlap
    read two vectors."""
    total = 0
    for c, m in zip(chains, ms):
        V = 8 << c.h.L
        per_call = 0
        for k in range(m):
            last = k == m - 1
            if k == 0:
                per_call += 1 + (0 if last else 2)
            else:
                before = 0 if last else (k if c.reorth else 1)
                per_call += 3 + before + (1 if last else 3)
        per_call += m + 1
        total += V * ((2 * c.N - 1) * per_call + 2 * c.N + 2)
    return total


def time_batched(kg, torch, workloads, steps=3, fp64=True):
    """The batched form on the 64-chain workload (L in 10..16, N in 50..300): the
    autotuned persistent launch (complex64 vectors, FP64 scalars; m per chain from
    the a-priori error bound), timed over `steps` launches, against the FP64 path
    run chain by chain with the same m (the batched kernel has no complex128
    form)."""
    import numpy as np
    from paper_2010_03598_amd import batched
    wl = workloads.batched()
    chains = batched.from_workload(wl)
    b, info = batched.autotune(chains, caps=(2, 4, 8, 16, 32, 64))
    b.gradient()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.gradient()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    b.check_status()
    nbytes = batched_algorithmic_bytes(chains, b.m)
    out = {"chains": len(chains), "value": len(chains) / sec, "unit": "chain gradient evals/s",
           "ms_per_launch": sec * 1e3, "launches": steps, "team_cap": info["best_cap"],
           "m": sorted(set(b.m)), "m_per_chain": list(b.m), "team_per_chain": list(b.teams),
           "element_slices": int(sum(c.N << c.h.L for c in chains)),
           "algorithmic_GB_per_launch": nbytes / 1e9,
           "algorithmic_GBps": nbytes / sec / 1e9,
           "frac_of_peak": nbytes / sec / 1e9 / HBM_PEAK_GBS,
           "note": "vectors of 8-512 KiB: the working set sits in the caches, so the "
                   "fraction of the HBM peak can exceed what HBM alone would allow"}
    if fp64:
        F32 = b.F.cpu().numpy()
        errs_g, errs_F = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = []
        for i, c in enumerate(chains):
            r = kg.grape_gradient(c.h, c.u.to("cuda"), c.dt, kg.Krylov(b.m[i]),
                                  c.psi0.to(torch.complex128).to("cuda"),
                                  c.target.to(torch.complex128).to("cuda"))
            res.append(r)
        torch.cuda.synchronize()
        sec64 = time.perf_counter() - t0
        for i, r in enumerate(res):
            g64 = r.grad.cpu().numpy()
            g32 = b.grad_of(i).cpu().numpy()
            errs_g.append(float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64)))
            F64 = float(r.F.cpu())
            errs_F.append(abs(float(F32[i]) - F64) / F64)
        out["fp64_chain_by_chain"] = {"value": len(chains) / sec64, "unit": "chain gradient evals/s",
                                      "seconds": sec64}
        out["mixed_vs_fp64_error"] = {"grad_rel_l2_max": max(errs_g), "F_rel_max": max(errs_F)}
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lanczos_L20_c64_traffic.md")
KERNEL_OF_CLASS = {"pass_a": "k_pass_a", "pass_b": "k_pass_b", "combine": "k_combine"}


def sources_sha256():
    """Hash of the HIP/C++ sources the counters in TRAFFIC_FILE were taken on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2010_03598_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(cls):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 counter
    summary, or None when it was taken on other sources (or is missing)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    tag = "<!-- traffic-json: "
    if tag not in text:
        return None
    rec = json.loads(text.split(tag, 1)[1].split(" -->", 1)[0])
    if rec.get("sources_sha256") != sources_sha256():
        return None
    k = rec.get("per_kernel", {}).get(KERNEL_OF_CLASS.get(cls, ""))
    return None if k is None else float(k["hbm_bytes_per_launch"])


def cpu_baseline(c, budget_s=20.0):
    """The oracle (NumPy/SciPy FP64) on a bounded prefix of the same workload:
    forward Krylov propagations of the first slices, extrapolated to the
    oracle's full gradient (2N-1 propagations + N brackets, store-all)."""
    from oracle import krylov as ok
    from oracle import model as om

    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    t_build = time.perf_counter()
    ch = om.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    t_build = time.perf_counter() - t_build
    psi = c.psi0.copy()
    n_done = 0
    t0 = time.perf_counter()
    while True:
        psi = ok.expv(lambda v, uj=c.u[n_done]: ch.apply(uj, v), psi, c.dt, c.m, True)
        n_done += 1
        if time.perf_counter() - t0 > budget_s or n_done >= c.N:
            break
    t_call = (time.perf_counter() - t0) / n_done
    tb = time.perf_counter()
    np.vdot(c.target, ch.apply_hc(psi))
    t_bracket = time.perf_counter() - tb
    per_grad = t_call * (2 * c.N - 1) + t_bracket * c.N
    return {"value": 1.0 / per_grad, "unit": "gradient evals/s", "cores": int(blas_threads),
            "kind": "oracle",
            "sample": f"{n_done} Krylov propagations (m={c.m}, L={c.L}) of the first slices, "
                      f"{t_call:.2f} s each, plus one bracket; extrapolated to 2N-1={2 * c.N - 1} "
                      f"propagations and N={c.N} brackets per gradient (sparse-matrix build "
                      f"{t_build:.1f} s excluded)",
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--fp64-warmup", type=int, default=1)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the L=24, N=500 large-form leg of the default run")
    ap.add_argument("--profile-every", type=int, default=64,
                    help="time every n-th Krylov call's kernels with HIP events (0: off)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-pe", action="store_true", help="skip the reduced-basis leg")
    ap.add_argument("--only-batched", action="store_true",
                    help="time only the 64-chain batched launch (no FP64 comparison)")
    ap.add_argument("--only-pe", action="store_true",
                    help="run only the reduced-basis leg (--steps evaluations) and print its JSON")
    ap.add_argument("--hv-only", type=int, default=0, metavar="L",
                    help="run only the graph-timed H v at this L (complex64 and complex128)")
    ap.add_argument("--fig2b", type=str, default="", metavar="L:K,L:K,...",
                    help="run only the optimisation run-time study at these sizes, e.g. 8:4,10:4")
    ap.add_argument("--large", action="store_true",
                    help="time one gradient of the L=24, N=500 large form (c64 and c128) only")
    ap.add_argument("--large-no-fp64", action="store_true", help="with --large: complex64 only")
    ap.add_argument("--variants", action="store_true",
                    help="time only the gradient variants and operator control at L=20")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (calibrates the HBM byte "
                         "counters against a kernel of known traffic) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the chain's "
              "slices are sequential and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n}))
        return

    import paper_2010_03598_amd as kg
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only_batched:
        print(json.dumps(time_batched(kg, torch, workloads, fp64=False)), flush=True)
        return
    if args.only_pe:
        print(json.dumps(time_pe(kg, torch, workloads, steps=args.steps)), flush=True)
        return
    if args.hv_only:
        print(json.dumps({"hv": [time_hv(kg, torch, args.hv_only, dt, reps=20)
                                 for dt in (torch.complex64, torch.complex128)]}), flush=True)
        return
    if args.fig2b:
        sizes = [tuple(int(v) for v in p.split(":")) for p in args.fig2b.split(",")]
        print(json.dumps({"study": "transfer-task optimisation run time (Fig. 2)",
                          "rows": fig2b(kg, torch, workloads, sizes)}), flush=True)
        return
    if args.large:
        print(json.dumps(time_large(kg, torch, workloads, not args.large_no_fp64)), flush=True)
        return
    if args.variants:
        print(json.dumps(time_variants(kg, torch, workloads)), flush=True)
        return
    c = workloads.adjoint()
    ckpt = workloads.ADJOINT_CKPT_EVERY
    log(f"workload: L={c.L} N={c.N} m={c.m} dt={c.dt} Delta={c.Delta} ckpt_every={ckpt}")

    sec64, F64, g64, prof = time_gradients(kg, torch, c, torch.complex64, ckpt, args.steps,
                                           args.warmup, args.profile_every)
    if args.fp64_steps > 0:
        sec128, F128, g128, _ = time_gradients(kg, torch, c, torch.complex128, ckpt,
                                               args.fp64_steps, args.fp64_warmup, 0)
    else:
        sec128, F128, g128 = float("nan"), F64, g64
    errF = abs(F64 - F128) / abs(F128)
    errg = float(np.linalg.norm(g64 - g128) / np.linalg.norm(g128))
    errg_inf = float(np.abs(g64 - g128).max() / np.abs(g128).max())

    if prof is None:
        print(json.dumps({"metric": METRIC, "value": 1.0 / sec64, "unit": "gradient evals/s",
                          "ms_per_step": sec64 * 1e3, "profile": "off"}), flush=True)
        return
    # dominant kernel: the class with the largest sampled time
    dom = max(("pass_a", "pass_b", "combine", "bracket", "overlap"), key=lambda k: prof[k]["ms"])
    d = prof[dom]
    per_launch_s = d["ms"] / d["launches"] * 1e-3
    bytes_per_launch = d["bytes"] / d["launches"]
    achieved = bytes_per_launch / per_launch_s / 1e9
    # every sampled record stands for profile_every launches of its class, so
    # the sampled bytes scale to the whole step's algorithmic bytes
    step_bytes = sum(v["bytes"] for v in prof.values()) * args.profile_every / args.steps
    classes = {k: {"launches_timed": v["launches"],
                   "avg_us": (v["ms"] / v["launches"] * 1e3) if v["launches"] else None,
                   "avg_algorithmic_GB": (v["bytes"] / v["launches"] / 1e9) if v["launches"] else None,
                   "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] else None}
               for k, v in prof.items() if v["launches"]}

    hv20 = time_hv(kg, torch, 20, torch.complex64)
    hv24 = time_hv(kg, torch, 24, torch.complex64, reps=20)
    hv24_128 = time_hv(kg, torch, 24, torch.complex128, reps=20)
    copy_bw = time_copy(torch)
    for rec in (hv20, hv24, hv24_128):
        rec["frac_of_copy"] = rec["algorithmic_GBps"] / copy_bw["GBps"]
    # a copy whose buffers fit in the Infinity Cache: the reference for the
    # cache-resident batched form
    copy_cached = time_copy(torch, mib=64, reps=100)

    bat = None if args.no_batched else time_batched(kg, torch, workloads)
    if bat:
        bat["cache_resident_copy_GBps"] = copy_cached["GBps"]
        bat["frac_of_cache_resident_copy"] = bat["algorithmic_GBps"] / copy_cached["GBps"]
    if bat:
        log(f"batched: {bat['value']:.1f} chain gradient evals/s")
    pe = None if args.no_pe else time_pe(kg, torch, workloads)
    if pe:
        log(f"reduced basis: {pe['value']:.2f} gradient evals/s")
    large = None if args.no_large else time_large(kg, torch, workloads)
    meff = m_eff_histogram(kg, torch, c)
    cpu = None if args.no_cpu else cpu_baseline(c, args.cpu_budget)

    out = {
        "metric": METRIC,
        "value": 1.0 / sec64,
        "unit": "gradient evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "adjoint: open XXZ L=20 (D=2^20), J=1, Delta=1, Hc=Sx site 1, "
                               "N=400, dt=0.05, m=20 full reorth, ckpt every 20, seed 2; "
                               "step = F = fidelity(u) and F.backward() through the "
                               "torch.autograd.Function",
                   "L": c.L, "N": c.N, "m": c.m, "dt": c.dt, "ckpt_every": ckpt,
                   "precision": "complex64 vectors, FP64 scalars", "parallelism": "1 GPU"},
        "fp64": {"value": 1.0 / sec128, "unit": "gradient evals/s", "ms_per_step": sec128 * 1e3,
                 "steps": args.fp64_steps, "warmup": args.fp64_warmup},
        "mixed_vs_fp64_error": {"F_rel": errF, "grad_rel_l2": errg, "grad_rel_inf": errg_inf,
                                "F_fp64": F128},
        "hv": {"L20_c64": hv20, "L24_c64": hv24, "L24_c128": hv24_128,
               "peak_GBps": HBM_PEAK_GBS, "copy": copy_bw},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(dom),
                     "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT),
                     "avg_us": per_launch_s * 1e6, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "sampled_launches": d["launches"],
                     "concurrency": "the costate sweep's launches run beside the segment "
                                    "recomputation's, on a second stream: each launch's "
                                    "duration includes the other stream's share of the chip",
                     "step_algorithmic_GB": step_bytes / 1e9,
                     "step_achieved": step_bytes / sec64 / 1e9,
                     "step_frac": step_bytes / sec64 / 1e9 / HBM_PEAK_GBS},
        "kernels": classes,
        "m_eff": meff,
        "batched": bat,
        "reduced_basis": pe,
        "large": large,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
