"""Throughput of the semi-explicit eddy-current step on one MI355X.

Workload: the nonlinear 48^3-cell FIT grid (unit cube, PEC walls) with a
16^3-cell Brauer iron conductor (sigma = 2e6 S/m, nu = 3.8 exp(2.17 B^2) +
396.2), a coil current ramped linearly over 1000 steps, dt = half the
explicit-Euler stability bound (eq. 8, power method on the GPU), PCG to a
relative residual of 1e-8.  Each timed step is one explicit Euler step of
eqs. (6)-(7): two pseudo-inverse solves (source and coupling sequences),
their start vectors and history updates, and the conducting-region update.

The headline value is steps/s with SPE start vectors (window m = 8) replayed
from a captured HIP graph; CSPE (the growing basis: SPE with up to 19
columns), ZERO (plain zero-start PCG), PREV and POD (20 snapshots, at most
10 modes) run the same steps for comparison.
Inputs are synthetic (seeded geometry; no benchmark data).

Usage: python bench.py [--steps K] [--warmup W] [--methods spe,cspe,pod,prev,zero]
                       [--cpu-steps S] [--no-cpu] [--no-probe] [--no-c3] [--no-adjoint]
                       [--no-batch] [--c3-check-steps S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
COPY_BYTES = 512 << 20
METRIC = "Euler steps/sec at rel. residual 1e-8; PCG iters/step; SpMV HBM GB/s"


# captured PCG launches per solve beyond the warm-up median
BUDGET_MARGIN = 0
# at most this many iteration kernels per captured solve on grids that run the
# node-parallel iteration; a longer solve continues in the persistent tail
# (an iteration there costs about 3 us more than a launched one at 48^3, a
# launch that finds the solve finished 1-2 us), so a short warm-up whose last
# steps still need many iterations (an SPE window that is not yet full)
# cannot make every replay issue dozens of kernels that find the solve
# finished.  48^3, SPE: caps of 12/16/20/24/28/32/40 gave 2275/2417/2441/
# 2440/2419/2353/2215 steps/s over steps 6-25 (after 5 warm-up steps, 20.3
# PCG iterations per step) and 3938/3896/3896/3899/3899/3896/3889 over steps
# 41-240 (warm-up median 13, 6.15 iterations per step)
BUDGET_CAP_NODE = 24
# The cap per start method: only the SPE windows shrink their solves' needs
# after a short warm-up; the other methods need about as many iterations in
# the timed steps as in the last warm-up ones, and a cap would only move
# their iterations into the slower tail.  Steps 6-25 at 48^3, caps 24/48/96/
# none: POD 817/880/921/919 steps/s, PREV 304/322/366/406, ZERO 273/288/323/
# 361, the growing SPE basis 2469/2082/1685/1682.
METHOD_BUDGET_CAP = {"spe": BUDGET_CAP_NODE, "cspe": BUDGET_CAP_NODE, "pod": None,
                     "prev": None, "zero": None}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1611_06721_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def method_opts(ec, name, rtol, graph_iters=(0, 0)):
    kw = dict(rtol=rtol, maxit=100000, graph_iters=graph_iters)
    if name == "spe":
        return ec.step_opts(ec.SV_SPE, window=8, pod_kmax=8, **kw)
    if name == "cspe":       # the paper's growing basis: up to 19 columns
        return ec.step_opts(ec.SV_SPE, window=19, pod_kmax=8, **kw)
    if name == "pod":
        return ec.step_opts(ec.SV_POD, window=20, pod_kmax=10, pod_eps=1e-4, **kw)
    if name == "prev":
        return ec.step_opts(ec.SV_PREV, window=1, **kw)
    return ec.step_opts(ec.SV_ZERO, window=1, **kw)


def graph_budgets(its, warmup, cap=None):
    """Iteration kernels per captured solve (source, coupling) from the
    per-solve iteration counts of the eager warm-up (its: source and coupling
    counts of each step, interleaved).  Typical, not worst-case, counts: the
    median over the last min(W/2, W-2) warm-up steps (never the first step
    from rest while W > 2); a longer solve is finished by the persistent tail
    kernel.  A sequence that needs no iteration (the source solves once their
    window holds the source shape) gets two: an iteration kernel, then a tail
    launch, both of which find the solve finished.  At most `cap` each."""
    import numpy as np
    its = np.asarray(its)
    h = min(warmup // 2, max(warmup - 2, 0))
    med = [int(np.median(its[2 * h + q::2])) for q in (0, 1)]
    budgets = [max(1, v + BUDGET_MARGIN) if v > 0 else 2 for v in med]
    if cap:
        budgets = [min(b, cap) for b in budgets]
    return budgets


def run_method(ec, torch, G, name, dt, steps, warmup, rtol, make_opts=None, cap=None):
    """`warmup` eager steps from rest (not timed; they also fill the start-vector
    histories), then `steps` replays of the captured step, continuing the same
    run, timed with events on the library's stream.  Each captured solve issues
    a fixed number of PCG iteration kernels (`graph_budgets`: the last warm-up
    steps, capped at `cap`); a solve that needs more continues in one
    persistent launch.  If a solve still fails (maxit), the measurement is
    repeated with twice the budget."""
    if make_opts is None:
        def make_opts(graph_iters=(0, 0)):
            return method_opts(ec, name, rtol, graph_iters)
    budgets = None
    for attempt in range(4):
        A = G.zeros()
        G.set_state(A, rtol=rtol)
        info = G.info(2 * warmup)
        G.run(A, 0, warmup, dt, make_opts(), info=info)
        its = ec.info_array(info)["iters"]
        if budgets is None:
            budgets = graph_budgets(its, warmup, cap)
        G.counters_reset()
        graph = G.graph_capture(A, dt, make_opts(tuple(budgets)))
        torch.cuda.synchronize()
        s = G.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            graph.launch_raw()
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        c = G.counters()
        graph.close()
        if c["worst_status"] == 0 and c["steps"] == steps:
            break
        log(f"[bench] {name}: budget {budgets} insufficient (status {c['worst_status']}), retry")
        budgets = [2 * b for b in budgets]
    else:
        raise RuntimeError(f"{name}: solves did not converge within the graph budget")
    return {
        "steps_per_s": steps / (ms * 1e-3),
        "ms_per_step": ms / steps,
        "iters_per_step": (c["iters_src"] + c["iters_cpl"]) / steps,
        "iters_src_per_step": c["iters_src"] / steps,
        "iters_cpl_per_step": c["iters_cpl"] / steps,
        "graph_iteration_budget": list(budgets),
        "final_state_norm": float(A.norm().item()),
    }, A


def precision_c3(ec, torch, steps, warmup, check_steps, rtol=1e-8, N=128):
    """FP64 PCG vs FP32 inner PCG in the FP64 residual loop on the 128^3
    Brauer grid, SPE m = 8, the same captured-step measurement as the
    headline (with its own `warmup`).  The first `check_steps` steps from
    rest are also run eagerly in both precisions and their states kept on the
    host: the CPU leg compares them with the FP64 oracle step by step."""
    import synth
    G = ec.Problem(synth.nonlinear(N), window_cap=8)
    lam = G.cfl(iters=40, rtol=1e-10)
    dt = 0.5 * 2.0 / lam
    out, finals, traj = {}, {}, {}
    for prec, tag in ((ec.PREC_FP64, "fp64"), (ec.PREC_FP32_REFINED, "fp32_refined")):
        def make_opts(graph_iters=(0, 0), prec=prec):
            return ec.step_opts(ec.SV_SPE, window=8, rtol=rtol, maxit=100000, precision=prec,
                                inner_rtol=1e-5, inner_maxit=200, outer_max=4,
                                graph_iters=graph_iters)
        if check_steps > 0:
            A = G.zeros()
            G.set_state(A, rtol=rtol)
            rec = []
            for m in range(1, check_steps + 1):
                G.step(A, m, dt, make_opts())
                rec.append(A.cpu().numpy())
            traj[tag] = rec
        r, A = run_method(ec, torch, G, "spe", dt, steps, warmup, rtol, make_opts)
        out[tag] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
        finals[tag] = A.clone()
        log(f"[bench] 128^3 {tag}: {r['steps_per_s']:.1f} steps/s, {r['iters_per_step']:.2f} iters/step")
    a64, a32 = finals["fp64"], finals["fp32_refined"]
    out["final_state_rel_diff_fp32_vs_fp64"] = float((a32 - a64).norm() / a64.norm())
    out["workload"] = (f"nonlinear {N}^3, {steps} captured steps after {warmup} eager warm-up "
                       f"steps, SPE m=8, rtol {rtol:g}")
    out["speedup_fp32_refined"] = round(out["fp32_refined"]["steps_per_s"] /
                                        out["fp64"]["steps_per_s"], 3)
    G.close()
    torch.cuda.empty_cache()
    return out, {"N": N, "dt": dt, "rtol": rtol, "traj": traj}


def adjoint_c5(ec, torch, steps=500, every=50, N=64, rtol=1e-8, check_steps=100):
    """Hand-written adjoint on the 64^3 Brauer grid: forward steps with a
    checkpoint every `every` steps (Joule loss), then the backward pass
    (segment recompute + adjoint recursion, dL/dsigma and dL/dk1), timed with
    events; the gradients of a `check_steps` run at rtol 1e-12 are compared
    with central differences of the GPU loss."""
    import synth
    wl = synth.nonlinear(N)
    G = ec.Problem(wl, window_cap=8)
    dt = 0.5 * 2.0 / G.cfl(iters=40, rtol=1e-10)
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=rtol)
    ws = G.adjoint_workspace(steps, every)
    s = G.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    G.counters_reset()
    A = G.zeros()
    ev[0].record(s)
    loss = G.adjoint_forward(A, steps, dt, every, opts, ws)
    ev[1].record(s)
    c_fwd = G.counters()
    g = G.adjoint_backward(steps, dt, every, opts, ws, 1)
    ev[2].record(s)
    ev[2].synchronize()
    c_all = G.counters()
    t_f, t_b = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    gr = g.cpu().numpy()
    out = {"workload": f"nonlinear {N}^3, {steps} steps, checkpoint every {every}, SPE m=8, "
                       f"rtol {rtol:g}",
           "loss": float(loss.item()), "dL_dsigma": float(gr[0]), "dL_dk1": float(gr[1]),
           "forward_steps_per_s": round(steps / (t_f * 1e-3), 2),
           "backward_steps_per_s": round(steps / (t_b * 1e-3), 2),
           "forward_iters_per_step": round((c_fwd["iters_src"] + c_fwd["iters_cpl"]) / steps, 3),
           "adjoint_iters_per_step": round(c_all["iters_adj"] / steps, 3),
           "workspace_MB": round(ws[2] / 2 ** 20, 1)}
    del ws
    # gradient check at rtol 1e-12 on the first check_steps steps
    m = wl.materials[0]
    o12 = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-12)
    wsc = G.adjoint_workspace(check_steps, every)
    G.set_material(1, m.sigma, m.k1, m.k2, m.k3)
    G.adjoint_forward(G.zeros(), check_steps, dt, every, o12, wsc)
    gc = G.adjoint_backward(check_steps, dt, every, o12, wsc, 1).cpu().numpy()

    def L(sigma, k1):
        G.set_material(1, sigma, k1, m.k2, m.k3)
        return float(G.adjoint_forward(G.zeros(), check_steps, dt, every, o12, wsc).item())
    # relative steps 1e-6 (the workload's) and 1e-4: the loss carries the
    # solves' 1e-12 residual noise, which a step of 1e-6 amplifies 1e6 times
    for key, h in (("fd_check", 1e-6), ("fd_check_h1e-4", 1e-4)):
        fd_s = (L(m.sigma * (1 + h), m.k1) - L(m.sigma * (1 - h), m.k1)) / (2 * h * m.sigma)
        fd_k = (L(m.sigma, m.k1 * (1 + h)) - L(m.sigma, m.k1 * (1 - h))) / (2 * h * m.k1)
        out[key] = {"steps": check_steps, "rtol": 1e-12, "h": h,
                    "rel_err_dsigma": float(abs(gc[0] - fd_s) / abs(fd_s)),
                    "rel_err_dk1": float(abs(gc[1] - fd_k) / abs(fd_k))}
    del wsc
    G.close()
    torch.cuda.empty_cache()
    return out


def batch_c4(ec, torch, steps=300, warmup=20, count=64, rtol=1e-8):
    """64 uneven instances (seeded draws: N in [16, 64], sigma = 10^U(5,7),
    Brauer coefficients within 10 %), each at half its own stability bound,
    SPE m = 8.  After `warmup` eager batched steps, `steps` replays of one
    graph holding every instance's step (batched PCG launches, autotuned
    grids, the persistent batched tail past the budget) are timed; then with
    every batched PCG solve as one persistent launch (budget 1); then the
    same steps as 64 per-instance graphs launched one after the other."""
    import numpy as np
    import synth
    wls = synth.batch_workloads(count)
    s = torch.cuda.Stream()
    probs = [ec.Problem(w, window_cap=8, stream=s) for w in wls]
    dts = [0.5 * 2.0 / p.cfl(iters=15, rtol=1e-8) for p in probs]
    B = ec.Batch(probs)
    cache = os.path.expanduser("~/.cache/paper_1611_06721_amd/batch_tiles.txt")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tiles, tuned_us = B.autotune(cache)
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=rtol)
    out = {"workload": f"{count} instances, N in [16, 64], {steps} steps, SPE m=8, rtol {rtol:g}",
           "edges_total": int(sum(p.n_pad for p in probs)),
           "autotuned_tiles_per_block": tiles, "batched_iteration_us": round(tuned_us, 2)}
    for mode in ("batched_graph", "batched_persistent", "per_instance_graphs"):
        As = [p.zeros() for p in probs]
        for p, A in zip(probs, As):
            p.set_state(A, rtol=rtol)
        B.run(0, warmup, dts, As, opts)
        # iteration budget per solve: the median over the instances of the
        # largest count of the last warm-up steps; solves that need more
        # continue in the persistent batched tail
        mx = np.zeros((len(probs), 2), dtype=np.int64)
        for _ in range(6):
            for p in probs:
                p.counters_reset()
            B.step(dts, As, opts)
            for i, p in enumerate(probs):
                c = p.counters()
                mx[i] = np.maximum(mx[i], [c["iters_src"], c["iters_cpl"]])
        budgets = [max(2, int(np.median(mx[:, q]))) for q in (0, 1)]
        if mode == "batched_persistent":
            budgets = [1, 1]         # every batched PCG solve: one persistent launch
        gopts = ec.step_opts(ec.SV_SPE, window=8, rtol=rtol, graph_iters=tuple(budgets))
        for p in probs:
            p.counters_reset()
        if mode != "per_instance_graphs":
            graphs = [B.graph_capture(dts, As, gopts)]
        else:
            # each problem alone on its own default PCG grid (the batch had
            # set the grids of the handles it borrows)
            # as chains: with 64 different graphs launched in turn, graphs
            # whose history pushes fork onto a branch ran slower (2,128
            # against 2,309 instance-steps/s on the same box)
            for p in probs:
                p.set_pcg_kernel(-1)
            sopts = ec.step_opts(ec.SV_SPE, window=8, rtol=rtol, graph_iters=tuple(budgets),
                                 graph_serial=True)
            graphs = [p.graph_capture(A, dt, sopts) for p, A, dt in zip(probs, As, dts)]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            for g in graphs:
                g.launch_raw()
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        cs = [p.counters() for p in probs]
        for g in graphs:
            g.close()
        del graphs
        iters = sum(c["iters_src"] + c["iters_cpl"] for c in cs)
        out[mode] = {"instance_steps_per_s": round(count * steps / (ms * 1e-3), 1),
                     "batch_steps_per_s": round(steps / (ms * 1e-3), 2),
                     "ms_per_batch_step": round(ms / steps, 3),
                     "iters_per_instance_step": round(iters / (count * steps), 3),
                     "graph_iteration_budget": budgets,
                     "worst_status": min(c["worst_status"] for c in cs)}
        log(f"[bench] batch {mode}: {out[mode]['instance_steps_per_s']} instance-steps/s")
    out["speedup_batched"] = round(out["batched_graph"]["instance_steps_per_s"] /
                                   out["per_instance_graphs"]["instance_steps_per_s"], 3)
    out["tail_blocks"] = "persistent batched tail: at most 2 blocks per CU, all resident"
    B.close()
    for p in probs:
        p.close()
    del B, probs
    torch.cuda.empty_cache()
    return out


def implicit_vs_explicit(ec, torch, dt_e, steps_e=400, factor=20, warm=20, rtol=1e-8):
    """The paper's comparison (Sec. IV): the semi-explicit scheme with SPE
    start vectors against implicit Euler with Newton over the same simulated
    interval.  48^3 Brauer grid with the time-indexed source
    J0 (1 - exp(-t/tau)), tau = 300 dt_e (a ramp indexed by steps would run
    at another speed under another dt).  After `warm` explicit steps from rest
    (untimed, also the implicit run's start), steps_e explicit steps of dt_e
    (captured SPE step) and steps_e / factor implicit steps of factor dt_e
    (Newton to 1e-8, GMRES(20) to 1e-4, K_n^+ solves to 1e-10 from zero) are
    timed on the device / by the host clock (the implicit call synchronises)."""
    import copy
    import numpy as np
    import synth
    wl = copy.deepcopy(synth.nonlinear(48))
    wl.waveform = synth.WF_EXP
    wl.tau = 300 * dt_e
    G = ec.Problem(wl, window_cap=8)
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=rtol)
    A = G.zeros()
    G.set_state(A, rtol=rtol)
    info = G.info(2 * warm)
    G.run(A, 0, warm, dt_e, opts, info=info)
    A_w = A.clone()
    its = ec.info_array(info)["iters"]
    budgets = [max(2, min(int(np.median(its[q::2][-4:])), BUDGET_CAP_NODE)) for q in (0, 1)]
    graph = G.graph_capture(A, dt_e, ec.step_opts(ec.SV_SPE, window=8, rtol=rtol,
                                                  graph_iters=tuple(budgets)))
    G.counters_reset()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(G.stream)
    for _ in range(steps_e):
        graph.launch_raw()
    e1.record(G.stream)
    e1.synchronize()
    t_e = e0.elapsed_time(e1) * 1e-3
    ce = G.counters()
    graph.close()
    A_e = A.clone()
    # implicit: from the same state, steps of factor dt_e (t = m dt_i)
    dt_i = factor * dt_e
    G.set_state(A_w, rtol=1e-10)
    Ai = A_w.clone()
    m0 = warm // factor
    tot = {"newton_iters": 0, "gmres_iters": 0, "kn_solves": 0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m in range(m0 + 1, m0 + steps_e // factor + 1):
        r = G.implicit_step(Ai, m, dt_i, newton_rtol=1e-8, max_newton=20, gmres_m=20,
                            gmres_max=400, gmres_rtol=1e-4, inner_rtol=1e-10,
                            method=ec.SV_ZERO)
        for k in tot:
            tot[k] += r[k]
        if r["status"] != 0:
            raise RuntimeError(f"implicit step {m}: {r}")
    torch.cuda.synchronize()
    t_i = time.perf_counter() - t0
    ni = steps_e // factor
    out = {"workload": f"nonlinear 48^3, source 1 - exp(-t/tau), tau = 300 dt_e, interval "
                       f"{steps_e} dt_e after {warm} steps",
           "explicit": {"dt": dt_e, "steps": steps_e, "seconds": round(t_e, 5),
                        "pcg_iters_per_step": round((ce["iters_src"] + ce["iters_cpl"]) /
                                                    steps_e, 3)},
           "implicit": {"dt": dt_i, "steps": ni, "seconds": round(t_i, 5),
                        "newton_per_step": round(tot["newton_iters"] / ni, 2),
                        "gmres_per_step": round(tot["gmres_iters"] / ni, 2),
                        "kn_solves_per_step": round(tot["kn_solves"] / ni, 2)},
           "explicit_over_implicit_time": round(t_e / t_i, 4),
           "final_state_rel_diff": float((Ai - A_e).norm() / A_e.norm())}
    G.close()
    torch.cuda.empty_cache()
    return out


def stability_and_mass(ec, torch, dt, rtol=1e-8, warm=40, steps=200):
    """The device stability estimate (power method on M_c^-1 (J_N - S), eq. 8)
    at the state after `warm` SPE steps, 30 iterations with zero- and
    SPE-started inner solves (device events); and explicit steps with the
    consistent conductivity matrix (M_c solves with zero and SPE starts, dt
    of the lumped bound / 9: the consistent matrix is at least 1/9 of the
    lumped one), `steps` captured steps after `warm` eager ones."""
    import numpy as np
    import synth
    G = ec.Problem(synth.nonlinear(48), window_cap=8)
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=rtol)
    A = G.zeros()
    G.set_state(A, rtol=rtol)
    G.run(A, 0, warm, dt, opts)
    out = {}
    for meth, tag in ((ec.SV_ZERO, "zero"), (ec.SV_SPE, "spe")):
        lam = G.tensor(np.zeros(1))
        G.counters_reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        G.cfl_estimate(A, iters=30, rtol=1e-10, method=meth, window=8, jacobian=True, lam=lam)
        e1.record(G.stream)
        e1.synchronize()
        out[f"cfl_estimate_{tag}"] = {"ms": round(e0.elapsed_time(e1), 3),
                                      "lambda_jacobian": float(lam.item())}
    out["cfl_estimate_note"] = (f"30 power iterations on M_c^-1 (J_N - S) at the state after {warm} "
                                f"SPE steps, inner solves to 1e-10; the secant bound of dt: "
                                f"lambda = {2.0 / dt * 0.5:.6g}")
    dtc = dt / 9.0
    for meth, tag in ((ec.SV_ZERO, "zero"), (ec.SV_SPE, "spe")):
        G.set_mass(ec.MASS_CONSISTENT, meth, window=8, rtol=1e-10, maxit=40)
        A = G.zeros()
        G.set_state(A, rtol=rtol)
        G.run(A, 0, warm, dtc, opts)
        graph = G.graph_capture(A, dtc, ec.step_opts(ec.SV_SPE, window=8, rtol=rtol,
                                                     graph_iters=(2, BUDGET_CAP_NODE)))
        G.counters_reset()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        for _ in range(steps):
            graph.launch_raw()
        e1.record(G.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        c, mc = G.counters(), G.mass_counters()
        graph.close()
        out[f"consistent_mass_{tag}"] = {
            "steps_per_s": round(steps / (ms * 1e-3), 1),
            "mass_iters_per_step": round(mc["iters"] / max(mc["solves"], 1), 2),
            "pcg_iters_per_step": round((c["iters_src"] + c["iters_cpl"]) / steps, 2),
            "worst_status": c["worst_status"]}
    out["consistent_mass_note"] = (f"48^3, dt = lumped bound / 9, SPE K_n starts, {steps} captured "
                                   f"steps after {warm}; M_c solves to 1e-10, 40 kernels budgeted")
    G.set_mass(ec.MASS_LUMPED, ec.SV_SPE, window=8, rtol=1e-10, maxit=40)
    G.close()
    torch.cuda.empty_cache()
    return out


def time_cg_iteration(ec, torch, G, reps=400):
    """Average duration of one PCG iteration kernel (FP64, every iteration
    active): solves that run exactly 100 and 100 + reps iterations, timed with
    events on the library's stream; the difference divided by reps removes the
    per-solve kernels (init, final record) and the host polling."""
    b = torch.randn(G.n_pad, dtype=torch.float64, device=G.device)
    b = G.apply(ec.OP_KN, b)             # a consistent right-hand side
    x = G.zeros()

    def solve_ms(n):
        ms = None
        for _ in range(2):               # the first run sets the chunk hint to n
            s = G.stream
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            G.solve(b, x=x, method=ec.SV_ZERO, rtol=1e-300, maxit=n)
            e1.record(s)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
        return ms
    short = solve_ms(100)
    long_ = solve_ms(100 + reps)
    return 1e3 * (long_ - short) / reps


def traffic_record(kernel, workload):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, scaled by a
    copy kernel) if recorded for the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    ent = rec.get(f"{kernel}@{workload}")
    if not ent or ent.get("sources") != kernel_sources_hash():
        return None
    return ent.get("bytes_per_launch")


def host_info():
    """lscpu model, sockets and physical cores of the host, and the CPU share
    this process may use (the GPU machine grants 16 threads per GPU)."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = dict(l.split(":", 1) for l in txt.splitlines() if ":" in l)
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "1"))
        cps = int(kv.get("Core(s) per socket", "0"))
        info["sockets"] = sockets
        info["physical_cores"] = sockets * cps
        info["threads_per_core"] = int(kv.get("Thread(s) per core", "1"))
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except OSError:
        info["affinity_cpus"] = os.cpu_count()
    return info


def triad_gbs(threads, n=1 << 26, reps=5):
    """Host STREAM-style triad a = b + s c over 3 x 512 MiB FP64 arrays with
    torch's CPU kernels on `threads` threads (24 B per element)."""
    import torch
    old = torch.get_num_threads()
    torch.set_num_threads(threads)
    b = torch.rand(n, dtype=torch.float64)
    c = torch.rand(n, dtype=torch.float64)
    a = torch.empty_like(b)
    best = 1e30
    for _ in range(reps):
        t = time.perf_counter()
        torch.add(b, c, alpha=3.0, out=a)
        best = min(best, time.perf_counter() - t)
    torch.set_num_threads(old)
    del a, b, c
    return round(24.0 * n / best / 1e9, 1)


def cpu_baseline(steps, warmup, dt, c3_ref=None, single_steps=20):
    """The oracle (plain FP64 C + OpenMP, zero-start CG, as it stands) on the
    host: steps warmup+1 .. warmup+steps of the headline workload (the steps
    the GPU line times; the state at `warmup` comes from an untimed oracle
    run) on the process's CPU share, and the first `single_steps` of them on
    one thread; lscpu and a triad probe beside the numbers.  With c3_ref it
    also runs the oracle over the first steps of the 128^3 run and returns the
    per-step error of the GPU's FP64 and FP32-refined states against it."""
    import numpy as np
    import oracle
    import synth
    hi = host_info()
    share = max(1, min(hi.get("affinity_cpus") or 16, 16))
    O = oracle.Problem(synth.nonlinear(48))

    def timed(threads, n):
        oracle.set_threads(threads)
        A0, sc0 = None, None
        if warmup > 0:
            A0, sc0, *_ = O.run(dt, warmup, rtol=1e-8)
        t = time.time()
        O.run(dt, n, rtol=1e-8, A=A0, sc=sc0, m0=warmup)
        return time.time() - t, oracle.get_threads()

    el, used = timed(share, steps)
    el1, _ = timed(1, min(single_steps, steps))
    out = {"value": steps / el, "unit": "steps/s", "cores": used, "kind": "oracle",
           "sample": f"steps {warmup + 1}..{warmup + steps} of the 48^3 nonlinear run (the GPU "
                     f"line's timed steps), zero-start CG at rtol 1e-8, {el:.1f} s wall on "
                     f"{used} threads",
           "single_thread": {"value": min(single_steps, steps) / el1, "unit": "steps/s",
                             "cores": 1,
                             "sample": f"steps {warmup + 1}..{warmup + min(single_steps, steps)}"
                                       f", {el1:.1f} s wall"},
           "host": hi,
           "triad_GBs": {"threads_%d" % used: triad_gbs(used), "threads_1": triad_gbs(1)}}
    if c3_ref and c3_ref["traj"]:
        oracle.set_threads(share)
        wl = synth.nonlinear(c3_ref["N"])
        P = oracle.Problem(wl)
        n = min(len(v) for v in c3_ref["traj"].values())
        t = time.time()
        _, _, rec, its, itc = P.run(c3_ref["dt"], n, rtol=c3_ref["rtol"], rec_every=1)
        el3 = time.time() - t
        C, N = P.C, P.N

        def rel(a, b):
            return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        errs = {}
        for tag, tr in c3_ref["traj"].items():
            e = {"a_c": [], "B": [], "Kn_an": [], "a_n": [], "A": []}
            for m in range(n):
                g, o = tr[m], rec[m]
                e["a_c"].append(rel(g[C], o[C]))
                e["B"].append(rel(P.curl(g), P.curl(o)))
                e["Kn_an"].append(rel(P.kn(np.where(N, g, 0.0)), P.kn(np.where(N, o, 0.0))))
                e["a_n"].append(rel(g[N], o[N]))
                e["A"].append(rel(g, o))
            errs[tag] = {k: [float("%.3g" % x) for x in v] for k, v in e.items()}
        out["precision_128_vs_oracle"] = {
            "steps": n, "rtol": c3_ref["rtol"],
            "note": "relative 2-norm error per step against the FP64 oracle (zero-start CG at "
                    "the same rtol); a_n also holds a gauge (gradient) part that the "
                    "gauge-invariant a_c, B = C a and K_n a_n do not see",
            "errors": errs,
            "oracle_steps_per_s": round(n / el3, 4),
            "oracle_iters_per_step": float(np.mean(its + itc))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--methods", default="spe,cspe,pod,prev,zero")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps timed on the host (default: the GPU's timed steps, "
                         "at most 300)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 128^3 FP64 / FP32-refined runs")
    ap.add_argument("--c3-steps", type=int, default=200)
    ap.add_argument("--c3-warmup", type=int, default=20,
                    help="eager warm-up steps of the 128^3 runs (their own, not --warmup)")
    ap.add_argument("--c3-check-steps", type=int, default=8,
                    help="first steps of the 128^3 run compared with the FP64 oracle per step")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 64^3 adjoint runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch runs")
    ap.add_argument("--no-implicit", action="store_true",
                    help="skip the explicit-vs-implicit (Newton) comparison")
    ap.add_argument("--no-stability", action="store_true",
                    help="skip the stability estimate and consistent-mass runs")
    ap.add_argument("--budget-margin", type=int, default=None,
                    help="PCG iterations budgeted per captured solve beyond the warm-up median")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the dominant-kernel timing and a 512 MiB device copy "
                         "(the reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.budget_margin is not None:
        global BUDGET_MARGIN
        BUDGET_MARGIN = args.budget_margin
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    import synth
    import paper_1611_06721_amd as ec

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    rtol = 1e-8
    wl = synth.nonlinear(48)
    G = ec.Problem(wl, window_cap=20)
    if args.roofline_only:
        cg_us = time_cg_iteration(ec, torch, G)
        G128 = ec.Problem(synth.nonlinear(128), window_cap=1)
        cg128_us = time_cg_iteration(ec, torch, G128, reps=200)
        del G128
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=G.device)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"k_cg_iter<double>@48^3_us": round(cg_us, 3),
                          "k_cg_iter25<double,64>@128^3_us": round(cg128_us, 3),
                          "copy_bytes_each_way": COPY_BYTES}), flush=True)
        return
    lam = G.cfl(iters=60, rtol=1e-10)
    dt = 0.5 * 2.0 / lam
    log(f"[bench] 48^3 nonlinear: n_pad {G.n_pad}, lambda_max {lam:.6g}, dt {dt:.4g}")

    results = {}
    for name in args.methods.split(","):
        log(f"[bench] method {name}: warmup {args.warmup}, {args.steps} steps")
        r, _ = run_method(ec, torch, G, name, dt, args.steps, args.warmup, rtol,
                          cap=METHOD_BUDGET_CAP.get(name))
        results[name] = r
        log(f"[bench] {name}: {r['steps_per_s']:.1f} steps/s, {r['iters_per_step']:.2f} iters/step")
    head = "spe" if "spe" in results else next(iter(results))

    # dominant kernel: the PCG iteration (single-reduction Jacobi-PCG, FP64)
    N = 48
    n_alg = 3 * N * (N + 1) ** 2                 # padded edge elements (algorithmic unit)
    cg_us = time_cg_iteration(ec, torch, G)
    cg_bytes = 80.0 * n_alg
    achieved = cg_bytes / (cg_us * 1e-6) / 1e9
    traffic = traffic_record("k_cg_iter", "48^3")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic, "kernel": "k_cg_iter<double> (one PCG iteration)",
                "avg_us": round(cg_us, 3), "bytes_per_launch": cg_bytes}
    extra = {}
    G.close()
    del G
    torch.cuda.empty_cache()

    if not args.no_probe:
        os.makedirs(os.path.expanduser("~/.cache/paper_1611_06721_amd"), exist_ok=True)
        # HBM-resident sizes: the working set exceeds the 256 MB Infinity Cache
        # (the 2.5D kernel is the default on these grids)
        for Np in (128, 256):
            Gp = ec.Problem(synth.nonlinear(Np), window_cap=1)
            tuned = Gp.tune_pcg(os.path.expanduser("~/.cache/paper_1611_06721_amd/pcg_tiling.txt"))
            nn = 3 * Np * (Np + 1) ** 2
            us = time_cg_iteration(ec, torch, Gp, reps=60 if Np == 256 else 200)
            extra[f"cg_iter_{Np}"] = {"kernel": (f"k_cg_iter25<double,{tuned[0]}> (2.5D, LDS-staged, "
                                                 f"{tuned[1]} planes per block)" if tuned[0]
                                                 else "k_cg_iter<double> (node-parallel)"),
                                      "avg_us": round(us, 2),
                                      "achieved_GBs": round(80.0 * nn / (us * 1e-6) / 1e9, 1),
                                      "frac": round(80.0 * nn / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                                      "traffic": traffic_record("k_cg_iter25", f"{Np}^3")}
            Gp.close()
            del Gp
            torch.cuda.empty_cache()
            log(f"[bench] probe {Np}^3: cg iteration {us:.1f} us")

    c3, c3_ref = None, None
    if not args.no_c3:
        c3, c3_ref = precision_c3(ec, torch, args.c3_steps, args.c3_warmup, args.c3_check_steps)

    impl = None
    if not args.no_implicit:
        impl = implicit_vs_explicit(ec, torch, dt)
        log(f"[bench] implicit vs explicit 48^3: {impl['explicit']['seconds']} s explicit, "
            f"{impl['implicit']['seconds']} s implicit")
    stab = None
    if not args.no_stability:
        stab = stability_and_mass(ec, torch, dt)
        log(f"[bench] stability / consistent mass: {stab}")

    adj = None
    if not args.no_adjoint:
        adj = adjoint_c5(ec, torch)
        log(f"[bench] adjoint 64^3: forward {adj['forward_steps_per_s']} steps/s, backward "
            f"{adj['backward_steps_per_s']} steps/s, fd check {adj['fd_check']}")

    batch = None
    if not args.no_batch:
        batch = batch_c4(ec, torch)

    cpu = None
    if not args.no_cpu:
        cpu_steps = args.cpu_steps if args.cpu_steps else min(args.steps, 300)
        cpu = cpu_baseline(cpu_steps, args.warmup, dt, c3_ref)
        log(f"[bench] cpu oracle: {cpu['value']:.3f} steps/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.3f} on one")
        if c3 is not None and "precision_128_vs_oracle" in cpu:
            c3["vs_oracle"] = cpu.pop("precision_128_vs_oracle")

    r = results[head]
    line = {
        "metric": METRIC,
        "value": round(r["steps_per_s"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "nonlinear 48^3 FIT cube, Brauer iron 16^3, coil ramp 1000 "
                               "steps, dt = 0.5 x CFL bound, rtol 1e-8",
                   "timed_steps": f"m = {args.warmup + 1}..{args.warmup + args.steps} "
                                  f"(after {args.warmup} eager warm-up steps from rest)",
                   "start_vector": {"spe": "SPE window 8", "cspe": "SPE growing to 19 columns",
                                    "pod": "POD 20 snapshots <=10 modes",
                                    "prev": "previous solution", "zero": "zero"}[head],
                   "graph": True},
        "iters_per_step": round(r["iters_per_step"], 3),
        "spmv_hbm_gbs": round(achieved, 2),      # the SpMV is fused into the PCG kernel
        "methods": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in results.items()},
        "roofline": roofline,
        "probe": extra,
        "precision_128": c3,
        "implicit_vs_explicit_48": impl,
        "stability_and_consistent_mass_48": stab,
        "adjoint_64": adj,
        "batch_64": batch,
        "cpu_baseline": cpu,
    }
    if "zero" in results and head != "zero":
        line["speedup_vs_zero_start"] = round(r["steps_per_s"] / results["zero"]["steps_per_s"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
