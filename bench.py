"""Benchmark: forward + adjoint evaluations of C -> B_z per second on one MI355X.

Workload: the 8x8 metasurface (64 square loops of 3 cm at 3.5 cm pitch, 32
segments each), B_z on 256x256 points at z = 1 cm (65,536 points), 21
frequencies 118..138 MHz, a batch of 4,096 capacitance configurations.  One
step is one cosim_loss_and_grad call over the whole batch: the forward solve of
every (configuration, frequency) system, B_z = G I with the loss epilogue, the
adjoint contraction G^T conj(w), the adjoint solve and the gradient reduction.
Inputs are resident in HBM before the timed region.  Before each mode is
timed, cosim_plan_autotune picks the fastest fused-kernel variant for it
(outside the timed region, like the one-time assembly).

The value is the mixed-precision throughput (matrix-core contraction in the
chosen mixed mode, FP64 solves); the FP64 mode is timed on the same GPU and
reported beside it.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2}
# the sources the fused kernel is compiled from (the traffic record names their hash)
FUSED_KERNEL_SRCS = [os.path.join(ROOT, "paper_2503_18479_amd", "csrc", f)
                     for f in ("fused.hip", "epilogue.h", "internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_traffic.json")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mixed", default="bf16x3", choices=["fp32", "bf16x3"],
                    help="mixed mode reported as the value")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--freqs", type=int, default=21)
    ap.add_argument("--two-planes", action="store_true",
                    help="131,072 points (z = 1 cm and 3 cm) instead of 65,536")
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="timed steps of the FP64 comparison (default: steps/2, >= 3)")
    ap.add_argument("--cpu-configs", type=int, default=24,
                    help="configurations the oracle evaluates for the CPU baseline (0: skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip cosim_plan_autotune (use the default kernel variants)")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="run only this many steps of the headline mode (for rocprofv3)")
    ap.add_argument("--ragged", type=int, default=2048,
                    help="also time this many independent instances of the ragged configuration "
                         "(16-256 loops, 16k-65k points, 1-8 frequencies; 2048 is the full set; 0: skip)")
    ap.add_argument("--large-adam", type=int, default=200,
                    help="the 32x32 array (1,024 loops, 262,144 points, batch 256): this many "
                         "Adam steps after the per-step timing (0: skip the line)")
    ap.add_argument("--sparam", type=int, default=3,
                    help="timed steps of the S-parameter pipeline on the 8x8 shape (0: skip)")
    ap.add_argument("--profile-sparam", type=int, default=None,
                    help="only the S-parameter line: this many steps per precision, for a profiler run")
    ap.add_argument("--profile-large", type=int, default=None,
                    help="only the 32x32 array: time this many steps per mode (no Adam, no "
                         "8x8 line), for a profiler run")
    ap.add_argument("--profile-assembly", type=int, default=None,
                    help="only the one-time assembly (G in every precision, M) of the 8x8 and 32x32 "
                         "arrays, this many times each, for a profiler run")
    ap.add_argument("--profile-ragged", type=int, default=None,
                    help="only the ragged line (eager steps and graph replays), this many steps "
                         "each, for a profiler run")
    ap.add_argument("--lines", default="single_loop,line_8x1,two_planes",
                    help="further workload lines (comma list of single_loop, line_8x1, "
                         "two_planes; empty: none)")
    ap.add_argument("--variant", type=int, default=None,
                    help="with --profile-steps: use this fused-kernel variant instead of tuning")
    return ap.parse_args()


def _src_hash(paths) -> str:
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def time_mode(plan, C, om, T, prec: str, steps: int, warmup: int, torch, tune: bool = True):
    tuned = None
    if tune:
        chosen, ms = plan.autotune(C, om, T, precision=PREC_CODE[prec], reps=2)
        tuned = {"variant": int(chosen), "variant_ms": [float(x) for x in ms]}
    loss = torch.empty((C.shape[0],), dtype=torch.float64, device=C.device)
    grad = torch.empty_like(C)
    st = torch.empty((C.shape[0], om.shape[0]), dtype=torch.int32, device=C.device)
    out = (loss, grad, st)
    for _ in range(warmup):
        plan.loss_and_grad(C, om, T, precision=PREC_CODE[prec], out=out)
    torch.cuda.synchronize()
    plan.timing(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.loss_and_grad(C, om, T, precision=PREC_CODE[prec], out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    phases = plan.timing_read()
    plan.timing(0)
    bad = int((st != 0).sum())
    time_mode.last = (loss.cpu().numpy(), grad.cpu().numpy())
    return dt, phases, bad, tuned


GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden(name: str) -> dict:
    """Stored FP64 oracle values (written by tests/golden/make_fullsize_golden.py)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def vs_oracle(loss, grad, ref: dict) -> dict:
    """Loss (relative) and dL/dC (normwise relative) of the stored
    configurations against the FP64 oracle's values."""
    cfg = ref["configs"]
    rl, rg = np.asarray(ref["loss"]), np.asarray(ref["grad"])
    el = np.abs(np.asarray(loss)[cfg] - rl) / np.abs(rl)
    eg = np.linalg.norm(np.asarray(grad)[cfg] - rg, axis=1) / np.linalg.norm(rg, axis=1)
    return {"configs": len(cfg), "loss_rel_max": float(el.max()),
            "grad_normwise_rel_max": float(eg.max())}


def cpu_baseline(wl, n_configs: int):
    """The FP64 oracle on the host cores, on a bounded sample of the workload."""
    import oracle as O
    try:
        import threadpoolctl
        threads = max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or 1
    except Exception:  # pragma: no cover
        threads = 1
    g = wl.geom
    t0 = time.perf_counter()
    G = O.field_matrix(g.verts, g.seg_off, wl.pts)
    M = (O.inductance_matrix_lattice(g.verts, g.seg_off, g.wire_a, g.nx, g.ny) if g.n > 1
         else O.inductance_matrix(g.verts, g.seg_off, g.wire_a))
    Phi = O.flux(g.verts, g.seg_off, wl.bext_z)
    t_asm = time.perf_counter() - t0
    C = wl.C[:n_configs]
    # repeated until at least 2 s have passed, so that small workloads are
    # timed over enough work
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.evaluate(G, M, g.R, Phi, C, wl.omega, wl.target)
        O.grad_adjoint(G, M, g.R, Phi, C, wl.omega, wl.target)
        reps += 1
        t_eval = time.perf_counter() - t0
        if t_eval >= 2.0:
            break
    one = None
    try:  # the same work on one core, for two configurations
        import threadpoolctl
        with threadpoolctl.threadpool_limits(1):
            t0 = time.perf_counter()
            O.evaluate(G, M, g.R, Phi, C[:2], wl.omega, wl.target)
            O.grad_adjoint(G, M, g.R, Phi, C[:2], wl.omega, wl.target)
            one = 2 / (time.perf_counter() - t0)
    except Exception:  # pragma: no cover
        pass
    return {
        "value": reps * n_configs / t_eval,
        "unit": "evals/s",
        "cores": int(threads),
        "kind": "oracle",
        "value_one_core": one,
        "sample": (f"{n_configs} configurations x {wl.F} frequencies at all {wl.P} points "
                   f"(loss + adjoint gradient, {reps} pass{'es' if reps > 1 else ''}, {t_eval:.1f} s); "
                   f"G/M assembly by the oracle "
                   f"took {t_asm:.1f} s and is excluded, as on the GPU"),
    }


def ragged_line(n_inst: int, mixed: str, steps: int, torch) -> dict:
    """Independent instances of the ragged configuration, one
    cosim_loss_and_grad_many call per step (plans keep only the mixed
    precision's copies of G)."""
    import workloads as W
    from paper_2503_18479_amd import Geometry, Plan, ManyCall
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wls = W.config4_instances(n_inst)
    plans, Cs, Os, Ts = [], [], [], []
    for wl in wls:
        pl = Plan(Geometry.from_workload(wl.geom), torch.tensor(wl.pts, device=dev), wl.bext_z,
                  precisions=[mixed])
        pl.reserve(wl.B, wl.F)
        plans.append(pl)
        Cs.append(torch.tensor(wl.C, device=dev))
        Os.append(torch.tensor(wl.omega, device=dev))
        Ts.append(torch.tensor(wl.target, device=dev))
    t_setup = time.perf_counter() - t0
    # the arguments of the 2,048 instances checked once (ManyCall); each step
    # enqueues the call again
    call = ManyCall(plans, Cs, Os, Ts, precision=PREC_CODE[mixed])
    outs = call.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # the same call captured once in a HIP graph and replayed
    from paper_2503_18479_amd import capture_loss_and_grad_many
    gr, gouts = capture_loss_and_grad_many(plans, Cs, Os, Ts, precision=PREC_CODE[mixed])
    gr.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gr.replay()
    torch.cuda.synchronize()
    dt_graph = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(outs, gouts))
    bad = sum(int((o[2] != 0).sum()) for o in outs)
    systems = sum(wl.B * wl.F for wl in wls)
    flops = sum(8.0 * wl.P * wl.geom.n * wl.B * wl.F for wl in wls)
    return {"instances": n_inst, "instance_evals_per_s": n_inst / dt, "ms_per_step": 1e3 * dt,
            "ms_per_step_graph": 1e3 * dt_graph, "graph_equals_eager": same,
            "steps": steps, "systems": systems, "contraction_tflops": flops / dt / 1e12,
            "loops": sorted(set(wl.geom.n for wl in wls)), "points_min": min(wl.P for wl in wls),
            "points_max": max(wl.P for wl in wls), "flagged_systems": bad,
            "setup_s": t_setup, "precision": mixed}


def sparam_line(steps: int, torch, batch: int = 4096) -> dict:
    """The S-parameter pipeline (cosim_sp_*) on the 8x8 shape: 64 ports, 65,536
    points, 21 frequencies, batch 4,096.  The exports stand in for full-wave
    data and come from the quasi-static model of the same array: S0 of the
    structure j w M, the field per unit incident wave of each port
    G (I - S0) / Z0.  The paper's one-port loads: the RC reflections (Eq. 2-3)
    are the variable entries, on the S_C11 diagonal; one drive port couples to
    every loop through a constant S_C12 (proportional to the loops' flux of a
    uniform field) and is fed with 1 W behind 50 ohm.  A step is
    cosim_sp_rc + cosim_sp_loss_and_grad + cosim_sp_rc_backward (C -> loss,
    dL/dC)."""
    import workloads as W
    from paper_2503_18479_amd import Geometry, Plan, SParamPlan, sp_rc, sp_rc_backward
    dev = torch.device("cuda:0")
    wl = W.config3_array8x8(batch=batch)
    g = wl.geom
    t0 = time.perf_counter()
    zp = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z,
              precisions=["fp64"])
    Gd = zp.G().to(torch.complex128)                          # [P][n]
    M, phi = zp.M(), zp.phi()
    del zp
    n, F, P, Z0 = g.n, wl.F, wl.P, 50.0
    om = torch.tensor(wl.omega, device=dev)
    S0h = np.empty((F, n, n), dtype=np.complex128)
    for f in range(F):
        Zs = 1j * wl.omega[f] * M
        S0h[f] = (Zs - Z0 * np.eye(n)) @ np.linalg.inv(Zs + Z0 * np.eye(n))
    S0 = torch.tensor(S0h, device=dev)
    fields = torch.empty((F, P, 1, n), dtype=torch.complex128, device=dev)
    for f in range(F):
        fields[f, :, 0, :] = Gd @ torch.tensor((np.eye(n) - S0h[f]) / Z0, device=dev)
    del Gd
    N = n + 1
    sch = np.zeros((F, N, N), dtype=np.complex128)
    kap = 0.5 * phi / np.linalg.norm(phi)
    sch[:, :n, n] = kap
    sch[:, n, :n] = kap
    scc = torch.tensor(sch, device=dev)
    ix = np.arange(n, dtype=np.int32)
    sp = SParamPlan(S0, fields, ix, ix, np.array([np.sqrt(Z0 * 1.0)]), sc_const=scc)
    del fields
    B = wl.B
    sp.reserve(B)
    C = torch.tensor(wl.C, device=dev)
    R = torch.tensor(g.R, device=dev)
    T = torch.tensor(wl.target, device=dev)
    vals = torch.empty((B, F, n), dtype=torch.complex128, device=dev)
    loss = torch.empty((B,), dtype=torch.float64, device=dev)
    gv = torch.empty((B, F, n), dtype=torch.complex128, device=dev)
    st = torch.empty((B, F), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    out = {"workload": wl.name, "ports": n, "points": P, "freqs": F, "batch": B,
           "systems": B * F, "setup_s": t_setup, "modes": {}}
    # complex contractions: 8 real flops per complex multiply-add, forward and adjoint
    flops = 2 * 8.0 * P * n * B * F
    for prec in ("fp32", "fp64"):
        def step():
            sp_rc(R, C, om, Z0, out=vals)
            sp.loss_and_grad(vals, T, 0, 0, prec, out=(loss, gv, st))
            return sp_rc_backward(R, C, om, gv, Z0)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            gC = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out["modes"][prec] = {"ms_per_step": 1e3 * dt, "evals_per_s": B / dt, "steps": steps,
                              "contraction_tflops_step_bound": flops / dt / 1e12,
                              "flagged_systems": int((st != 0).sum()),
                              "finite_grad": bool(torch.isfinite(gC).all())}
        print(f"[bench] S-parameter pipeline {prec}: {1e3 * dt:.1f} ms per step", file=sys.stderr,
              flush=True)
    out["flops_per_step"] = flops
    out["fp32_vs_fp64"] = out["modes"]["fp64"]["ms_per_step"] / out["modes"]["fp32"]["ms_per_step"]
    return out


def workload_line(wl, ref: dict, mixed: str, steps: int, warmup: int, cpu_configs: int,
                  torch) -> dict:
    """One workload of the path at its own shape: cosim_loss_and_grad per step
    in the mixed precision and in FP64 (evaluations per second, phases), the
    fused contraction's fraction of its precision's matrix-core peak, the
    error against stored oracle values, and the oracle's own time on a sample
    of the same workload."""
    from paper_2503_18479_amd import Geometry, Plan
    dev = torch.device("cuda:0")
    g = wl.geom
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z,
                precisions=[mixed, "fp64"])
    C = torch.tensor(wl.C, device=dev)
    om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    plan.reserve(wl.B, wl.F)
    S = wl.B * wl.F
    flops = 8.0 * wl.P * g.n * S
    out = {"workload": wl.name, "loops": g.n, "points": wl.P, "freqs": wl.F, "batch": wl.B,
           "systems": S, "modes": {}}
    for m in (mixed, "fp64"):
        dt, ph, bad, tuned = time_mode(plan, C, om, T, m, steps, warmup, torch)
        fused = float(np.mean(ph[:, 1]))
        ach = flops / (fused * 1e-3) / 1e12
        out["modes"][m] = {
            "evals_per_s": wl.B * steps / dt, "ms_per_step": 1e3 * dt / steps, "steps": steps,
            "phase_ms": {name: float(np.mean(ph[:, i])) for i, name in enumerate(Plan.PHASES)},
            "flagged_systems": bad, "variant": (tuned or {}).get("variant"),
            "roofline": {"bound": "mfma", "kernel": "fused contraction", "achieved": ach,
                         "peak": PEAK_TFLOPS[m], "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[m],
                         "flops_per_launch": flops, "avg_launch_ms": fused},
            "vs_oracle": vs_oracle(*time_mode.last, ref)}
        print(f"[bench] {wl.name} {m}: {out['modes'][m]['evals_per_s']:.0f} evals/s, "
              f"{out['modes'][m]['ms_per_step']:.3f} ms/step, vs oracle "
              f"{out['modes'][m]['vs_oracle']}", file=sys.stderr, flush=True)
    out["mixed_vs_fp64"] = out["modes"][mixed]["evals_per_s"] / out["modes"]["fp64"]["evals_per_s"]
    del plan
    if cpu_configs > 0:
        out["cpu_baseline"] = cpu_baseline(wl, min(cpu_configs, wl.B))
    return out


def reference_copy(torch, dev):
    """A device copy of known size (256 MiB read + 256 MiB written) that
    calibrates the HBM byte counters of a profiler run."""
    x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
    x.fill_(1.0)
    y = x.clone()
    torch.cuda.synchronize()
    del x, y


def large_line(adam_steps: int, mixed: str, steps: int, torch) -> dict:
    """The 32x32 array (1,024 loops, 512x512 points at z = 2 cm, batch 256,
    one frequency): per-step time and phases of cosim_loss_and_grad in the
    mixed precision and in FP64, the mixed-precision loss and gradient against
    FP64 at the same C, and `adam_steps` Adam steps (eager launches) from the
    seeded C in the mixed precision."""
    import workloads as W
    from paper_2503_18479_amd import Geometry, Plan
    dev = torch.device("cuda:0")
    wl = W.config5_array32x32()
    t0 = time.perf_counter()
    plan = Plan(Geometry.from_workload(wl.geom), torch.tensor(wl.pts, device=dev), wl.bext_z,
                precisions=["fp64", mixed])
    C = torch.tensor(wl.C, device=dev)
    om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    plan.reserve(wl.B, wl.F)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    n, S = wl.geom.n, wl.B * wl.F
    modes, vals = {}, {}

    def rel_err(a, b):
        (la, ga), (lb, gb) = a, b
        return {"loss_rel_max": float(np.max(np.abs(la - lb) / np.abs(lb))),
                "grad_normwise_rel_max": float(np.max(np.linalg.norm(ga - gb, axis=1)
                                                      / np.linalg.norm(gb, axis=1)))}

    # FP64 factor first, then the FP32 factor with FP64 refinement
    for refined in (False, True):
        plan.set_refinement(refined)
        plan.reserve(wl.B, wl.F)
        for m in (mixed, "fp64"):
            key = m + ("+refined" if refined else "")
            dt, ph, bad, _ = time_mode(plan, C, om, T, m, steps, 1, torch, tune=False)
            loss, grad, _ = plan.loss_and_grad(C, om, T, precision=PREC_CODE[m])
            vals[key] = (loss.cpu().numpy(), grad.cpu().numpy())
            pm = {name: float(np.mean(ph[:, i])) for i, name in enumerate(Plan.PHASES)}
            # complex-symmetric LDL^T: (4/3) n^3 real flops per system (the
            # solve_forward phase also holds the assembly and forward solve);
            # the contraction phase: 8 P n flops per system (forward and
            # adjoint, real-split)
            ldl_tf = S * 4.0 / 3.0 * n ** 3 / (pm["solve_forward"] * 1e-3) / 1e12
            modes[key] = {"ms_per_step": 1e3 * dt / steps, "evals_per_s": wl.B * steps / dt,
                          "steps": steps, "phase_ms": pm, "flagged_systems": bad,
                          "solve_forward_ldl_tflops": ldl_tf,
                          "contraction_tflops": 8.0 * wl.P * n * S
                          / (pm["fused_contraction"] * 1e-3) / 1e12}
            if refined:
                modes[key]["vs_fp64_factor"] = rel_err(vals[key], vals[m])
            print(f"[bench] 32x32 {key}: {modes[key]['ms_per_step']:.1f} ms/step, phases {pm}",
                  file=sys.stderr, flush=True)
    plan.set_refinement(False)
    err = rel_err(vals[mixed], vals["fp64"])
    ref = golden("array_32x32_full.json")
    oracle_err = {key: vs_oracle(v[0], v[1], ref) for key, v in vals.items()}
    adam = None
    if adam_steps > 0:
        C1 = C.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, st = plan.optimize(C1, om, T, adam_steps, precision=PREC_CODE[mixed])
        torch.cuda.synchronize()
        t_adam = time.perf_counter() - t0
        h = hist.cpu().numpy()
        adam = {"steps": adam_steps, "s": t_adam, "ms_per_step": 1e3 * t_adam / adam_steps,
                "loss_first_mean": float(h[0].mean()), "loss_last_mean": float(h[-1].mean()),
                "flagged_systems": int((st != 0).sum()), "precision": mixed, "lr": 1e-13}
        print(f"[bench] 32x32 Adam: {adam_steps} steps in {t_adam:.1f} s, mean loss "
              f"{adam['loss_first_mean']:.4e} -> {adam['loss_last_mean']:.4e}", file=sys.stderr,
              flush=True)
    return {"workload": wl.name, "loops": n, "points": wl.P, "batch": wl.B, "freqs": wl.F,
            "setup_s": t_setup, "modes": modes, "mixed_vs_fp64_error": err,
            "vs_oracle": oracle_err,
            "mixed_vs_fp64_speed": modes["fp64"]["ms_per_step"] / modes[mixed]["ms_per_step"],
            "refined_speedup": {m: modes[m]["ms_per_step"] / modes[m + "+refined"]["ms_per_step"]
                                for m in (mixed, "fp64")},
            "adam": adam,
            "solve": "blocked complex-symmetric LDL^T, FP64 matrix cores; '+refined': complex64 "
                     "factor on FP32 matrix cores with FP64 iterative refinement"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the batch shards over configurations; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2503_18479_amd import Geometry, Plan

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.profile_sparam is not None:
        out = sparam_line(args.profile_sparam, torch)
        reference_copy(torch, dev)
        print(f"[bench] profiled the S-parameter pipeline: {out['modes']}", file=sys.stderr, flush=True)
        return
    if args.profile_ragged is not None:
        out = ragged_line(args.ragged, args.mixed, args.profile_ragged, torch)
        print(f"[bench] profiled the ragged line: {out['ms_per_step']:.1f} ms eager, "
              f"{out['ms_per_step_graph']:.1f} ms graph", file=sys.stderr, flush=True)
        return
    if args.profile_assembly is not None:
        for wl in (W.config3_array8x8(batch=1), W.config5_array32x32(batch=1)):
            geom = Geometry.from_workload(wl.geom)
            pts = torch.tensor(wl.pts, device=dev)
            for _ in range(args.profile_assembly):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Plan(geom, pts, wl.bext_z, precisions=["fp64", "fp32", "bf16x3"])
                torch.cuda.synchronize()
                print(f"[bench] assembled {wl.summary()} in {time.perf_counter() - t0:.3f} s",
                      file=sys.stderr, flush=True)
        reference_copy(torch, dev)
        print("[bench] profiled the assembly and a 256 MiB copy", file=sys.stderr, flush=True)
        return
    if args.profile_large is not None:
        out = large_line(0, args.mixed, args.profile_large, torch)
        reference_copy(torch, dev)
        print(f"[bench] profiled the 32x32 array: {out['modes']}", file=sys.stderr, flush=True)
        return
    wl = W.config3_array8x8(batch=args.batch, grid=args.grid, two_planes=args.two_planes,
                            n_freq=args.freqs)
    g = wl.geom
    t0 = time.perf_counter()
    plan = Plan(Geometry.from_workload(g), torch.tensor(wl.pts, device=dev), wl.bext_z)
    t_asm = time.perf_counter() - t0
    C = torch.tensor(wl.C, device=dev)
    om = torch.tensor(wl.omega, device=dev)
    T = torch.tensor(wl.target, device=dev)
    plan.reserve(wl.B, wl.F)
    print(f"[bench] assembled {wl.summary()} in {t_asm:.2f} s", file=sys.stderr, flush=True)

    if args.profile_steps is not None:
        if args.variant is not None:
            plan.set_variant(PREC_CODE[args.mixed], args.variant)
        time_mode(plan, C, om, T, args.mixed, args.profile_steps, 1, torch,
                  tune=not args.no_autotune and args.variant is None)
        reference_copy(torch, dev)
        print(f"[bench] profiled {args.profile_steps} steps of {args.mixed} and a 256 MiB copy",
              file=sys.stderr)
        return

    S = wl.B * wl.F
    flops = 8.0 * wl.P * g.n * S  # forward 4 P n S + adjoint 4 P n S (real-split)
    res = {}
    modes = [args.mixed, "fp64"]
    other = "fp32" if args.mixed == "bf16x3" else "bf16x3"
    modes.append(other)
    for m in modes:
        steps = args.steps if m != "fp64" else (args.fp64_steps or max(3, args.steps // 2))
        dt, ph, bad, tuned = time_mode(plan, C, om, T, m, steps, args.warmup, torch,
                                       tune=not args.no_autotune)
        fused = float(np.mean(ph[:, 1]))
        res[m] = {
            "evals_per_s": wl.B * steps / dt,
            "ms_per_step": 1e3 * dt / steps,
            "steps": steps,
            "phase_ms": {name: float(np.mean(ph[:, i])) for i, name in enumerate(Plan.PHASES)},
            "fused_tflops": flops / (fused * 1e-3) / 1e12,
            "flagged_systems": bad,
            "autotune": tuned,
        }
        if wl.B == 4096 and wl.F == 21 and wl.P == 65536:
            res[m]["vs_oracle"] = vs_oracle(*time_mode.last, golden("array_8x8_full.json"))
        print(f"[bench] {m}: {res[m]['evals_per_s']:.0f} evals/s, {res[m]['ms_per_step']:.2f} ms/step, "
              f"phases {res[m]['phase_ms']}", file=sys.stderr, flush=True)

    head = res[args.mixed]
    fused_ms = head["phase_ms"]["fused_contraction"]
    achieved = head["fused_tflops"]
    traffic = None
    tuned_variant = (head["autotune"] or {}).get("variant", 0)
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if (tr.get("kernel_src_sha256_16") == _src_hash(FUSED_KERNEL_SRCS)
                and tr.get("precision") == args.mixed and tr.get("workload") == wl.name
                and tr.get("batch") == wl.B and tr.get("points") == wl.P):
            traffic = (tr.get("variants") or {}).get(str(tuned_variant), {}).get("bytes_per_launch")
    # FP64 solve phases: LDL^T (4/3 n^3 real flops) + one substitution pair
    # (8 n^2) per system in the forward phase, one substitution pair in the
    # adjoint phase; the factor record is n(n-1)/2 complex per system.
    n = g.n
    rec_bytes = S * n * (n - 1) / 2 * 16.0
    phases = {}
    for name, flops_ps, byts in (("solve_forward", 4.0 / 3.0 * n ** 3 + 8.0 * n * n, 2 * rec_bytes),
                                 ("solve_adjoint", 8.0 * n * n, rec_bytes)):
        ms = head["phase_ms"][name]
        tf = S * flops_ps / (ms * 1e-3) / 1e12
        gbs = byts / (ms * 1e-3) / 1e9
        phases[name] = {"ms": ms, "fp64_tflops": tf, "fp64_frac": tf / PEAK_TFLOPS["fp64"],
                        "record_gbs": gbs, "hbm_frac": gbs / 8000.0}

    line = {
        "metric": "fwd+adjoint C->B_z evals/sec, 8x8 array, 65k pts: mixed vs FP64, same GPU",
        "value": head["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.mixed}+f64",
        "data": "synthetic",
        "config": {
            "workload": wl.name, "loops": g.n, "segments_per_loop": 32, "points": wl.P,
            "freqs": wl.F, "batch": wl.B, "systems": S, "precision": args.mixed,
            "solve": "fp64 LDL^T (pivoted fallback)", "loss": "magnitude MSE",
        },
        "fp64": {"value": res["fp64"]["evals_per_s"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "steps": res["fp64"]["steps"]},
        "mixed_vs_fp64": head["evals_per_s"] / res["fp64"]["evals_per_s"],
        "modes": res,
        "roofline": {
            "bound": "mfma",
            "kernel": "fused contraction (B = G I, loss epilogue, G^T conj(w))",
            "achieved": achieved,
            "peak": PEAK_TFLOPS[args.mixed],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[args.mixed],
            "traffic": traffic,
            "flops_per_launch": flops,
            "avg_launch_ms": fused_ms,
            "variant": tuned_variant,
            "phases": phases,
        },
    }
    # gradients with respect to R, L and w on the same batch (mixed precision)
    plan.loss_and_grad_params(C, om, T, precision=PREC_CODE[args.mixed])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out_p = plan.loss_and_grad_params(C, om, T, precision=PREC_CODE[args.mixed])
    torch.cuda.synchronize()
    dtp = (time.perf_counter() - t0) / args.steps
    line["params"] = {"ms_per_step": 1e3 * dtp, "steps": args.steps,
                      "overhead_vs_loss_and_grad": dtp * 1e3 / head["ms_per_step"] - 1.0,
                      "outputs": "loss, dL/dC, dL/dR, dL/dL (series inductance), dL/dw",
                      "finite": bool(all(torch.isfinite(t).all() for t in out_p[:5]))}
    print(f"[bench] with R, L, w gradients: {1e3 * dtp:.2f} ms/step", file=sys.stderr, flush=True)
    del plan
    torch.cuda.empty_cache()
    wanted = [x for x in args.lines.split(",") if x]
    line["lines"] = {}
    for name in wanted:
        print(f"[bench] workload line {name}", file=sys.stderr, flush=True)
        if name == "single_loop":
            wl1 = W.config1_single_loop(batch=64, grid=32)
            ref = golden("single_loop_full.json")
        elif name == "line_8x1":
            wl1 = W.config2_line8(batch=1024, grid=64)
            ref = golden("line_8x1_full.json")
        elif name == "two_planes":
            wl1 = W.config3_array8x8(batch=4096, two_planes=True)
            ref = golden("array_8x8_full.json")["two_planes"]
        else:
            raise SystemExit(f"unknown line {name}")
        # the oracle's time beside each line; the two-plane array is the
        # headline's array with twice the points (its oracle G alone takes
        # minutes on the host), so its oracle time is the headline's
        cpu = {"single_loop": 64, "line_8x1": 1024, "two_planes": 0}[name]
        line["lines"][name] = workload_line(wl1, ref, args.mixed, args.steps, args.warmup,
                                            cpu if args.cpu_configs > 0 else 0, torch)
        torch.cuda.empty_cache()
    if args.ragged > 0:
        print(f"[bench] ragged configuration: {args.ragged} instances", file=sys.stderr, flush=True)
        line["ragged"] = ragged_line(args.ragged, args.mixed, 3, torch)
        print(f"[bench] ragged: {line['ragged']['ms_per_step']:.1f} ms per step, "
              f"{line['ragged']['ms_per_step_graph']:.1f} ms replayed from a graph", file=sys.stderr,
              flush=True)
    if args.large_adam > 0:
        print("[bench] 32x32 array", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        line["large"] = large_line(args.large_adam, args.mixed, 3, torch)
    if args.sparam > 0:
        print("[bench] S-parameter pipeline", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        line["sparam"] = sparam_line(args.sparam, torch)
    if args.cpu_configs > 0:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_configs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
