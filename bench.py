"""Benchmark of the staggered space-time DG hot path on one MI355X.

Default workload (the largest configuration that the pressure metric is
quoted for): periodic unit cube, 48^3 hexahedra x 6 = 663,552 tetrahedra,
p = 3, p_gamma = 0 (20 DoF per element, 13,271,040 pressure DoF), nu = dt =
1e-3, velocity = 16 seeded divergence-free Fourier modes (amplitude |k|^-2,
normalised to max |v| = 1 over the nodes).  `--config c2` runs the
82,944-element p = 3, p_gamma = 1 cube instead, `--config c5` the
196,608-element p = 2, p_gamma = 1 cube.

A step is one Picard time step (Sec. 2.6, 2 Picard iterations, every row of
the hot path): averaging and Lambda, convection, viscous solve, goback,
Krylov initial guess, pressure-correction solve to a 1e-10 relative
residual, velocity update, inputs resident in HBM.  Before the timed steps
`--record` steps are recorded and the guess model is trained on them on the
GPU (reported, not timed).  The timed steps use the chosen form: pressure by
the time-decoupled CG with FP32 inner solves (block-Jacobi preconditioned) in
FP64 refinement, each solve started from the extrapolation of its own
history (the learned start, extrapolation plus a fitted network term, is
measured beside it and does not beat it here); viscous solve by block-Jacobi
preconditioned BiCGStab.

`value` is the Schur-operator throughput E N_st / t_apply of the chosen
inner operator (the FP32 spatial operator B (x) I on MFMA), t_apply the
median over `--applies` (>= 20) launches each timed by its own pair of HIP
events on the library's stream; the FP64 apply y = S x is timed the same way
and reported beside it.  The pressure-solve comparison runs one step from the
same saved state per form: plain (the paper's: FP64 CG from zero) against
chosen (FP32 refinement PCG, extrapolated guess), with ablations that change
one thing at a time (precision, preconditioner, initial guess, the learned
guess).

The roofline entry is for the step's dominant kernel, the one-kernel FP32 CG
iteration (k_lane_chunk<N> on meshes whose 64-element runs share a geometry
class, k_elem_iter<N, G> on meshes whose elements mostly carry their own
blocks, k_cg_op<N, true> otherwise), together with the one-block scalar
kernel k_cg_red that precedes each launch.  Its duration per iteration is the
library's own HIP-event measurement on its stream around the back-to-back
iteration launches of the timed steps (stdg_step_report.pressure_fused_iter_us).
Algorithmic bytes per iteration: read z, p, w, x and write them once (8 x 4 B
per DoF) plus 20 B of indices per element, plus, for k_elem_iter, the six
FP32 N x N blocks of every element (24 N^2 B per element).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

CONFIGS = {
    "c3": dict(n=48, p=3, pg=0, dt=1e-3, nu=1e-3, n_pic=2),
    "c2": dict(n=24, p=3, pg=1, dt=1e-3, nu=1e-3, n_pic=2),
    "c5": dict(n=32, p=2, pg=1, dt=1e-3, nu=1e-3, n_pic=2),
}
# HBM bytes per launch of k_lane_chunk<20> on the 663,552-element cube from
# rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
# for a device copy of known size; valid only for the kernel source they were
# measured on (sha256 prefix).  None until measured.
MEASURED_TRAFFIC = {"source": "paper_1601_07384_amd/csrc/cg_lane.hip", "sha256": "7a1a70f3332b4361",
                    "bytes": 530775654, "config": "c3"}
FP64_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", choices=sorted(CONFIGS), default="c3")
    ap.add_argument("--applies", type=int, default=50, help="timed launches per operator (>= 20)")
    ap.add_argument("--no-ablation", action="store_true", help="skip the plain-form and ablation steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=4096)
    ap.add_argument("--cpu-cores", type=int, default=0, help="oracle worker processes (0: min(16, host cores))")
    ap.add_argument("--record", type=int, default=12, help="steps recorded to train the learned guess")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--experiment", choices=["learned"], default=None,
                    help="learned: the held-out initial-guess experiment (record and train on the first "
                         "--train-steps steps, then compare the guesses on the next --eval-steps steps); "
                         "prints its own JSON line instead of the benchmark line")
    ap.add_argument("--train-steps", type=int, default=100)
    ap.add_argument("--eval-steps", type=int, default=100)
    ap.add_argument("--jitter", type=float, default=0.0,
                    help="move interior vertices by up to this fraction of h: every element then "
                         "has its own geometry class (operator blocks streamed per element)")
    a = ap.parse_args()
    a.applies = max(a.applies, 20)
    return a


def measured_traffic(cfg_name):
    import hashlib
    if MEASURED_TRAFFIC["sha256"] is None or cfg_name != MEASURED_TRAFFIC["config"]:
        return None
    with open(os.path.join(ROOT, MEASURED_TRAFFIC["source"]), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    return MEASURED_TRAFFIC["bytes"] if digest.startswith(MEASURED_TRAFFIC["sha256"]) else None


def workload_label(c, jitter):
    E = 6 * c["n"] ** 3
    N = (c["p"] + 1) * (c["p"] + 2) * (c["p"] + 3) // 6
    G = c["pg"] + 1
    s = (f"periodic unit cube, {c['n']}^3 hexahedra x 6 = {E:,} tets, p={c['p']}, p_gamma={c['pg']} "
         f"({N * G} DoF/tet, {E * N * G:,} pressure DoF), nu={c['nu']:g}, dt={c['dt']:g}, "
         f"{c['n_pic']} Picard iterations per step, 16 seeded Fourier modes")
    if jitter:
        s += f", interior vertices jittered by up to {jitter} h"
    return s


def _oracle_rows(args):
    """Worker: the oracle's operator rows `rows` (first call integrates their
    face matrices, then `calls` timed calls); returns the call times."""
    rows, calls = args
    ts = []
    apply_S(_ORACLE["ops"], _ORACLE["x"], elements=rows)
    for _ in range(calls):
        t0 = time.perf_counter()
        apply_S(_ORACLE["ops"], _ORACLE["x"], elements=rows)
        ts.append(time.perf_counter() - t0)
    return ts


_ORACLE = {}


def cpu_baseline(rows, X, T, c, cores):
    """The FP64 oracle's operator on a bounded sample of rows of the same
    mesh, split over `cores` forked worker processes of the host: each worker
    first integrates its rows' face matrices (not timed), then applies them
    five times; the rate is the sample's values over the median of the
    slowest worker's call times."""
    import multiprocessing as mp
    global apply_S
    from oracle.mesh import Mesh as OracleMesh
    from oracle.spacetime import SpaceTimeOperators
    from oracle.pressure import apply_S
    om = OracleMesh(X, T, periodic=True)
    ops = SpaceTimeOperators(om, c["p"], c["pg"], c["dt"])
    _ORACLE["ops"] = ops
    _ORACLE["x"] = np.random.default_rng(0).standard_normal((om.E, ops.Nst))
    sample = np.linspace(0, om.E - 1, rows).astype(np.int64)
    parts = [(part, 5) for part in np.array_split(sample, cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        times = pool.map(_oracle_rows, parts)
    wall = time.perf_counter() - t0
    t = float(np.median(np.max(np.array(times), axis=0)))
    return {"value": rows * ops.Nst / t / 1e9, "unit": "GDoF/s", "cores": cores, "kind": "oracle",
            "sample": f"{rows} evenly spaced rows of the {om.E:,}-element Schur operator (literal space-time "
                      f"matrices, extended-precision numpy), split over {cores} worker processes; each worker "
                      f"integrates its rows' face matrices once, then applies them 5 times; median over the "
                      f"calls of the slowest worker: {t:.3f} s per call ({wall:.1f} s in all)",
            "host_cores": os.cpu_count()}


def learned_guess_experiment(args, P, torch, m, c, vhat, vbar, p, hist, opts, label):
    """The learned initial guess on held-out steps.  Steps 1 .. T (T =
    --train-steps) of the trajectory are recorded (right-hand side and
    solution of each step's first pressure solve) and the model is trained on
    them on the GPU; each of the next --eval-steps steps is then run from the
    same state with the previous-step, the extrapolated and the learned start
    of its first pressure solve (the trajectory continues with the learned
    one), all with the chosen solver (FP32 refinement PCG to 1e-10)."""
    n = m.E * m.Nst
    T = args.train_steps
    Xr = torch.zeros(T * n, dtype=torch.float64, device="cuda:0")
    Br = torch.zeros(T * n, dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    for k in range(T):
        m.picard_step(vhat, vbar, p, None,
                      opts=opts(P.STDG_KRYLOV_EXTRAPOLATE, rec=(Br[k * n:(k + 1) * n], Xr[k * n:(k + 1) * n])))
    torch.cuda.synchronize()
    record_s = time.perf_counter() - t0
    progress(f"recorded {T} steps: {record_s:.1f} s")
    model = P.Model(m, hidden=128, precision=P.STDG_FP32, batch=m.E, lr=args.lr, seed=1601,
                    loss=P.STDG_LOSS_RESIDUAL)
    S = T - 2
    train = model.train(Xr[n:(T - 1) * n], Xr[:S * n], Br[2 * n:], Xr[2 * n:], epochs=args.epochs)
    del Xr, Br
    torch.cuda.empty_cache()
    progress(f"trained on {S} steps: {train.seconds:.1f} s, loss {train.first_loss:.3g} -> {train.last_loss:.3g}")
    guesses = [("previous", P.STDG_KRYLOV_PREVIOUS), ("extrapolated", P.STDG_KRYLOV_EXTRAPOLATE),
               ("learned", P.STDG_KRYLOV_LEARNED)]
    res = {g: {"first_iters": [], "first_s": [], "step_iters": [], "step_pressure_s": [], "r0": []}
           for g, _ in guesses}
    weights = []
    max_diff = 0.0
    for step in range(args.eval_steps):
        state = (vhat.clone(), vbar.clone(), p.clone(), hist.clone())
        out = {}
        for g, kg in guesses:
            vh, vb, pp, hh = (t.clone() for t in state)
            r = m.picard_step(vh, vb, pp, None, opts=opts(kg, model=model if g == "learned" else None, h=hh))
            torch.cuda.synchronize()
            d = res[g]
            d["first_iters"].append(r.first_pressure_iters)
            d["first_s"].append(r.first_pressure_seconds)
            d["step_iters"].append(r.pressure_iters)
            d["step_pressure_s"].append(r.pressure_seconds)
            d["r0"].append(r.first_initial_residual)
            if g == "learned":
                weights.append(r.guess_weight_network)
            out[g] = (vh, vb, pp, hh)
        pl = out["learned"][2]
        for g in ("previous", "extrapolated"):
            max_diff = max(max_diff, float((out[g][2] - pl).abs().max() / pl.abs().max()))
        vhat.copy_(out["learned"][0]); vbar.copy_(out["learned"][1]); p.copy_(pl); hist.copy_(out["learned"][3])
        del out, state
        if (step + 1) % 10 == 0:
            progress(f"held-out step {step + 1}: first-solve iterations " +
                     ", ".join(f"{g} {sum(res[g]['first_iters'])}" for g, _ in guesses))
    summary = {g: {"first_solve_iters": int(sum(d["first_iters"])), "first_solve_s": float(sum(d["first_s"])),
                   "step_pressure_iters": int(sum(d["step_iters"])),
                   "step_pressure_s": float(sum(d["step_pressure_s"])),
                   "mean_first_initial_rel_residual": float(np.mean(d["r0"]))} for g, d in res.items()}
    le, ex = summary["learned"]["first_solve_iters"], summary["extrapolated"]["first_solve_iters"]
    print(json.dumps({
        "metric": "first pressure-solve iterations and time to 1e-10 on held-out steps, by initial guess",
        "config": {"workload": label, "train_steps": T, "eval_steps": args.eval_steps, "epochs": args.epochs,
                   "lr": args.lr, "solver": "FP32-inner block-Jacobi PCG in FP64 refinement, rtol 1e-10"},
        "by_guess": summary,
        "learned_vs_extrapolated_first_iters": le / ex if ex else None,
        "network_beats_extrapolation": le < ex,
        "mean_network_weight": float(np.mean(weights)) if weights else None,
        "max_pressure_rel_diff_between_guesses": max_diff,
        "train": {"samples": train.samples, "seconds": train.seconds, "loss_first_epoch": train.first_loss,
                  "loss_last_epoch": train.last_loss, "record_s": record_s}}))


def progress(msg):
    """One line per finished phase on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1601_07384_amd as P
    from stdg_inputs import kuhn_mesh, node_coordinates, fourier_modes, fourier_velocity

    c = CONFIGS[args.config]
    X, T = kuhn_mesh(c["n"], jitter=args.jitter, seed=7)
    t0 = time.perf_counter()
    m = P.Mesh(X, T, c["p"], c["pg"], dt=c["dt"], nu=c["nu"], periodic=True)
    build_s = time.perf_counter() - t0
    progress(f"mesh built: {build_s:.1f} s ({m.E} elements, {m.n_classes} geometry classes)")
    perm = m.permutation()
    E, G, N, Nst = m.E, m.G, m.N, m.Nst
    run_layout = m.inner_layout == P.STDG_LAYOUT_RUN
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    # initial state: nodal Fourier field (constant over the slab), its dual projection
    modes = fourier_modes(seed=1601)
    xn = node_coordinates(X, T, c["p"])
    v = fourier_velocity(xn, modes)
    v /= np.sqrt((v * v).sum(-1)).max()
    vb = np.tile(np.transpose(v, (2, 0, 1))[:, perm, None, :], (1, 1, G, 1))    # [3][E][G][N]
    vbar = torch.tensor(np.ascontiguousarray(vb).ravel(), dtype=torch.float64, device=dev)
    del vb, v, xn
    vhat = torch.empty(3 * m.n_face * Nst, dtype=torch.float64, device=dev)
    m.dual_from_main(vbar, vhat)
    p = torch.zeros(E * Nst, dtype=torch.float64, device=dev)

    visc = {"method": P.STDG_BICGSTAB, "restart": 30, "rtol": 1e-10, "check_every": 1}
    press = {"method": P.STDG_CG_TIME, "precision": P.STDG_FP32, "rtol": 1e-10, "inner_rtol": 1e-5,
             "max_iter": 200000}
    n = E * Nst
    n_pic = c["n_pic"]
    hist = torch.zeros(2 * n_pic * n, dtype=torch.float64, device=dev)

    def opts(kg, model=None, h=None, rec=None, pressure=None):
        return P.step_opts(n_picard=n_pic, pressure=pressure or press, viscous=visc, krylov_guess=kg,
                           model=model, hist=hist if h is None else h,
                           rec_b=rec[0] if rec else None, rec_x=rec[1] if rec else None)

    if args.experiment == "learned":
        learned_guess_experiment(args, P, torch, m, c, vhat, vbar, p, hist, opts, workload_label(c, args.jitter))
        return

    # ---- trajectory for the learned guess: record the first pressure solve of
    # each step (right-hand side and solution), then train on the GPU
    t0 = time.perf_counter()
    Xr = torch.zeros(args.record * n, dtype=torch.float64, device=dev)
    Br = torch.zeros(args.record * n, dtype=torch.float64, device=dev)
    for k in range(args.record):
        m.picard_step(vhat, vbar, p, None,
                      opts=opts(P.STDG_KRYLOV_EXTRAPOLATE, rec=(Br[k * n:(k + 1) * n], Xr[k * n:(k + 1) * n])))
    torch.cuda.synchronize()
    record_s = time.perf_counter() - t0
    progress(f"recorded {args.record} steps: {record_s:.1f} s")
    model = P.Model(m, hidden=128, precision=P.STDG_FP32, batch=E, lr=args.lr, seed=1601,
                    loss=P.STDG_LOSS_RESIDUAL)
    S = args.record - 2
    train = model.train(Xr[n:(args.record - 1) * n], Xr[:S * n], Br[2 * n:], Xr[2 * n:], epochs=args.epochs)
    del Xr, Br
    torch.cuda.empty_cache()
    progress(f"guess model trained: {train.seconds:.1f} s")
    # the chosen start of each step's first solve is the extrapolation of the
    # solve's history: on this workload the trained network does not reduce
    # the iteration count below it (see the learned_guess entry of the line)
    chosen = opts(P.STDG_KRYLOV_EXTRAPOLATE)
    for _ in range(args.warmup):
        m.picard_step(vhat, vbar, p, None, opts=chosen)
    torch.cuda.synchronize()
    state = (vhat.clone(), vbar.clone(), p.clone(), hist.clone())
    reps = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        reps.append(m.picard_step(vhat, vbar, p, None, opts=chosen))
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t_start
    progress(f"timed steps: {t_steps / args.steps * 1e3:.1f} ms per step")

    # ---- operator launches, each timed by its own HIP events on the stream
    def median_launch_us(fn):
        for _ in range(5):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.applies)]
        torch.cuda.synchronize()
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs])) * 1e3

    x64 = torch.randn(n, dtype=torch.float64, device=dev)
    y64 = torch.empty_like(x64)
    fp64_us = median_launch_us(lambda: m.apply(x64, y64))
    op32 = None
    try:
        xf = torch.randn(m.inner_len, dtype=torch.float32, device=dev)
        yf = torch.empty_like(xf)
        op32 = median_launch_us(lambda: m.apply_spatial_f32(xf, yf))
        del xf, yf
    except P.StdgError:
        pass                         # no FP32 MFMA operator kernel for this degree
    del x64, y64
    dofs = E * Nst
    flops = 2.0 * N * N * G * 5 * E + 2.0 * N * G * G * E          # 5 N x N blocks x G columns + time mix
    inner_us = op32 if op32 is not None else fp64_us
    progress(f"operator launches: FP32 inner {op32} us, FP64 {fp64_us:.1f} us")

    # ---- pressure-solve comparison: one step per form from the saved state
    forms = {}
    err = None
    if not args.no_ablation:
        fp64_cg = {"method": P.STDG_CG_TIME, "precision": P.STDG_FP64, "rtol": 1e-10, "max_iter": 200000}
        fp32_cg = dict(press, precond=P.STDG_PRECOND_NONE)
        plan = [
            ("plain", "FP64 CG from zero (the paper's solve)", P.STDG_KRYLOV_ZERO, fp64_cg),
            ("fp64_extrapolated", "FP64 CG, extrapolated guess", P.STDG_KRYLOV_EXTRAPOLATE, fp64_cg),
            ("fp32_cg_extrapolated", "FP32-inner CG in FP64 refinement, no preconditioner, extrapolated guess",
             P.STDG_KRYLOV_EXTRAPOLATE, fp32_cg),
            ("fp32_pcg_zero", "chosen solver, zero guess", P.STDG_KRYLOV_ZERO, press),
            ("fp32_pcg_previous", "chosen solver, previous-step guess", P.STDG_KRYLOV_PREVIOUS, press),
            ("fp32_pcg_learned", "chosen solver, learned guess (extrapolation + fitted network term)",
             P.STDG_KRYLOV_LEARNED, press),
            ("chosen", "FP32-inner block-Jacobi PCG in FP64 refinement, extrapolated guess",
             P.STDG_KRYLOV_EXTRAPOLATE, press),
        ]
        out_state = {}
        for name, desc, kg, pr in plan:
            vh, vbb, pp, hh = (t.clone() for t in state)
            torch.cuda.synchronize()
            r = m.picard_step(vh, vbb, pp, None, opts=opts(kg, model=model, h=hh, pressure=pr))
            torch.cuda.synchronize()
            forms[name] = {"form": desc, "step_pressure_s": r.pressure_seconds,
                           "step_pressure_iters": r.pressure_iters,
                           "first_solve_s": r.first_pressure_seconds, "first_solve_iters": r.first_pressure_iters,
                           "first_initial_rel_residual": r.first_initial_residual,
                           "max_rel_residual": r.max_pressure_residual, "converged": r.status == P.STDG_OK}
            if kg == P.STDG_KRYLOV_LEARNED:
                forms[name]["network_weight"] = r.guess_weight_network
            if name in ("plain", "chosen"):
                out_state[name] = (vh, pp)
            else:
                del vh, pp
            del vbb, hh
            progress(f"form {name}: {r.pressure_seconds:.3f} s in the pressure solves")
        (vp, pp_), (vc, pc) = out_state["plain"], out_state["chosen"]
        err = {"vhat": float((vp - vc).abs().max() / vp.abs().max()),
               "p": float((pp_ - pc).abs().max() / pp_.abs().max())}
        del out_state, vp, pp_, vc, pc

    # one-kernel FP32 CG iteration (B (x) I): z, p, w, x read and written once
    it_us = sum(r.pressure_fused_iter_us * r.pressure_iters for r in reps) / max(
        sum(r.pressure_iters for r in reps if r.pressure_fused_iter_us > 0), 1)
    k_bytes = 8.0 * dofs * 4 + 20.0 * E + (24.0 * N * N * E if m.inner_per_element else 0.0)
    k_flops = 2.0 * N * N * 5 * E * G
    k_s = it_us * 1e-6 if it_us > 0 else float("nan")
    first = reps[0]
    out = {
        "metric": "Schur-op GDoF/s; pressure-solve time to 1e-10 rel residual, plain vs chosen",
        "value": dofs / (inner_us * 1e-6) / 1e9,
        "unit": "GDoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_steps / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 inner operator, f64 refinement", "data": "synthetic",
        "config": {"workload": workload_label(c, args.jitter), "pressure_dof": dofs,
                   "geometry_classes": m.n_classes},
        "operator": {"kernel": ((f"k_elem_op<{N},{G}> (FP32 B (x) I, per-element blocks)" if m.inner_per_element
                                 else f"{'k_lane_op' if run_layout else 'k_cg_op'}<{N}> (FP32 B (x) I on MFMA)")
                                if op32 is not None else "FP64 S x"), "median_us": inner_us,
                     "launches": args.applies,
                     "fp64_apply": {"median_us": fp64_us, "gdofs": dofs / fp64_us / 1e3,
                                    "tflops": flops / fp64_us / 1e6,
                                    "frac_fp64_peak": flops / fp64_us / 1e6 / FP64_PEAK_TFLOPS}},
        "step": {"pressure_s": first.pressure_seconds, "viscous_s": first.viscous_seconds,
                 "pressure_iters": first.pressure_iters, "viscous_iters": first.viscous_iters,
                 "max_pressure_residual": max(r.max_pressure_residual for r in reps),
                 "all_timed_steps_converged": all(r.status == P.STDG_OK for r in reps)},
        "pressure_solve_s": {
            "plain": forms.get("plain", {}).get("step_pressure_s"),
            "chosen": forms.get("chosen", {}).get("step_pressure_s"),
            "plain_form": "FP64 CG from zero, every pressure solve of one step",
            "chosen_form": "FP32-inner block-Jacobi PCG in FP64 refinement, extrapolated guess for the "
                           "first solve of the step",
            "chosen_vs_plain_rel_diff": err, "forms": forms},
        "roofline": {"bound": "hbm", "achieved": k_bytes / k_s / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": k_bytes / k_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.config) if args.jitter == 0 else None,
                     "kernel": (f"k_lane_chunk<{N}> + k_cg_red (one PCG iteration)" if run_layout
                                else (f"k_elem_iter<{N},{G}> + k_cg_red (one PCG iteration)" if m.inner_per_element
                                      else f"k_cg_op<{N},true> + k_cg_red (one PCG iteration)")), "kernel_us": it_us,
                     "kernel_launches": sum(r.pressure_iters for r in reps),
                     "bytes_per_launch": k_bytes, "flops_per_launch": k_flops,
                     "mfma_tflops": k_flops / k_s / 1e12,
                     "mfma_frac_fp32": k_flops / k_s / 1e12 / FP32_MFMA_PEAK_TFLOPS},
        "learned_guess": {"record_steps": args.record, "lr": args.lr, "record_s": record_s,
                          "train_samples": train.samples, "epochs": train.epochs, "train_s": train.seconds,
                          "loss_first_epoch": train.first_loss, "loss_last_epoch": train.last_loss,
                          "first_solve_iters_learned": forms.get("fp32_pcg_learned", {}).get("first_solve_iters"),
                          "first_solve_iters_extrapolated": forms.get("chosen", {}).get("first_solve_iters"),
                          "network_beats_extrapolation": (
                              forms["fp32_pcg_learned"]["first_solve_iters"] < forms["chosen"]["first_solve_iters"]
                              if "chosen" in forms else None)},
        "mesh_build_s": build_s,
    }
    if not args.no_cpu_baseline:
        progress("oracle sample on the host")
        cores = args.cpu_cores or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(args.cpu_rows, X, T, c, cores)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
