"""Benchmark of the staggered space-time DG hot path on one MI355X.

Workload: periodic unit cube, 24^3 hexahedra x 6 = 82,944 tetrahedra, p = 3,
p_gamma = 1 (40 space-time DoF per element, 3,317,760 pressure DoF),
nu = 1e-3, dt = 1e-3, velocity = 16 seeded divergence-free Fourier modes
(amplitude |k|^-2, normalised to max |v| = 1 over the nodes).

A step is one Picard time step (Sec. 2.6, p_gamma + 1 = 2 Picard iterations):
averaging and Lambda, convection, viscous solve, goback, learned initial
guess, pressure-correction solve to a 1e-10 relative residual, velocity
update -- every row of the hot path, inputs resident in HBM.  Before the
timed steps, `--record` steps are recorded and the guess model is trained on
them on the GPU (reported, not timed).  The timed steps use the chosen form
(pressure: time-decoupled CG with FP32 inner solves in FP64 refinement,
block-Jacobi preconditioned, learned guess for each step's first solve;
viscous: block-Jacobi preconditioned BiCGStab); extra steps from the same state
give the first solve's iterations from the zero, previous, extrapolated and
learned guesses, and one step in the plain form (FP64 GMRES(50) from zero, as
in the paper) gives the plain-vs-chosen pressure-solve comparison.

`value` is the whole-job Schur-operator throughput: pressure-operator
applications in the timed steps x DoF / timed wall time (GDoF/s).  The
roofline entry is for the step's dominant kernel, the one-kernel FP32 CG
iteration k_cg_op<N, true> (z = M^-1 r and p updates of the gathered rows,
q = (B (x) I) p on MFMA, w = M^-1 q, r = M z and x on the own rows, five
dot-product partials).  Its duration
is the library's own HIP-event measurement on its stream around the
back-to-back iteration launches of every inner solve of the timed steps
(stdg_step_report.pressure_fused_iter_us).  Algorithmic bytes per launch:
read z, p, w, x and write z, p, w, x once (8 x 4 B per DoF) plus 20 B of
indices per element; flops: 2 N^2 x 5 blocks per column.  The plain FP32
operator kernel (stdg_pressure_apply_spatial_f32) and the FP64 Schur apply
are timed with HIP events over bursts of launches (context).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_HEX, P_DEG, P_GAMMA, DT, NU = 24, 3, 1, 1e-3, 1e-3
# HBM bytes per launch of k_cg_op<20, true> from rocprofv3 FETCH_SIZE (x 2.0)
# and WRITE_SIZE (x 1.0), calibrated by a device copy of known size; valid
# only for the kernel source they were measured on (sha256 prefix).
MEASURED_TRAFFIC = {"source": "paper_1601_07384_amd/csrc/cg_fused.hip", "sha256": "fe6057e5558e2004",
                    "bytes": 117609.2 * 1024.0}
FP64_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--applies", type=int, default=200)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=256)
    ap.add_argument("--record", type=int, default=12, help="steps recorded to train the learned guess")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--jitter", type=float, default=0.0,
                    help="move interior vertices by up to this fraction of h: every element then "
                         "has its own geometry class (operator blocks streamed per element)")
    return ap.parse_args()


def measured_traffic():
    import hashlib
    path = os.path.join(ROOT, MEASURED_TRAFFIC["source"])
    with open(path, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    return MEASURED_TRAFFIC["bytes"] if digest.startswith(MEASURED_TRAFFIC["sha256"]) else None


def cpu_baseline(rows, X, T):
    """The FP64 oracle's literal operator on a bounded sample of rows."""
    from oracle.mesh import Mesh as OracleMesh
    from oracle.spacetime import SpaceTimeOperators
    from oracle.pressure import apply_S
    om = OracleMesh(X, T, periodic=True)
    ops = SpaceTimeOperators(om, P_DEG, P_GAMMA, DT)
    x = np.random.default_rng(0).standard_normal((om.E, ops.Nst))
    sample = np.linspace(0, om.E - 1, rows).astype(np.int64)
    t0 = time.perf_counter()
    apply_S(ops, x, elements=sample)
    t = time.perf_counter() - t0
    return {"value": rows * ops.Nst / t / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} rows of the 82,944-element Schur operator (literal space-time "
                      f"matrices integrated per face, extended precision), {t:.1f} s"}


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

    X, T = kuhn_mesh(N_HEX, jitter=args.jitter, seed=7)
    t0 = time.perf_counter()
    m = P.Mesh(X, T, P_DEG, P_GAMMA, dt=DT, nu=NU, periodic=True)
    build_s = time.perf_counter() - t0
    progress(f"mesh built: {build_s:.1f} s")
    perm = m.permutation()
    E, G, N, Nst = m.E, m.G, m.N, m.Nst
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    # initial state: nodal Fourier field (constant over the slab), its dual projection
    modes = fourier_modes(seed=1601)
    xn = node_coordinates(X, T, P_DEG)
    v = fourier_velocity(xn, modes)
    v /= np.sqrt((v * v).sum(-1)).max()
    vb = np.tile(np.transpose(v, (2, 0, 1))[:, perm, None, :], (1, 1, G, 1))    # [3][E][G][N]
    vbar = torch.tensor(np.ascontiguousarray(vb).ravel(), dtype=torch.float64, device=dev)
    vhat = torch.empty(3 * m.n_face * Nst, dtype=torch.float64, device=dev)
    m.dual_from_main(vbar, vhat)
    p = torch.zeros(E * Nst, dtype=torch.float64, device=dev)

    visc = {"method": P.STDG_BICGSTAB, "restart": 30, "rtol": 1e-10, "check_every": 1}
    press = {"method": P.STDG_CG_TIME, "precision": P.STDG_FP32, "rtol": 1e-10, "inner_rtol": 1e-5,
             "max_iter": 200000}
    n = E * Nst
    hist = torch.zeros(2 * G * n, dtype=torch.float64, device=dev)     # 2 steps x p_gamma + 1 solves

    def opts(kg, model=None, h=None, rec=None):
        return P.step_opts(pressure=press, viscous=visc, krylov_guess=kg, model=model,
                           hist=hist if h is None else h,
                           rec_b=rec[0] if rec else None, rec_x=rec[1] if rec else None)

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
    progress(f"guess model trained: {train.seconds:.1f} s")
    chosen = opts(P.STDG_KRYLOV_LEARNED, model=model)
    plain = P.step_opts(pressure={"method": P.STDG_GMRES, "restart": 50, "precision": P.STDG_FP64,
                                  "rtol": 1e-10, "max_iter": 200000},
                        viscous=visc)
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
    applies = sum(r.pressure_applies for r in reps)
    progress(f"timed steps: {t_steps / args.steps * 1e3:.1f} ms per step")

    # ---- the first pressure solve of the first timed step from each guess
    guess = {}
    for name, kg in (("zero", P.STDG_KRYLOV_ZERO), ("previous", P.STDG_KRYLOV_PREVIOUS),
                     ("extrapolated", P.STDG_KRYLOV_EXTRAPOLATE), ("learned", P.STDG_KRYLOV_LEARNED)):
        vh, vbb, pp, hh = (t.clone() for t in state)
        r = m.picard_step(vh, vbb, pp, None, opts=opts(kg, model=model, h=hh))
        guess[name] = {"iters": r.first_pressure_iters, "seconds": r.first_pressure_seconds,
                       "initial_rel_residual": r.first_initial_residual}
        guess[name]["step_pressure_iters"] = r.pressure_iters
        if kg == P.STDG_KRYLOV_LEARNED:
            guess[name]["network_weight"] = r.guess_weight_network
    torch.cuda.synchronize()

    progress("first solves by guess done")
    # ---- Schur-apply kernel burst (HIP events on the library's stream)
    x = p.clone()
    y = torch.empty_like(x)
    for _ in range(10):
        m.apply(x, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.applies):
        m.apply(x, y)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_apply = ev0.elapsed_time(ev1) / 1e3 / args.applies
    # ---- the fused FP32 CG operator kernel (same kernel, beta = 0) in a burst
    xf = torch.randn(E * Nst, dtype=torch.float32, device=dev)
    yf = torch.empty_like(xf)
    for _ in range(10):
        m.apply_spatial_f32(xf, yf)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.applies):
        m.apply_spatial_f32(xf, yf)
    ev1.record(stream)
    torch.cuda.synchronize()
    k_us = ev0.elapsed_time(ev1) * 1e3 / args.applies
    dofs = E * Nst
    flops = 2.0 * N * N * G * 5 * E + 2.0 * N * G * G * E          # 5 N x N blocks x G columns + time mix
    # x and y once, 5 int32 indices, the five N x N blocks of every geometry class once
    bytes_alg = 2.0 * dofs * 8 + 20.0 * E + 8.0 * 5 * N * N * m.n_classes
    # one-kernel FP32 CG iteration (B (x) I): r, p, q, x read and written once
    it_us = sum(r.pressure_fused_iter_us * r.pressure_iters for r in reps) / max(
        sum(r.pressure_iters for r in reps if r.pressure_fused_iter_us > 0), 1)
    # ... and the five blocks and the block-Jacobi inverse of every class once
    k_bytes = 8.0 * dofs * 4 + 20.0 * E + 4.0 * 6 * N * N * m.n_classes
    k_flops = 2.0 * N * N * 5 * E * G
    k_s = it_us * 1e-6 if it_us > 0 else float("nan")

    progress("kernel bursts done")
    # ---- plain form from the state before the timed steps
    plain_rep = None
    if not args.no_plain:
        vh, vbb, pp, _ = (t.clone() for t in state)
        plain_rep = m.picard_step(vh, vbb, pp, None, opts=plain)
        torch.cuda.synchronize()
        # compare with the first chosen step from the same state
        vh2, vbb2, pp2, hh2 = (t.clone() for t in state)
        m.picard_step(vh2, vbb2, pp2, None, opts=opts(P.STDG_KRYLOV_LEARNED, model=model, h=hh2))
        torch.cuda.synchronize()
        err_v = float((vh - vh2).abs().max() / vh.abs().max())
        err_p = float((pp - pp2).abs().max() / pp.abs().max())
        progress(f"plain FP64 GMRES step: {plain_rep.pressure_seconds:.1f} s in the pressure solve")

    first = reps[0]
    out = {
        "metric": "Schur-op GDoF/s; pressure-solve time to 1e-10 rel residual, plain vs chosen",
        "value": applies * dofs / t_steps / 1e9,
        "unit": "GDoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_steps / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "periodic unit cube, 24^3 hexahedra x 6 = 82,944 tets, p=3, "
                               "p_gamma=1 (40 DoF/tet), nu=1e-3, dt=1e-3, 2 Picard iterations "
                               "per step, 16 seeded Fourier modes"
                               + (f", interior vertices jittered by up to {args.jitter} h"
                                  if args.jitter else ""),
                   "pressure_dof": dofs, "geometry_classes": m.n_classes},
        "step": {"pressure_s": first.pressure_seconds, "viscous_s": first.viscous_seconds,
                 "pressure_iters": first.pressure_iters, "viscous_iters": first.viscous_iters,
                 "pressure_applies": first.pressure_applies,
                 "max_pressure_residual": first.max_pressure_residual,
                 "all_timed_steps_converged": all(r.status == P.STDG_OK for r in reps)},
        "pressure_solve_s": {
            "chosen": first.pressure_seconds,
            "chosen_form": "time-decoupled CG, block-Jacobi preconditioned, FP32 inner / FP64 "
                           "refinement, learned initial guess for the first solve of each step",
            "plain": plain_rep.pressure_seconds if plain_rep else None,
            "plain_form": "FP64 GMRES(50) on the space-time system",
            "plain_iters": plain_rep.pressure_iters if plain_rep else None,
            "chosen_vs_plain_rel_diff": {"vhat": err_v, "p": err_p} if plain_rep else None},
        "fp64_apply_kernel": {"kernel": "schur_apply_lds<20,2,double>", "us": t_apply * 1e6,
                              "gdofs": dofs / t_apply / 1e9, "tflops": flops / t_apply / 1e12,
                              "frac_fp64_peak": flops / t_apply / 1e12 / FP64_PEAK_TFLOPS,
                              "hbm_gbs_algorithmic": bytes_alg / t_apply / 1e9},
        "roofline": {"bound": "hbm", "achieved": k_bytes / k_s / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": k_bytes / k_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if N == 20 and args.jitter == 0 else None,
                     "kernel": f"k_cg_op<{N},true> (+ k_cg_red, one CG iteration)", "kernel_us": it_us,
                     "kernel_launches": sum(r.pressure_iters for r in reps),
                     "plain_operator_kernel": {"kernel": f"k_cg_op<{N},false>", "us": k_us,
                                               "launches": args.applies},
                     "bytes_per_launch": k_bytes, "flops_per_launch": k_flops,
                     "mfma_tflops": k_flops / k_s / 1e12,
                     "mfma_frac_fp32": k_flops / k_s / 1e12 / FP32_MFMA_PEAK_TFLOPS},
        "first_solve_by_guess": guess,
        "learned_guess": {"record_steps": args.record, "lr": args.lr, "record_s": record_s, "train_samples": train.samples,
                          "epochs": train.epochs, "train_s": train.seconds,
                          "loss_first_epoch": train.first_loss, "loss_last_epoch": train.last_loss},
        "mesh_build_s": build_s,
    }
    if not args.no_cpu_baseline:
        progress("oracle sample on the host")
        out["cpu_baseline"] = cpu_baseline(args.cpu_rows, X, T)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
