"""Benchmark of the pressure Schur path on one MI355X.

Workload: 24^3 hexahedra x 6 = 82,944 tetrahedra of the periodic unit cube,
p = 3, p_gamma = 1 (40 space-time DoF per element, 3,317,760 pressure DoF),
dt = 1e-3 (the larger plain-FP64 configuration: GMRES(50) to 1e-10).

A step is one pressure solve to a 1e-10 relative residual, plain FP64 GMRES(50)
from a zero guess, on the right-hand side produced by a smooth seeded
pressure field; every step also times the FP32-inner / FP64-refinement form.
`value` is the Schur-operator throughput E*G*N / t_apply (GDoF/s) from HIP
events around the operator kernel on the stream it runs on.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_HEX, P_DEG, P_GAMMA, DT = 24, 3, 1, 1e-3
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--applies", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=256)
    return ap.parse_args()


def smooth_pressure(xn):
    """A smooth periodic scalar field from the seeded Fourier modes."""
    from stdg_inputs import fourier_modes
    k, e, phi = fourier_modes(seed=1601)
    arg = 2 * np.pi * np.tensordot(xn, k.T, axes=1) + phi
    return np.cos(arg) @ (1.0 / np.sum(k * k, axis=1))


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
    return {"value": rows * ops.Nst / t / 1e9, "unit": "GDoF/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{rows} rows of the 82,944-element operator (literal space-time "
                      f"matrices built per face), {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          "--gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1601_07384_amd as P
    from stdg_inputs import kuhn_mesh, node_coordinates

    X, T = kuhn_mesh(N_HEX)
    t0 = time.perf_counter()
    m = P.Mesh(X, T, P_DEG, P_GAMMA, dt=DT, periodic=True)
    build_s = time.perf_counter() - t0
    perm = m.permutation()
    E, G, N, Nst = m.E, m.G, m.N, m.Nst
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    q = smooth_pressure(node_coordinates(X, T, P_DEG))       # (E, N)
    xq = torch.tensor(np.tile(q, (1, G))[perm].ravel(), dtype=torch.float64, device=dev)
    b = torch.empty_like(xq)
    m.apply(xq, b)
    x = torch.zeros_like(b)

    # ---- operator throughput (HIP events on the library's stream)
    y = torch.empty_like(b)
    for _ in range(10):
        m.apply(xq, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.applies):
        m.apply(xq, y)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_apply = ev0.elapsed_time(ev1) / 1e3 / args.applies
    dofs = E * Nst
    flops = 2.0 * N * N * G * 5 * E + 2.0 * N * G * G * E
    bytes_alg = 2.0 * dofs * 8 + 20.0 * E

    # ---- timed steps: plain FP64 GMRES(50) solve to 1e-10
    opts_plain = P.solve_opts(method=P.STDG_GMRES, restart=50, rtol=1e-10, precision=P.STDG_FP64)
    opts_ir = P.solve_opts(method=P.STDG_GMRES, restart=50, rtol=1e-10, precision=P.STDG_FP32,
                           inner_rtol=1e-4)
    for _ in range(args.warmup):
        x.zero_()
        m.solve(b, x, opts=opts_plain)
    torch.cuda.synchronize()
    reps = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        reps.append(m.solve(b, x, opts=opts_plain))
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t_start
    x_plain = x.clone()
    ir_reps = []
    t_ir0 = time.perf_counter()
    for _ in range(max(1, args.steps)):
        x.zero_()
        ir_reps.append(m.solve(b, x, opts=opts_ir))
    torch.cuda.synchronize()
    t_ir = (time.perf_counter() - t_ir0) / max(1, args.steps)
    err_ir = float((x - x_plain).abs().max() / x_plain.abs().max())

    out = {
        "metric": "Schur-op GDoF/s; pressure-solve time to 1e-10 rel residual, plain vs chosen",
        "value": dofs / t_apply / 1e9,
        "unit": "GDoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_steps / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "periodic unit cube, 24^3 hexahedra x 6 = 82,944 tets, "
                               "p=3, p_gamma=1 (40 DoF/tet), dt=1e-3, GMRES(50) to 1e-10",
                   "pressure_dof": dofs},
        "apply_us": t_apply * 1e6,
        "solve_plain": {"seconds": t_steps / args.steps, "iters": reps[-1].inner_iters,
                        "rel_residual": reps[-1].rel_residual},
        "solve_chosen": {"form": "FP32 inner GMRES(50) in FP64 refinement",
                         "seconds": t_ir, "outer": ir_reps[-1].outer_iters,
                         "inner_iters": ir_reps[-1].inner_iters,
                         "rel_residual": ir_reps[-1].rel_residual,
                         "max_rel_diff_vs_plain": err_ir},
        "roofline": {"bound": "alu", "achieved": flops / t_apply / 1e12, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / t_apply / 1e12 / FP64_PEAK_TFLOPS,
                     "traffic": None, "kernel": "schur_apply_rows<2,double>",
                     "hbm_gbs_algorithmic": bytes_alg / t_apply / 1e9},
        "mesh_build_s": build_s,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_rows, X, T)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
