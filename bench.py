#!/usr/bin/env python
"""Throughput of the gradient-enhanced damage hot path on one MI355X.

Workload: the 64x64x64 Hex8 unit cube (262 144 elements, 2 097 152
quadrature points, 1 098 500 dofs, 115 024 912 CSR entries) with the
3 -> 64 -> 64 -> 64 -> 1 energy network and the 1 -> 16 -> 1 yield network,
seeded heterogeneous stretch field, phi ~ U(0, 0.2), kappa ~ U(0, 0.1).
A step is one FP64 residual + consistent-tangent assembly: quadrature inputs,
energy-network jets, history update, element integration and coloured CSR
scatter.  The metric is quadrature-point residual+tangent evaluations per
second with every input resident in HBM.

Also reported: the mixed-precision (BF16 matrix-core) assembly of the same
workload when available, the per-phase split measured with HIP events on the
library's stream, the roofline of the dominant kernel, and the FP64 oracle
timed on the host cores over a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0


def jet_flops_per_qp(width, n_hidden, with_hessian=True):
    """Matrix-core flops of the energy-network jet per quadrature point: each
    hidden->hidden layer multiplies 4 forward columns (activation increment and
    three input tangents) and, for the Hessian, 1 adjoint column by the
    width x width weights: 2 * width^2 flops per column."""
    cols = 5 if with_hessian else 4
    return (n_hidden - 1) * cols * 2 * width * width


def time_assembly(ctx, fields, out, precision, steps, warmup, torch):
    for _ in range(warmup):
        ctx.assemble(*fields, precision, out=out)
    torch.cuda.synchronize()
    ctx.check_status()
    ctx.profile(True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        ctx.assemble(*fields, precision, out=out)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.check_status()
    return ms, prof


def cpu_baseline(case, n_elems):
    """The oracle, as it stands, on the first n_elems elements of the workload."""
    import torch

    import workloads as W
    from oracle import fem

    model = fem.Model(case)
    d = fem.dof_vector(case.u, case.phi)
    sub = W.Mesh(case.mesh.dim, case.mesh.X, case.mesh.conn[:n_elems])
    t0 = time.perf_counter()
    fem.assemble(model, sub, d, case.kappa[:n_elems])
    dt = time.perf_counter() - t0
    nq = n_elems * case.mesh.nqp
    return dict(value=nq / dt, unit="qp/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"FP64 residual+tangent assembly of the first {n_elems} elements "
                       f"({nq} qp) of the 64^3 Hex8 workload, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-elems", type=int, default=8192)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "bf16", "fp16"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharded "
              f"design is described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2604_03411_amd import gedmg as G

    torch.cuda.set_device(0)
    case = W.make_case(4)
    mesh = case.mesh
    nq = mesh.n_elems * mesh.nqp
    print(f"[bench] {case.name}: {mesh.n_elems} elements, {nq} qp, building context", file=sys.stderr,
          flush=True)
    ctx = G.Context.from_case(case)
    fields = ctx.fields(case.u, case.phi, case.kappa)
    out = (torch.empty(ctx.ndof, dtype=torch.float64, device="cuda"),
           torch.empty(ctx.nnz, dtype=torch.float64, device="cuda"),
           torch.empty(mesh.n_elems, mesh.nqp, dtype=torch.float64, device="cuda"))
    print(f"[bench] nnz {ctx.nnz}; timing {args.steps} {args.precision} assemblies", file=sys.stderr,
          flush=True)
    ms, prof = time_assembly(ctx, fields, out, args.precision, args.steps, args.warmup, torch)
    ms_step = ms / args.steps
    value = nq / (ms_step * 1e-3)
    H, L = case.energy.width, case.energy.n_hidden
    jet_ms = prof["jets"] / max(prof["calls"], 1)
    elem_ms = prof["elements"] / max(prof["calls"], 1)
    fill_ms = prof["fills"] / max(prof["calls"], 1)
    in_ms = prof["inputs"] / max(prof["calls"], 1)
    flops = jet_flops_per_qp(H, L) * nq
    peak = PEAK_FP64_TFLOPS if args.precision == "fp64" else PEAK_BF16_TFLOPS
    jet_tf = flops / (jet_ms * 1e-3) / 1e12
    dominant = "energy_jet" if jet_ms >= elem_ms else "element"
    roofline = dict(bound="mfma", achieved=round(jet_tf, 3), peak=peak, unit="TFLOP/s",
                    frac=round(jet_tf / peak, 4), traffic=None, kernel=f"jet_{args.precision}_kernel",
                    flops_per_qp=jet_flops_per_qp(H, L), ms_per_launch=round(jet_ms, 4))
    print(f"[bench] {ms_step:.3f} ms/step; phases ms: inputs {in_ms:.3f} jets {jet_ms:.3f} "
          f"elements {elem_ms:.3f} fills {fill_ms:.3f}", file=sys.stderr, flush=True)

    extra = {}
    if args.precision == "fp64":
        try:
            ms2, prof2 = time_assembly(ctx, fields, out, "bf16", args.steps, args.warmup, torch)
            extra["mixed_bf16"] = dict(value=nq / (ms2 / args.steps * 1e-3), ms_per_step=ms2 / args.steps,
                                       speedup_vs_fp64=ms / ms2,
                                       jet_ms=prof2["jets"] / max(prof2["calls"], 1),
                                       element_ms=prof2["elements"] / max(prof2["calls"], 1))
        except G.GedmgError as e:
            extra["mixed_bf16"] = f"unavailable: {e}"

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the oracle on {args.cpu_sample_elems} elements", file=sys.stderr, flush=True)
        cpu = cpu_baseline(case, args.cpu_sample_elems)

    line = dict(
        metric="qp residual+tangent evals/sec", value=value, unit="qp/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64" if args.precision == "fp64" else args.precision,
        data="synthetic",
        config=dict(workload=case.name, elements=mesh.n_elems, qp=nq, dofs=ctx.ndof, nnz=ctx.nnz,
                    energy_net=f"3-{H}x{L}-1", yield_net=f"1-{case.yield_.width}x{case.yield_.n_hidden}-1",
                    precision=args.precision),
        phases_ms=dict(inputs=in_ms, jets=jet_ms, elements=elem_ms, fills=fill_ms, dominant=dominant),
        roofline=roofline, cpu_baseline=cpu, **extra)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
