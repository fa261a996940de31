#!/usr/bin/env python
"""Throughput of the gradient-enhanced damage hot path on one MI355X.

Workload (headline): the 64x64x64 Hex8 unit cube (262 144 elements,
2 097 152 quadrature points, 1 098 500 dofs, 115 024 912 CSR entries) with
the 3 -> 64 -> 64 -> 64 -> 1 energy network and the 1 -> 16 -> 1 yield
network, seeded heterogeneous stretch field, phi ~ U(0, 0.2),
kappa ~ U(0, 0.1).  A step is one FP64 residual + consistent-tangent
assembly: quadrature inputs, energy-network jets, history update, element
integration and coloured CSR scatter.  The metric is quadrature-point
residual+tangent evaluations per second with every input resident in HBM.

Also reported on the same line:
  - the mixed-precision (BF16 and FP16 matrix-core) assembly of the same
    workload, with its error against the FP64 path on the residual
    (integrated stress), the tangent, and the converged displacement of a
    short notched-plate load path solved with the mixed tangent and the FP64
    residual;
  - the load-path adjoint on the 128x128 Q4 workload (20 steps, checkpoint
    every 5 steps), in seconds per load step, with its phases;
  - the per-phase split measured with HIP events on the library's stream, the
    roofline of the dominant kernel, and the FP64 oracle timed on the host
    cores over a bounded sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-mixed] [--no-mixed-paths] [--no-cube-newton] [--no-adjoint]
                       [--copy-probe] [--mfma-probe]
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

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 / FP16 matrix
PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2604_03411_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_energy_jet_fp64_hex8_64cube.txt")
JET_SOURCES = [os.path.join(CSRC, n) for n in ("icnn_jet.hip", "device_common.h")]
ELEM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_element_hex8_64cube.txt")
ELEM_SOURCES = [os.path.join(CSRC, n) for n in ("element.hip", "device_common.h")]
MFMA_FILE = os.path.join(ROOT, "profiles", "mfma_busy_energy_jet_fp64_hex8_64cube.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "sq_counters_assembly_kernels_hex8_64cube.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def jet_flops_per_qp(width, n_hidden):
    """Algorithmic matrix work of the energy-network jet per quadrature point:
    value, gradient (3) and Hessian (6) of the network with respect to its 3
    inputs are 10 columns per point, each multiplied by every width x width
    hidden->hidden weight matrix: (n_hidden - 1) * 10 * 2 * width^2 flops."""
    return (n_hidden - 1) * 10 * 2 * width * width


def jet_issued_flops_per_qp(width, n_hidden):
    """Matrix flops the FP64 jet kernel actually issues: 4 forward columns
    (activation increment, 3 input tangents) and 1 adjoint column per layer;
    the Hessian comes from the adjoint column and the tangents."""
    return (n_hidden - 1) * 5 * 2 * width * width


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


def per_call(prof, key):
    return prof[key] / max(prof["calls"], 1)


def rel_err(a, b):
    return float((a - b).abs().max() / b.abs().max())


def mixed_newton_error(G, W, torch, precision):
    """Converged-state error of a mixed-precision load path against the FP64
    path: notched Q4 32x32 plate, 4 of 8 tension steps, both to ||R_f|| <= 1e-11."""
    case = W.make_case(3, n=32)
    case.n_steps = 8
    out = {}
    for prec in ("fp64", precision):
        ctx = G.Context.from_case(case)
        u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
        iters = 0
        du = W.uniaxial_increment(case)
        for n in range(1, 5):
            bd, bv = W.uniaxial_bc(case, n)
            rep = ctx.newton_step(u, phi, kap, bd, bv, prec, reaction_dofs=W.reaction_dofs(case),
                                  predictor_du=du, newton_rtol=0.0, newton_atol=1e-11, krylov_rtol=1e-13)
            iters += rep["newton_iters"]
        torch.cuda.synchronize()
        out[prec] = (u.clone(), phi.clone(), rep["reaction"], iters)
        ctx.close()
    (u0, p0, r0, i0), (u1, p1, r1, i1) = out["fp64"], out[precision]
    return dict(displacement=rel_err(u1, u0), phi=rel_err(p1, p0), reaction=abs(r1 - r0) / abs(r0),
                newton_iters_fp64=i0, newton_iters_mixed=i1,
                path="notched Q4 32x32, 4 tension steps, ||R_f|| <= 1e-11")


CUBE_N = 12  # edge of the sub-cube of the converged-displacement check (Newton from the
#            seeded field diverges on 16^3 and larger meshes of this construction)


def cube_converged(G, W, torch, case, precision):
    """Converged state of the heterogeneous-stretch cube (the 64^3 workload's
    construction on a CUBE_N^3 mesh) with every boundary node (u and phi)
    prescribed to the seeded field and the interior solved by Newton (FP64
    residual, tangent in `precision`): the converged-displacement recipe of
    the mixed-precision error report.  Returns u, phi, iterations and the wall
    time per Newton iteration."""
    import math

    bd, bv = W.boundary_field_bc(case)
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    atol = 1e-9 * math.sqrt(case.mesh.ndof)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = ctx.newton_step(u, phi, kap, bd, bv, precision, newton_rtol=1e-10, newton_atol=atol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its = max(rep["newton_iters"], 1)
    ctx.close()
    return u, phi, dict(newton_iters=rep["newton_iters"], krylov_iters=rep["krylov_iters"],
                        s_total=dt, ms_per_newton_iter=1e3 * dt / its, residual=rep["res_norm"][-1],
                        backtracks=rep["backtracks"], krylov_fallbacks=rep["krylov_fallbacks"])


def bench_mixed(G, W, torch, ctx, fields, out, ref, steps, warmup, nq, case=None, cube_newton=True, paths=True):
    res = {}
    cube_ref = None
    if cube_newton:
        sub = W.make_case(4, n=CUBE_N)
        log(f"{CUBE_N}^3 heterogeneous cube, boundary on the seeded field: FP64 Newton solve")
        cube_ref = cube_converged(G, W, torch, sub, "fp64")
        log(f"  fp64: {cube_ref[2]['newton_iters']} Newton / {cube_ref[2]['krylov_iters']} Krylov iterations, "
            f"{cube_ref[2]['ms_per_newton_iter']:.1f} ms per Newton iteration")
        res["fp64_cube_newton"] = cube_ref[2]
    for prec in ("bf16", "fp16"):
        try:
            ms, prof = time_assembly(ctx, fields, out, prec, steps, warmup, torch)
        except G.GedmgError as e:
            res[prec] = f"unavailable: {e}"
            continue
        R, K, _ = out
        errs = dict(residual=rel_err(R, ref[0]), tangent=rel_err(K, ref[1]))
        log(f"{prec}: {ms / steps:.3f} ms/step, residual err {errs['residual']:.2e} "
            f"tangent err {errs['tangent']:.2e}" + ("; converged-displacement check" if paths else ""))
        if paths:
            errs.update(mixed_newton_error(G, W, torch, prec))
        if cube_ref is not None:
            u1, p1, info = cube_converged(G, W, torch, sub, prec)
            info.update(displacement=rel_err(u1, cube_ref[0]), phi=rel_err(p1, cube_ref[1]),
                        recipe=f"{CUBE_N}^3 heterogeneous-stretch cube (the 64^3 workload's construction), every "
                               "boundary node (u, phi) on the seeded field, interior solved; relative error "
                               "against the FP64 GPU solve (both to ||R_f|| <= max(1e-10 ||R_f^0||, "
                               "1e-9 sqrt(ndof))); the 6^3 case is compared with the oracle in the tests")
            errs["converged_cube"] = info
            log(f"  {prec} cube: u err {info['displacement']:.2e}, {info['newton_iters']} Newton / "
                f"{info['krylov_iters']} Krylov iterations, {info['ms_per_newton_iter']:.1f} ms per Newton iteration")
        res[prec] = dict(value=nq / (ms / steps * 1e-3), unit="qp/s", ms_per_step=ms / steps,
                         jet_ms=per_call(prof, "jets"), history_ms=per_call(prof, "history"),
                         element_ms=per_call(prof, "elements"),
                         error_vs_fp64=errs)
    return res


def bench_adjoint(G, W, torch, checkpoint_every=5):
    """Load-path adjoint on the 128x128 Q4 workload: targets from the forward
    run with the seeded perturbed weights, gradient at the seeded weights."""
    import numpy as np

    case = W.make_case(5)
    steps = case.n_steps
    ctx = G.Context.from_case(case)
    du = np.stack([W.uniaxial_increment(case)] * steps)
    bcs = [W.uniaxial_bc(case, n) for n in range(1, steps + 1)]
    rd = W.reaction_dofs(case)
    ctx.set_params(case.extra["theta_e_star"], case.extra["theta_y_star"])
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    targets = []
    for n in range(1, steps + 1):
        targets.append(ctx.newton_step(u, phi, kap, *bcs[n - 1], reaction_dofs=rd,
                                       predictor_du=du[n - 1])["reaction"])
    ctx.set_params(case.theta_e, case.theta_y)
    path = G.LoadPath(case.u, case.phi, case.kappa, bcs, rd, targets, predictor_du=du)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, ge, gy, rep = ctx.adjoint(path, checkpoint_every=checkpoint_every)
    dt = time.perf_counter() - t0
    ctx.close()
    return dict(workload=case.name, elements=case.mesh.n_elems, steps=steps, checkpoint_every=checkpoint_every,
                total_disp=case.extra["total_disp"],
                total_disp_note="the path stops at 0.125 (not 0.25): past the seeded networks' limit point "
                                "near 16 % strain displacement control has no unique converged state",
                n_params=int(ge.size + gy.size), s_per_step=dt / steps, total_s=dt, loss=loss,
                forward_s=rep["t_forward_s"], recompute_s=rep["t_recompute_s"], reverse_s=rep["t_reverse_s"],
                newton_iters=rep["newton_iters_total"], krylov_iters=rep["krylov_iters_total"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, n_elems_all, n_elems_one, runs=3):
    """The oracle, as it stands, on the first elements of the workload: the
    median of `runs` timings on all of the host threads torch uses and on one
    thread."""
    import statistics

    import torch

    import workloads as W
    from oracle import fem

    model = fem.Model(case)
    d = fem.dof_vector(case.u, case.phi)
    threads_all = torch.get_num_threads()

    def rate(n_elems, threads):
        torch.set_num_threads(threads)
        sub = W.Mesh(case.mesh.dim, case.mesh.X, case.mesh.conn[:n_elems])
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            fem.assemble(model, sub, d, case.kappa[:n_elems])
            ts.append(time.perf_counter() - t0)
        return n_elems * case.mesh.nqp / statistics.median(ts), ts

    v_all, t_all = rate(n_elems_all, threads_all)
    v_one, t_one = rate(n_elems_one, 1)
    torch.set_num_threads(threads_all)
    return dict(value=v_all, unit="qp/s", cores=threads_all, kind="oracle",
                sample=f"FP64 residual+tangent assembly of the first {n_elems_all} elements "
                       f"({n_elems_all * case.mesh.nqp} qp) of the 64^3 Hex8 workload on {threads_all} threads, "
                       f"median of {runs} ({', '.join(f'{t:.1f}' for t in t_all)} s); one thread: the first "
                       f"{n_elems_one} elements, median of {runs} ({', '.join(f'{t:.1f}' for t in t_one)} s)",
                single_thread=dict(value=v_one, unit="qp/s", cores=1),
                nproc=os.cpu_count(), cpu_model=cpu_model())


def profile_record(path, sources, key="jet_source_sha256"):
    """The JSON record of a committed rocprofv3 counter summary, if it was
    taken on the current sources of the kernel (its SHA-256 over `sources`
    matches); else None (counters of a changed kernel are not reported)."""
    try:
        with open(path) as f:
            rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
        h = hashlib.sha256()
        for p in sources:
            with open(p, "rb") as f:
                h.update(f.read())
        digest = h.hexdigest()
    except (OSError, ValueError, IndexError):
        return None
    if rec.get(key) != digest:
        return None
    return rec


def issue_record(kernel):
    """The instruction-issue row of `kernel` from the committed counter summary,
    if it was taken on the kernel's current sources; else None."""
    try:
        with open(SQ_FILE) as f:
            rows = json.loads([ln for ln in f if ln.startswith("[")][-1])
    except (OSError, ValueError, IndexError):
        return None
    for r in rows:
        if r.get("kernel") != kernel:
            continue
        h = hashlib.sha256()
        try:
            for n in r["hashed_sources"]:
                with open(os.path.join(CSRC, n), "rb") as f:
                    h.update(f.read())
        except (OSError, KeyError):
            return None
        return r if r.get("source_sha256") == h.hexdigest() else None
    return None


def jet_traffic():
    """HBM bytes per jet launch from the committed counter summary, or None."""
    rec = profile_record(TRAFFIC_FILE, JET_SOURCES)
    return None if rec is None else rec.get("bytes_per_launch")


def element_alg_bytes(case, nnz):
    """Algorithmic HBM bytes of the element phase of one assembly: the CSR values
    and the residual written once; nodal u, phi and coordinates and the
    connectivity read once; per point the jet row (80 B), the updated history
    (8 B) and its two sensitivities (16 B) read once."""
    m = case.mesh
    nq = m.n_elems * m.nqp
    return (8 * nnz + 8 * m.ndof + 8 * (2 * m.dim + 1) * m.n_nodes + 4 * m.n_elems * m.nen
            + nq * (80 + 8 + 16))


def copy_probe(torch, mib=1024, reps=3):
    """A plain device copy of known size for scaling the HBM byte counters."""
    a = torch.empty(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: {reps} copies of {mib} MiB")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-elems", type=int, default=8192,
                    help="elements of the oracle sample timed on all host threads")
    ap.add_argument("--cpu-sample-elems-1t", type=int, default=1024,
                    help="elements of the oracle sample timed on one thread")
    ap.add_argument("--no-cube-newton", action="store_true",
                    help="skip the converged-displacement solves of the heterogeneous sub-cube")
    ap.add_argument("--no-mixed-paths", action="store_true",
                    help="skip the mixed-precision load paths (assembly timing and errors only; for counter runs)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="run the FP64 matrix-core calibration probe first (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): it measures the "
              f"single-GPU hot path; a sharded path is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2604_03411_amd import gedmg as G

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(torch)
    if args.mfma_probe:
        # many short blocks, so that every SIMD gets the same share of the work
        n = G.probe_mfma(64 * 256, 250)
        log(f"mfma probe: {n} FP64 16x16x4 products ({n * 2048 / 1e9:.1f} GFLOP)")
    case = W.make_case(4)
    mesh = case.mesh
    nq = mesh.n_elems * mesh.nqp
    log(f"{case.name}: {mesh.n_elems} elements, {nq} qp, building context")
    ctx = G.Context.from_case(case)
    fields = ctx.fields(case.u, case.phi, case.kappa)
    out = (torch.empty(ctx.ndof, dtype=torch.float64, device="cuda"),
           torch.empty(ctx.nnz, dtype=torch.float64, device="cuda"),
           torch.empty(mesh.n_elems, mesh.nqp, dtype=torch.float64, device="cuda"))
    log(f"nnz {ctx.nnz}; timing {args.steps} FP64 assemblies")
    ms, prof = time_assembly(ctx, fields, out, "fp64", args.steps, args.warmup, torch)
    ms_step = ms / args.steps
    value = nq / (ms_step * 1e-3)
    H, L = case.energy.width, case.energy.n_hidden
    jet_ms, elem_ms = per_call(prof, "jets"), per_call(prof, "elements")
    fill_ms, in_ms, hist_ms = per_call(prof, "fills"), per_call(prof, "inputs"), per_call(prof, "history")
    flops = jet_flops_per_qp(H, L) * nq
    jet_tf = flops / (jet_ms * 1e-3) / 1e12
    issued_tf = jet_issued_flops_per_qp(H, L) * nq / (jet_ms * 1e-3) / 1e12
    mfma = profile_record(MFMA_FILE, JET_SOURCES)
    roofline = dict(bound="mfma", achieved=round(jet_tf, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(jet_tf / PEAK_FP64_TFLOPS, 4), traffic=jet_traffic(), kernel="jet_f64_kernel",
                    flops_per_qp=jet_flops_per_qp(H, L), qp_per_launch=nq, ms_per_launch=round(jet_ms, 4),
                    issued_flops_per_qp=jet_issued_flops_per_qp(H, L),
                    issued_frac=round(issued_tf / PEAK_FP64_TFLOPS, 4),
                    mfma_busy_frac=None if mfma is None else mfma.get("mfma_busy_frac"),
                    valu_issue_frac=(issue_record("jet_f64_kernel<64,3,true>") or {}).get("valu_issue_frac"))
    eb = element_alg_bytes(case, ctx.nnz)
    erec = profile_record(ELEM_TRAFFIC_FILE, ELEM_SOURCES, key="source_sha256")
    element_roofline = dict(bound="hbm", achieved=round(eb / (elem_ms * 1e-3) / 1e9, 1), peak=PEAK_HBM_GBS,
                            unit="GB/s", frac=round(eb / (elem_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                            traffic=None if erec is None else erec.get("bytes_per_assembly"),
                            kernel="element_kernel (all colours of one assembly)", algorithmic_bytes=eb,
                            ms_per_assembly=round(elem_ms, 4),
                            valu_issue_frac=(issue_record("element_kernel<3,true> (per colour)") or {}).get(
                                "valu_issue_frac"))
    log(f"{ms_step:.3f} ms/step; phases ms: inputs {in_ms:.3f} jets {jet_ms:.3f} history {hist_ms:.3f} "
        f"elements {elem_ms:.3f} fills {fill_ms:.3f}")

    extra = {}
    if not args.no_mixed:
        ref = (out[0].clone(), out[1].clone())
        extra["mixed"] = bench_mixed(G, W, torch, ctx, fields, out, ref, args.steps, args.warmup, nq, case,
                                     not (args.no_cube_newton or args.no_mixed_paths), not args.no_mixed_paths)
        del ref
    ctx.close()
    del out, fields
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        log("load-path adjoint, 128x128 Q4, 20 steps, checkpoint every 5")
        extra["adjoint"] = bench_adjoint(G, W, torch)
        log(f"adjoint {extra['adjoint']['s_per_step']:.3f} s/step")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle on {args.cpu_sample_elems} elements (all threads) and "
            f"{args.cpu_sample_elems_1t} elements (one thread)")
        cpu = cpu_baseline(case, args.cpu_sample_elems, args.cpu_sample_elems_1t)

    line = dict(
        metric="qp residual+tangent evals/sec", value=value, unit="qp/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=case.name, elements=mesh.n_elems, qp=nq, dofs=int(mesh.ndof), nnz=int(ctx.nnz),
                    energy_net=f"3-{H}x{L}-1", yield_net=f"1-{case.yield_.width}x{case.yield_.n_hidden}-1",
                    precision="fp64", mu_e=case.material["mu_e"],
                    mu_e_rule="initial shear modulus of psi_e = E / (2 (1 + nu)), E = 210, nu = 0.3",
                    energy_monotone_mask=case.energy.monotone_mask),
        phases_ms=dict(inputs=in_ms, jets=jet_ms, history=hist_ms, elements=elem_ms, fills=fill_ms,
                       dominant="energy_jet" if jet_ms >= elem_ms else "element"),
        roofline=roofline, element_roofline=element_roofline, cpu_baseline=cpu, **extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
