"""Benchmark of the CDG2 plaque operator on one MI355X.

One step = one SSP-RK3 time step (three fused operator + stage launches) of the
six-species model on the 64^3 hex grid with the Q2 basis (42,467,328 DOF,
float64), inputs resident in HBM.  Prints ONE JSON line.

  value        operator GDOF/s = 3 * DOF * steps / seconds (three operator
               applications per step)
  roofline     the fused stage kernels against the roof their counted arithmetic
               intensity puts them under: FP64 flops per step (rocprofv3 SQ
               counters, committed profile of the same sources) over the
               algorithmic bytes per step (64 B/DOF: stage 1 reads U and writes
               U1, stages 2 and 3 read two states and write one); above the
               ridge (78.6 TFLOP/s / 8 TB/s) the FP64 roof, else HBM.  The HBM
               fraction (algorithmic bytes / time / 8 TB/s) is reported beside it
               in every case ("hbm"), and the FP64 utilisation ("fp64")
  cpu_baseline the float64 oracle (test infrastructure) timed on the host cores
               for one operator application of the same workload

Extras in the same line (skipped with --no-extras): the 256^2 Q2/Q4 workloads
(graph-replayed applies, 100-step runs), the batched 256-instance run (autotuned
schedule and the best single launch per stage) against the plain entry point
(eager and graph-replayed), the adjoint (forward + gradient against forward), the
implicit SDIRK step against the explicit steps over the same interval, the
comparison diffusion fluxes on the exact heat solution, and the unstructured
triangle (P1-P3) and tetrahedral (P2, P3; the size of the paper's 3D run) meshes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
(default K = 50: the 50-step run of the 64^3 workload)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (dim, n, p, seed key)
    "3d-q2-64": (3, (64, 64, 64), 2, (2,)),
    "2d-q2-256": (2, (256, 256), 2, (1,)),
    "2d-q4-256": (2, (256, 256), 4, (1,)),
    "2d-q1-16": (2, (16, 16), 1, (0,)),
    "3d-q3-48": (3, (48, 48, 48), 3, (2,)),   # same DOF count as 3d-q2-64 (profiling the p = 3 kernel)
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6    # vector FP64 (= matrix FP64 on gfx950)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1403_1157_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_pmc(name: str):
    """The key = value lines of the committed rocprofv3 --pmc summary
    profiles/<name>_pmc.txt, if it was taken on the current kernel sources; else
    None."""
    path = os.path.join(ROOT, "profiles", f"{name}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    return kv


def read_profile(workload: str):
    """HBM traffic and counted FP64 flops per step of a Cartesian workload."""
    kv = read_pmc(f"op_kernel_{workload}")
    try:
        return {"bytes_per_step": float(kv["bytes_per_step"]), "flops_per_step": float(kv["flops_per_step"])}
    except (KeyError, TypeError, ValueError):
        return None


def fp64_of_apply(name: str, k: int, us_apply: float):
    """FP64 rate of one operator application of order k on a simplex mesh, from
    the counted flops per application in profiles/<name>_pmc.txt (None if the
    profile is missing or was taken on other kernel sources)."""
    kv = read_pmc(name)
    try:
        fl = float(kv[f"flops_apply_p{k}"])
    except (KeyError, TypeError, ValueError):
        return None
    tf = fl / (us_apply * 1e-6) / 1e12
    return {"flop_per_apply": fl, "tflop_s": round(tf, 3), "frac": round(tf / FP64_PEAK_TFS, 4)}


def host_cpu_model() -> str:
    """Model name of the host CPU (from /proc/cpuinfo, as lscpu reports it), with
    the CPU family, model and stepping numbers (a virtual machine may report only
    a generic name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = line.split(":", 1)
                    k = k.strip()
                    if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                        info[k] = v.strip()
                if not line.strip() and info:
                    break
    except OSError:
        pass
    name = info.get("model name", "unknown")
    nums = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    return f"{name} ({nums})" if nums else name


def cpu_baseline(dim, n, p, key, dof):
    """Oracle (float64, CPU) on the same workload: one operator application."""
    import torch

    from oracle.cdg2_oracle import Config, Oracle
    from paper_1403_1157_amd import inputs

    threads = torch.get_num_threads()
    U = torch.from_numpy(inputs.initial_modes(dim, n, p, key))
    o = Oracle(Config(dim=dim, n=n, order=p, coeffs=inputs.base_coeffs()))
    reps = 4
    t = time.perf_counter()
    for _ in range(reps):
        o.apply(U)
    sec = (time.perf_counter() - t) / reps
    # single-thread figure on a slab of the same grid (a quarter of the last axis)
    n1 = tuple(n[:-1]) + (max(2, n[-1] // 4),)
    U1 = torch.from_numpy(inputs.initial_modes(dim, n1, p, key))
    o1 = Oracle(Config(dim=dim, n=n1, order=p, coeffs=inputs.base_coeffs()))
    torch.set_num_threads(1)
    try:
        t = time.perf_counter()
        o1.apply(U1)
        sec1 = time.perf_counter() - t
    finally:
        torch.set_num_threads(threads)
    return {"value": round(dof / sec / 1e9, 6), "unit": "GDOF/s", "cores": threads,
            "kind": "oracle", "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{reps} float64 oracle operator applications on the full workload "
                      f"({dof} DOF), {sec:.2f} s each; GDOF/s = DOF / seconds per application",
            "one_thread": {"value": round(U1.numel() / sec1 / 1e9, 6), "unit": "GDOF/s",
                           "sample": f"one application on {'x'.join(map(str, n1))} cells "
                                     f"({U1.numel()} DOF) in {sec1:.2f} s, 1 thread"}}


def time_ms(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def bench_batched(steps=50):
    """256 independent 2D instances (grid side 32..128, order 1..3, coefficients
    within +-50%): the autotuned schedule (graph-replayed), the best single
    launch per stage for all orders (one workgroup per item or persistent),
    against 256 sequential plain per-instance rk_step runs of the same
    instances, eager and replayed from one graph."""
    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.batch import Batch
    from paper_1403_1157_amd.cdg2 import Operator

    insts = inputs.batch_instances(256)
    states, dts, ops = [], [], []
    for it in insts:
        U = torch.from_numpy(inputs.initial_modes(2, it["n"], it["order"], it["key"])).cuda()
        op = Operator(2, it["n"], it["order"], it["coeffs"])
        states.append(U)
        dts.append(op.max_dt(U, 0.9))
        ops.append(op)
    dof = sum(U.numel() for U in states)
    bt = Batch(insts)
    packed = bt.pack(states)
    tune = bt.autotune()
    work = packed.clone()
    bt.rk(work, dts, steps)          # capture + warm the graph
    bt.sync()
    ms_b = time_ms(lambda: bt.rk(work, dts, steps))
    bt.sync()
    # one launch per stage for all orders over the cost-sorted work list: one
    # workgroup per item, or a fixed number of persistent workgroups; best of a few
    ncu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    pers = None
    for eb, mult in ((32, 0), (64, 0), (32, 1), (32, 2), (32, 4), (64, 2)):
        bt.set_schedule(eb, mult * ncu, 0)
        bt.rk(work, dts, steps)
        bt.sync()
        ms = time_ms(lambda: bt.rk(work, dts, steps))
        bt.sync()
        if pers is None or ms < pers[1]:
            pers = ((eb, mult * ncu, 0), ms)
    bt.set_schedule(*tune["schedule"])
    plain = [U.clone() for U in states]

    def run_plain():
        for op, X, dt in zip(ops, plain, dts):
            op.rk_step(X, dt, steps)

    run_plain()
    ms_p = time_ms(run_plain)
    # the same plain launches replayed from one captured graph (no launch overhead)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run_plain()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run_plain()
    graph.replay()
    torch.cuda.synchronize()
    ms_pg = time_ms(graph.replay)
    del graph
    for op in ops:
        op.sync()
        op.close()
    bt.close()
    sched = tune["schedule"]
    return {"instances": 256, "steps": steps, "dof": dof,
            "schedule": sched,
            "schedule_meaning": ("one launch per polynomial order and stage (three per stage, side by side on "
                                 "forked streams), " + ("one workgroup per work item" if sched[1] == 0 else
                                                        f"{sched[1]} persistent workgroups each")
                                 if sched[2] == 2 else
                                 ("one launch per stage over the " + ("cost-sorted" if sched[2] == 0 else "instance-ordered")
                                  + " work list, " + ("one workgroup per work item" if sched[1] == 0 else
                                                      f"{sched[1]} persistent workgroups"))),
            "ms_batched": round(ms_b, 3),
            "single_launch": {"schedule": list(pers[0]), "ms": round(pers[1], 3),
                              "meaning": "one launch per stage for all orders over the cost-sorted list, "
                                         + ("one workgroup per work item" if pers[0][1] == 0 else
                                            f"{pers[0][1]} persistent workgroups")},
            "ms_plain_sequential": round(ms_p, 3), "ms_plain_graph": round(ms_pg, 3),
            "speedup_vs_plain": round(ms_p / ms_b, 3), "speedup_vs_plain_graph": round(ms_pg / ms_b, 3),
            "gdof_steps_per_s_batched": round(dof * steps / (ms_b * 1e-3) / 1e9, 3),
            "gdof_steps_per_s_plain": round(dof * steps / (ms_p * 1e-3) / 1e9, 3),
            "batched_hbm_frac": round(64.0 * dof * steps / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_adjoint(steps=200, ckpt=20):
    """128^2 Q2, 200 SSP-RK3 steps, checkpoints every 20: forward time, forward +
    gradient (loss: L2 mismatch of final n1 and c3 against a target run with the
    21 coefficients perturbed by 10%), and one J^T w apply against one f apply."""
    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.autograd import CDG2RK, mismatch_loss, theta_of
    from paper_1403_1157_amd.cdg2 import Operator

    n = (128, 128)
    c = inputs.adjoint_coeffs()
    U0 = torch.from_numpy(inputs.initial_modes(2, n, 2, (4,))).cuda()
    op = Operator(2, n, 2, c)
    dt = op.max_dt(U0, 0.9)
    tgt = U0.clone()
    opt = Operator(2, n, 2, inputs.adjoint_target_coeffs())
    opt.rk_step(tgt, dt, steps)
    opt.sync()
    vol = 1.0 / (n[0] * n[1])

    def fwd():
        X = U0.clone()
        op.rk_step(X, dt, steps)

    def fwd_bwd():
        X = U0.clone().requires_grad_(True)
        th = theta_of(c).requires_grad_(True)
        L = mismatch_loss(CDG2RK.apply(X, th, op, c, dt, steps, ckpt), tgt, vol)
        L.backward()

    fwd()
    ms_f = time_ms(fwd)
    fwd_bwd()
    ms_fb = time_ms(fwd_bwd)
    w = torch.randn_like(U0)
    out = torch.empty_like(U0)
    op.apply(U0, out)
    op.apply_adjoint(U0, w, out)
    us_a = time_ms(lambda: op.apply(U0, out), 20) * 1e3
    us_t = time_ms(lambda: op.apply_adjoint(U0, w, out), 20) * 1e3
    op.sync()
    return {"workload": "128x128 Q2, 200 SSP-RK3 steps, checkpoint every 20, 21 coefficients + U0",
            "ms_forward": round(ms_f, 3), "ms_forward_and_gradient": round(ms_fb, 3),
            "gradient_over_forward": round(ms_fb / ms_f, 3),
            "us_apply": round(us_a, 2), "us_apply_adjoint": round(us_t, 2),
            "adjoint_over_apply": round(us_t / us_a, 3)}


def bench_implicit(ratio=20.0, order=3):
    """256^2 Q2: one implicit SDIRK step (Jacobian-free Newton-GMRES) of ratio x the
    explicit CFL step against the ratio explicit SSP-RK3 steps that cover the same
    interval (the paper's integrator against the fused explicit one)."""
    import time

    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import Operator

    n = (256, 256)
    U0 = torch.from_numpy(inputs.initial_modes(2, n, 2, (1,))).cuda()
    op = Operator(2, n, 2, inputs.base_coeffs())
    dt = op.max_dt(U0, 0.9)
    kw = dict(order=order, max_newton=10, krylov_dim=30, newton_rtol=1e-8, krylov_rtol=1e-2)
    X = U0.clone()
    op.dirk_step(X, ratio * dt, **kw)            # warm-up (allocates the workspace)
    X = U0.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = op.dirk_step(X, ratio * dt, **kw)
    torch.cuda.synchronize()
    ms_imp = (time.perf_counter() - t) * 1e3
    nsteps = int(round(ratio))
    Y = U0.clone()
    ms_exp = time_ms(lambda: op.rk_step(Y, dt, nsteps))
    op.sync()
    Z = U0.clone()
    op.rk_step(Z, dt * ratio / nsteps, nsteps)
    op.sync()
    diff = float((X - Z).abs().max())
    return {"workload": f"256x256 Q2, SDIRK{order}, dt = {ratio:g} x the explicit CFL step",
            "ms_implicit_step": round(ms_imp, 3), "newton_iters": st["newton_iters"],
            "krylov_iters": st["krylov_iters"], "ms_explicit_same_interval": round(ms_exp, 3),
            "implicit_over_explicit": round(ms_imp / ms_exp, 3), "max_abs_diff_vs_explicit": diff}


def bench_fluxes(n=(128, 128), p=2, a=0.05, T=0.02):
    """The comparison diffusion fluxes on the exact heat solution (the paper's
    error-versus-time comparison, on a problem with a known solution): explicit dt of
    each flux, GPU time to T and the L2 distance to the projected exact solution
    (orthonormal modes: sqrt(|K| sum (U - P)^2), species n1)."""
    import math

    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import Operator

    c = inputs.diffusion_only_coeffs(a)
    U0 = torch.from_numpy(inputs.heat_modes(n, p, 0.0, a)).cuda()
    P = torch.from_numpy(inputs.heat_modes(n, p, T, a)).cuda()
    vol = 1.0 / (n[0] * n[1])
    out = {}
    for flux in ("cdg2", "br2", "ip", "bo", "cdg"):
        op = Operator(2, n, p, c, diff_flux=flux)
        dt = op.max_dt(U0, 0.9)
        nst = int(math.ceil(T / dt))
        U = U0.clone()
        op.rk_step(U, T / nst, 2)
        op.sync()
        U = U0.clone()
        ms = time_ms(lambda: op.rk_step(U, T / nst, nst))
        op.sync()
        err = math.sqrt(vol * float(((U[0] - P[0]) ** 2).sum()))
        out[flux] = {"dt": T / nst, "steps": nst, "ms": round(ms, 3), "l2_error_vs_projection": err}
    return {"workload": f"heat solution, {n[0]}x{n[1]} Q{p}, a = {a}, T = {T}, SSP-RK3 at the CFL step",
            "fluxes": out}


def bench_triangles(n=256, steps=100, reps=200):
    """Unstructured P_k triangles: an n x n Kuhn mesh of [0,1]^2 with jittered
    vertices (2 n^2 triangles), P1, P2 and P3; operator applications and an SSP-RK3
    run.  Algorithmic bytes as for the Cartesian grids (16 B/DOF per apply,
    64 B/DOF per step, state only); the FP64 rate of an application from the
    counted flops of the committed profile (the kernels are arithmetic-bound)."""
    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import TriOperator

    xy, nbr, nbe = inputs.kuhn_mesh(n, n, 0.2, (14,))
    out = {}
    for k in (1, 2, 3):
        op = TriOperator(k, xy, nbr, nbe, inputs.base_coeffs())
        U0 = torch.from_numpy(inputs.tri_modes(len(xy), k, key=(15, k), amp=0.005)).cuda()
        dof = U0.numel()
        F = torch.empty_like(U0)
        op.apply(U0, F)
        op.sync()
        us_apply = 1e3 * time_ms(lambda: op.apply(U0, F), reps)
        U = U0.clone()
        op.rk_step(U, 2e-8, 2)
        op.sync()
        U = U0.clone()
        us_step = 1e3 * time_ms(lambda: op.rk_step(U, 2e-8, steps)) / steps
        op.sync()
        out[f"p{k}"] = {"us_per_apply": round(us_apply, 2), "apply_frac": round(16 * dof / us_apply / 1e3 / HBM_PEAK_GBS, 4),
                        "apply_fp64": fp64_of_apply("tri_kernel_kuhn-256", k, us_apply),
                        "us_per_step": round(us_step, 2), "step_frac": round(64 * dof / us_step / 1e3 / HBM_PEAK_GBS, 4),
                        "gdof_s": round(3 * dof / us_step / 1e3, 3)}
    return {"workload": f"{n}x{n} Kuhn mesh, jittered ({2 * n * n} triangles), {reps} applies and a "
                        f"{steps}-step SSP-RK3 run", **out}


def bench_tetrahedra(n=(26, 26, 28), steps=20, reps=50):
    """Unstructured P_k tetrahedra at the size of the paper's 3D strong-scaling run
    (cubic elements, 113,549 tetrahedra): a jittered Kuhn mesh of 26 x 26 x 28
    cubes, 113,568 tetrahedra; P3 (13,628,160 DOF) and P2; operator applications
    and an SSP-RK3 run.  Algorithmic bytes as for the other grids (state only)."""
    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import TetOperator

    xyz, vid, nbr, nbe = inputs.kuhn_tet_mesh(*n, 0.2, (24,))
    out = {}
    for k in (3, 2):
        op = TetOperator(k, xyz, vid, nbr, nbe, inputs.base_coeffs())
        U0 = torch.from_numpy(inputs.tet_modes(len(xyz), k, key=(25, k), amp=0.005)).cuda()
        dof = U0.numel()
        F = torch.empty_like(U0)
        op.apply(U0, F)
        op.sync()
        us_apply = 1e3 * time_ms(lambda: op.apply(U0, F), reps)
        U = U0.clone()
        op.rk_step(U, 1e-8, 2)
        op.sync()
        U = U0.clone()
        us_step = 1e3 * time_ms(lambda: op.rk_step(U, 1e-8, steps)) / steps
        op.sync()
        out[f"p{k}"] = {"dof": dof, "us_per_apply": round(us_apply, 2),
                        "apply_fp64": fp64_of_apply("tet_kernel_kuhn-26", k, us_apply),
                        "apply_frac": round(16 * dof / us_apply / 1e3 / HBM_PEAK_GBS, 4),
                        "us_per_step": round(us_step, 2), "step_frac": round(64 * dof / us_step / 1e3 / HBM_PEAK_GBS, 4),
                        "gdof_s": round(3 * dof / us_step / 1e3, 3)}
    return {"workload": f"{'x'.join(map(str, n))} Kuhn cubes, jittered ({len(xyz)} tetrahedra), {reps} applies and "
                        f"a {steps}-step SSP-RK3 run", **out}


def bench_2d(reps=1000, steps=100):
    """The 256^2 workloads with Q2 and Q4: reps operator applications replayed
    from one captured HIP graph, and a steps-long SSP-RK3 run."""
    import torch

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import Operator

    out = {}
    for p in (2, 4):
        n = (256, 256)
        U0 = torch.from_numpy(inputs.initial_modes(2, n, p, (1,))).cuda()
        dof = U0.numel()
        op = Operator(2, n, p, inputs.base_coeffs())
        dt = op.max_dt(U0, 0.9)
        f = torch.empty_like(U0)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                op.apply(U0, f)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(10):
                op.apply(U0, f)
        g.replay()
        torch.cuda.synchronize()
        ms_a = time_ms(lambda: [g.replay() for _ in range(reps // 10)]) / reps
        U = U0.clone()
        op.rk_step(U, dt, 2)
        ms_s = time_ms(lambda: op.rk_step(U, dt, steps)) / steps
        op.sync()
        out[f"q{p}"] = {"us_per_apply_graph": round(ms_a * 1e3, 2),
                        "apply_frac": round(16.0 * dof / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "us_per_step": round(ms_s * 1e3, 2),
                        "step_frac": round(64.0 * dof / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "gdof_s": round(3 * dof / (ms_s * 1e-3) / 1e9, 3)}
    return {"workload": f"256x256, {reps} graph-replayed applies and a {steps}-step SSP-RK3 run", **out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="3d-q2-64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 2D, batched, adjoint, implicit and flux measurements")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the slab "
              "decomposition over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(max(1, args.steps)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": max(1, args.steps)}))
        return

    from paper_1403_1157_amd import inputs
    from paper_1403_1157_amd.cdg2 import Operator

    dim, n, p, key = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    U0 = torch.from_numpy(inputs.initial_modes(dim, n, p, key)).to(dev).contiguous()
    dof = U0.numel()
    op = Operator(dim, n, p, inputs.base_coeffs())
    dt = op.max_dt(U0, 0.9)
    U = U0.clone()
    out = torch.empty_like(U0)

    for _ in range(args.warmup):
        op.rk_step(U, dt, 1)
    op.sync()

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        op.rk_step(U, dt, 1)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    op.sync()

    # operator-only launches (apply_operator, 16 B/DOF) for the plain form
    for _ in range(2):
        op.apply(U0, out)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        op.apply(U0, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_apply = ev0.elapsed_time(ev1) / args.steps
    op.sync()

    # five more timed runs of the same K steps: median and minimum
    trials = []
    for _ in range(5):
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            op.rk_step(U, dt, 1)
        ev1.record(stream)
        torch.cuda.synchronize()
        trials.append(ev0.elapsed_time(ev1) / args.steps)
    op.sync()
    trials.sort()
    # plain device copy of the state size: the bandwidth this machine reaches
    src = U0.clone()
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst

    value = 3 * dof / (ms_step * 1e-3) / 1e9
    alg_bytes_step = 64.0 * dof
    achieved = alg_bytes_step / (ms_step * 1e-3) / 1e9
    prof = read_profile(args.workload)
    traffic = prof["bytes_per_step"] if prof else None
    hbm = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic}
    roofline = dict(hbm)
    if prof:
        # counted FP64 flops of the stage kernels (rocprofv3 SQ counters): the
        # arithmetic intensity against the algorithmic bytes decides the bound
        intensity = prof["flops_per_step"] / alg_bytes_step
        fp64_tf = prof["flops_per_step"] / (ms_step * 1e-3) / 1e12
        fp64 = {"achieved_tflop_s": round(fp64_tf, 3), "peak_tflop_s": FP64_PEAK_TFS,
                "frac": round(fp64_tf / FP64_PEAK_TFS, 4), "flop_per_dof_step": round(prof["flops_per_step"] / dof, 1),
                "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(FP64_PEAK_TFS / HBM_PEAK_GBS * 1e3, 2)}
        if intensity > FP64_PEAK_TFS / HBM_PEAK_GBS * 1e3:
            roofline = {"bound": "alu", "achieved": round(fp64_tf, 3), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": round(fp64_tf / FP64_PEAK_TFS, 5), "traffic": traffic,
                        "hbm_frac": hbm["frac"], "hbm_achieved_gb_s": hbm["achieved"]}
    else:
        fp64 = None
    line = {
        "metric": "CDG2 operator GDOF/s (SSP-RK3 stage applications, FP64)",
        "value": round(value, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: six-species CDG2 plaque model, "
                               f"{'x'.join(map(str, n))} cells, Q{p}, one SSP-RK3 step",
                   "dim": dim, "cells": list(n), "order": p, "dof": dof, "dt": dt},
        "roofline": roofline,
        "hbm": hbm,
        "fp64": fp64,
        "trials_ms_per_step": {"median": round(trials[2], 5), "min": round(trials[0], 5),
                               "max": round(trials[-1], 5)},
        "copy_gb_s": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        "apply": {"us_per_apply": round(ms_apply * 1e3, 2),
                  "gdof_s": round(dof / (ms_apply * 1e-3) / 1e9, 4),
                  "alg_gb_s": round(16.0 * dof / (ms_apply * 1e-3) / 1e9, 2)},
    }
    if not args.no_extras:
        line["2d"] = bench_2d()
        line["batched"] = bench_batched()
        line["adjoint"] = bench_adjoint()
        line["implicit"] = bench_implicit()
        line["fluxes"] = bench_fluxes()
        line["triangles"] = bench_triangles()
        line["tetrahedra"] = bench_tetrahedra()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(dim, n, p, key, dof)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
