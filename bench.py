"""Benchmark of the bake-off hot path on one MI355X.

Default workload: BP5 (stiffness, GLL q = N+1, Dirichlet), N = 7, perturbed
brick of E = 64^3 elements (n = N^3 E = 89,915,392 points), uniform[-1,1]
right-hand side (seed 0), Jacobi-PCG with a fixed iteration count (the
paper's timing mode). One step = one CG iteration: operator apply with
gather/scatter, the two fused vector updates and their reductions.

python bench.py [--gpus 1] [--steps 100] [--warmup 20] [--no-sweep] [--no-cpu]

Prints one JSON line (rank 0). DOFs/s = iterations * n / seconds with
n = N^3 E (section 2); the unique-node count is reported beside it. Timing
(section 2: the time of the given number of CG iterations): W warm-up
iterations, then --reps solves of exactly --steps iterations each; `value` is
taken from the median device time of those iterations (HIP events recorded
on the solve's stream before the first and after the last iteration), the
host wall clock around each call (which adds the solve's set-up) is reported
beside it. The operator's average launch comes from one more solve with an
event pair around every operator launch.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "BP5 DOFs/s (CG iters×n/s) at N=7 + n_0.8 on 1 MI355X; % HBM roofline"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_problem(bp: int, N: int, k: int, ncomp: int = 1, seed: int = 0, fp32: bool = False,
                  caller_order: bool | None = None):
    """Mesh, operator and rhs of BPj. The mass problems (BP1/BP2) keep the
    mesh's own lexicographic node numbering (BP_SETUP_CALLER_ORDER): their
    operator assembles Q^T w_L by a gather over the transposed map, which runs
    faster in that order (N=7, E=48^3: 0.900 against 0.944 ms per BP1
    iteration); the stiffness problems use the library's internal order, whose
    element-interior blocks take plain stores instead of atomics."""
    import numpy as np
    import torch

    import synth
    import paper_2004_06722_amd.bp as B
    q, quad = B.bp_quadrature(bp, N)
    ex, ey, ez = synth.element_grid(k) if isinstance(k, int) else k
    xi, _ = B.rule(N + 1, B.GLL)
    mesh = synth.brick_mesh(ex, ey, ez, N, xi, seed=0)
    dirich = mesh.boundary if bp >= 3 else None
    t0 = time.perf_counter()
    if caller_order is None:
        caller_order = bp in (1, 2)
    op = B.Operator(N, q, quad, mesh.elem_dofs, mesh.node_xyz, mesh.nglobal, dirich, ncomp=ncomp,
                    fp32=fp32, caller_order=caller_order)
    t_op = time.perf_counter() - t0
    b = synth.rhs_uniform(mesh.nglobal, seed, ncomp=ncomp, dirichlet=dirich)
    bd = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()     # component-major
    info = {"E": ex * ey * ez, "grid": [ex, ey, ez], "n": N ** 3 * ex * ey * ez,
            "n_unique": int(mesh.nglobal), "operator_setup_s": t_op,
            "node_order": "caller" if caller_order else "internal"}
    del mesh
    return op, bd, info


def time_solve(op, b, steps: int, warmup: int, reps: int = 1, which: int = 3):
    """W warm-up iterations, then `reps` solves of exactly `steps` fixed
    iterations each, synchronised before and after. Returns per solve the
    host wall time around the call (it includes the solve's set-up: the
    permutation into the internal node order and the initial residual) and
    the device time of the `steps` iterations alone (HIP events recorded on
    the solve's stream just before the first and after the last iteration,
    the timing of section 2: the given number of CG iterations)."""
    import torch
    if warmup:
        op.pcg_solve(b, which=which, maxit=warmup, fixed_iters=True)
    walls, loops = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = op.pcg_solve(b, which=which, maxit=steps, fixed_iters=True)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        loops.append(st["ms"] * 1e-3)
        del x
    return walls, loops, st


def median(v):
    v = sorted(v)
    m = len(v) // 2
    return v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_oracle_rate(N: int, k: int, target_s: float, jacobi: bool = True):
    """The oracle's Jacobi-PCG on BP5 at E = 2^k, timed on the host: DOFs/s over
    as many fixed iterations as fit in about target_s, and the cores it used
    (process CPU time over wall time: numpy's einsum and add.at run on one
    thread, a BLAS call may use more). jacobi=False hands the PCG the
    Dirichlet mask as its preconditioner vector instead of the inverse
    diagonal (the same work per iteration; the oracle's diagonal, a plain
    four-operand einsum, takes minutes at E = 32^3)."""
    import numpy as np

    import synth
    from oracle.operators import STIFF, Discretization
    from oracle.pcg import pcg
    from oracle.quadrature import bp_rule
    ex, ey, ez = synth.element_grid(k)
    rule = bp_rule(5, N)
    mesh = synth.brick_mesh(ex, ey, ez, N, rule.xi, seed=0)
    log(f"CPU oracle E={ex}x{ey}x{ez}: geometric factors")
    disc = Discretization(rule, mesh.elem_dofs, mesh.node_xyz, mesh.nglobal, mesh.boundary)
    b = synth.rhs_uniform(mesh.nglobal, 0, dirichlet=mesh.boundary)
    log(f"CPU oracle E={ex}x{ey}x{ez}: preconditioner ({'Jacobi' if jacobi else 'mask'})")
    dinv = disc.jacobi_inverse(STIFF) if jacobi else disc.mask.copy()
    A = lambda v: disc.apply(STIFF, v)
    log(f"CPU oracle E={ex}x{ey}x{ez}: iterations")
    t0 = time.perf_counter()
    pcg(A, b, dinv, maxit=1, fixed_iters=True)
    one = time.perf_counter() - t0
    iters = max(2, min(100, int(target_s / max(one, 1e-3))))
    c0, t0 = os.times(), time.perf_counter()
    pcg(A, b, dinv, maxit=iters, fixed_iters=True)
    dt = time.perf_counter() - t0
    c1 = os.times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    n = N ** 3 * ex * ey * ez
    log(f"CPU oracle E={ex}x{ey}x{ez}: {iters} iterations in {dt:.1f} s "
        f"({cpu / dt:.2f} cores busy)")
    return {"E": [ex, ey, ez], "n": n, "iters": iters, "seconds": dt,
            "DOFs_per_s": iters * n / dt, "cores_used": cpu / dt,
            "preconditioner": "Jacobi" if jacobi else "mask (stand-in, same work)"}


def cpu_baseline(N: int):
    """The oracle beside the GPU: BP5 at E = 16^3 and 32^3 (bounded samples of
    the E = 64^3 workload); the reported value is the 32^3 one."""
    import numpy as np
    small = cpu_oracle_rate(N, 12, 8.0)
    large = cpu_oracle_rate(N, 15, 15.0, jacobi=False)
    cores = max(1, int(round(max(small["cores_used"], large["cores_used"]))))
    return {"value": large["DOFs_per_s"], "unit": "DOFs/s", "cores": cores, "kind": "oracle",
            "sample": f"BP5 N={N}, E=32x32x32 (n={large['n']}): {large['iters']} fixed PCG "
                      f"iterations in {large['seconds']:.1f} s, {large['cores_used']:.2f} cores "
                      "busy (preconditioner vector: the Dirichlet mask, the same work per "
                      "iteration as the Jacobi diagonal, which the oracle takes minutes to form "
                      f"at this size); E=16x16x16 (n={small['n']}, Jacobi): {small['iters']} "
                      "iterations, "
                      f"{small['DOFs_per_s']:.3e} DOFs/s; numpy {np.__version__}, "
                      f"{cpu_model()}, {os.cpu_count()} logical CPUs visible",
            "samples": [small, large]}


def kernel_source_hash() -> str:
    """Hash of what the BK5 operator kernel is built from: kernels.hpp up to
    the end of k_stiff_colloc (its helpers and the kernel), its launcher in
    ops.hip and the compiler flags. Other kernels may change freely."""
    import hashlib
    from paper_2004_06722_amd import build as bp_build
    csrc = os.path.join(ROOT, "paper_2004_06722_amd", "csrc")
    with open(os.path.join(csrc, "kernels.hpp")) as fh:
        k = fh.read()
    k = k[:k.index("// Mass with collocated GLL quadrature")]
    with open(os.path.join(csrc, "ops.hip")) as fh:
        o = fh.read()
    a = o.index("int stiff_colloc(")
    o = o[a:o.index("\n}\n", a)]
    h = hashlib.sha256()
    flags = [f for f in bp_build.common_flags() if not f.startswith("-I")]
    for part in (k, o, " ".join(flags)):
        h.update(part.encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "bk5_p7_e64cube_hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def calib_copy():
    """Plain device copy of known size (2 GiB read + 2 GiB written, 3 times),
    the reference for scaling the HBM byte counters."""
    import torch
    n = 1 << 28
    a = torch.zeros(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"calib-copy: {n * 8} bytes read and written per launch, 3 launches")


def workload_stream(args):
    """Achievable HBM bandwidth on this device: STREAM-style copy (a = b) and
    triad (a = b + s c) over 2 GiB FP64 vectors with torch's kernels, the
    ceiling against which the streaming kernels of the iteration are read."""
    import torch
    n = 1 << 28
    a = torch.zeros(n, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.full_like(a, 2.0)
    out = {}
    for name, fn, words in (("copy", lambda: a.copy_(b), 2),
                            ("triad", lambda: torch.add(b, c, alpha=0.5, out=a), 3)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "GBs": words * 8 * n / (ms * 1e-3) / 1e9, "bytes": words * 8 * n}
        log(f"{name}: {ms:.3f} ms per launch, {out[name]['GBs']:.0f} GB/s")
    return {"workload": "STREAM-style copy and triad, 2^28 FP64 words per vector, 20 timed "
                        "launches after 3 warm-up launches, HIP events", "results": out}


def n08_from_sweep(points):
    """r_max, n_0.8 (log-interpolated first crossing of 0.8 r_max), t_0.8."""
    pts = sorted(points)
    rmax = max(r for _, r in pts)
    target = 0.8 * rmax
    n08 = None
    for (n0, r0), (n1, r1) in zip(pts, pts[1:]):
        if r0 < target <= r1:
            f = (target - r0) / (r1 - r0)
            n08 = math.exp(math.log(n0) + f * (math.log(n1) - math.log(n0)))
            break
    if n08 is None and pts[0][1] >= target:
        n08 = pts[0][0]
    return rmax, n08, (1.25 * n08 / rmax if n08 else None)


# ---------------------------------------------------------------------------
# secondary workloads (one JSON line each); the default run is the BP5 line
# ---------------------------------------------------------------------------
def run_fixed(bp, N, grid, ncomp, steps=100, warmup=10, seed=0, helm_beta=None):
    """Fixed-iteration PCG on BPj (or on H = A + beta B with helm_beta);
    returns a record dict with the operator kernel average."""
    import torch

    from paper_2004_06722_amd import model
    from paper_2004_06722_amd._lib import BP_OPT_TIME_APPLY
    op, b, info = build_problem(bp, N, grid, ncomp=ncomp, seed=seed)
    which = 1 if bp in (1, 2) else 3
    if helm_beta is not None:
        op.set_helmholtz(helm_beta)
        which = 4
    walls, loops, _ = time_solve(op, b, steps, warmup, reps=3, which=which)
    loop, wall = median(loops), median(walls)
    # operator average from a second run with per-launch events (they stay
    # out of the timed runs)
    op.set_option(BP_OPT_TIME_APPLY, 1)
    _, st = op.pcg_solve(b, which=which, maxit=min(steps, 30), fixed_iters=True)
    op.close()
    E, n = info["E"], info["n"]
    log(f"BP{bp} N={N} E={E} ncomp={ncomp}: {steps} iterations in {loop * 1e3:.1f} ms "
        f"(median of 3; wall {wall * 1e3:.1f} ms)")
    apply_ms = st["apply_ms"] / max(st["apply_count"], 1)
    if helm_beta is not None:
        ab = model.helm_apply_bytes(bp, N, E, ncomp)
    elif bp in (1, 2):   # the timed launch is the element kernel (w_L out, no assembly)
        ab = model.mass_element_bytes(N, E, ncomp)
    else:
        ab = model.apply_bytes(bp, N, E, ncomp)
    return {"bp": bp, "helm_beta": helm_beta, "N": N, "E": E, "ncomp": ncomp, "n": n,
            "n_unique": info["n_unique"], "node_order": info["node_order"],
            "iters": steps, "loop_ms": loop * 1e3, "wall_ms": wall * 1e3,
            "ms_per_iter": loop * 1e3 / steps, "DOFs_per_s": steps * n * ncomp / loop,
            "DOFs_per_s_wall": steps * n * ncomp / wall,
            "apply_avg_ms": apply_ms, "apply_alg_GBs": ab / (apply_ms * 1e-3) / 1e9,
            "apply_frac_hbm": ab / (apply_ms * 1e-3) / 1e9 / model.HBM_PEAK_GBS,
            "iter_alg_frac_hbm": model.iteration_bytes(bp, N, E, ncomp) * steps
                                 / loop / 1e9 / model.HBM_PEAK_GBS}


def workload_vector(args):
    """BP2/BP4/BP6 (3 components) against BP1/BP3/BP5 on the same mesh."""
    grid = (48, 48, 48)
    rows = []
    for sbp, vbp in ((1, 2), (3, 4), (5, 6)):
        if vbp not in args.vector_bps:
            continue
        s_rec = run_fixed(sbp, 7, grid, 1)
        log(f"BP{sbp}: {s_rec['DOFs_per_s']:.3e} DOFs/s")
        v_rec = run_fixed(vbp, 7, grid, 3, seed=0)
        log(f"BP{vbp}: {v_rec['DOFs_per_s']:.3e} DOFs/s (3 components)")
        v_rec["ratio_vs_scalar"] = v_rec["DOFs_per_s"] / s_rec["DOFs_per_s"]
        rows += [s_rec, v_rec]
    return {"workload": "vector BPs: BP2/BP4/BP6 (3 components) vs BP1/BP3/BP5, N=7, "
                        "E=48x48x48, 100 fixed PCG iterations, rhs seeds 0,1,2",
            "unit": "DOFs/s (components x n / s)", "records": rows}


def manufactured_problem(N, grid, fp32):
    import numpy as np
    import torch

    import synth
    import paper_2004_06722_amd.bp as B
    xi, _ = B.rule(N + 1, B.GLL)
    mesh = synth.brick_mesh(*grid, N, xi, seed=0)
    op = B.Operator(N, N + 1, B.GLL, mesh.elem_dofs, mesh.node_xyz, mesh.nglobal, mesh.boundary,
                    fp32=fp32)
    xyz = torch.from_numpy(mesh.global_coords()).cuda()
    ue = (torch.sin(np.pi * xyz[:, 0]) * torch.sin(np.pi * xyz[:, 1])
          * torch.sin(np.pi * xyz[:, 2])).contiguous()
    b = op.apply(B.MASS, (3 * np.pi ** 2 * ue).contiguous(), masked=False)
    b = b * torch.from_numpy(1.0 - mesh.boundary.astype(np.float64)).cuda()
    return op, b, ue, mesh.nglobal


def workload_mixed(args):
    """FP32-inner defect correction against FP64 PCG, both to 1e-10, for several
    inner tolerances (1e-5 is the configured one)."""
    import torch
    grid = synth_grid(18)
    op, b, ue, nu = manufactured_problem(7, grid, fp32=True)
    op.pcg_solve(b, maxit=5, fixed_iters=True)          # warm-up
    op.pcg_solve_mixed(b, outer_rtol=1e-2, inner_rtol=1e-1, max_inner=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x64, st64 = op.pcg_solve(b, rtol=1e-10, maxit=100000)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    log(f"FP64 PCG: {st64['iters']} iterations, {t64:.2f} s")
    runs = []
    # reliable updates need the FP32 recursion to stay close to the true
    # residual between replacements: at this conditioning a reduction of 1e-2
    # or more between replacements lets it drift (13k iterations at 1e-2), so
    # the sweep stays at 0.1-0.3 and the FP32 iteration budget at 3x FP64
    cases = [("restart", t) for t in (1e-5, 1e-4, 1e-3, 1e-2, 1e-1)] + \
            [("reliable", t) for t in (3e-1, 2e-1, 1e-1, 5e-2)]
    for mode, inner in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xm, stm = op.pcg_solve_mixed(b, outer_rtol=1e-10, inner_rtol=inner, max_outer=1000,
                                     max_inner=100000 if mode == "restart" else 3 * st64["iters"],
                                     reliable=mode == "reliable")
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        runs.append({"mode": mode, "inner_rtol": inner, "seconds": tm, "outer": stm["outer"],
                     "inner_iters": stm["iters"], "rel_res": stm["rel_res"][0],
                     "converged": stm["converged"], "speedup_vs_fp64": t64 / tm,
                     "max_err_vs_exact": (xm - ue).abs().max().item(),
                     "rel_diff_vs_fp64": ((xm - x64).norm() / x64.norm()).item()})
        log(f"mixed {mode} inner {inner:.0e}: {stm['outer']} outer, {stm['iters']} inner, "
            f"{tm:.2f} s, speedup {t64 / tm:.2f}")
    rec = {"workload": "BP5 N=7 E=64x64x64 manufactured solution sin(pi x)sin(pi y)sin(pi z), "
                       "rhs = M f; FP64 Jacobi-PCG vs FP32-inner FP64 defect correction "
                       "(restarted inner solves, or one FP32 CG with FP64 residual replacement "
                       "after a reduction by inner_rtol), all to relative residual 1e-10",
           "fp64": {"seconds": t64, "iters": st64["iters"], "rel_res": st64["rel_res"][0],
                    "max_err_vs_exact": (x64 - ue).abs().max().item()},
           "mixed": runs,
           "best_speedup": max(r["speedup_vs_fp64"] for r in runs)}
    op.close()
    return rec


def synth_grid(k):
    import synth
    return synth.element_grid(k)


def workload_adjoint(args):
    """Variable-coefficient Poisson with 8 right-hand sides: forward, loss,
    adjoint gradient, and a 32-direction central finite-difference check."""
    import numpy as np
    import torch

    import synth
    import paper_2004_06722_amd.bp as B
    from paper_2004_06722_amd.autograd import mass_norm_loss, poisson_solve
    N, grid, nc = 5, (32, 32, 32), 8
    rtol, maxit = 1e-13, 20000
    t0 = time.perf_counter()
    xi, _ = B.rule(N + 1, B.GLL)
    mesh = synth.brick_mesh(*grid, N, xi, seed=0)
    op = B.Operator(N, N + 1, B.GLL, mesh.elem_dofs, mesh.node_xyz, mesh.nglobal, mesh.boundary,
                    ncomp=nc)
    kap = synth.kappa_log(mesh.node_xyz, 0)              # GLL: quadrature points = nodes
    b = torch.from_numpy(np.ascontiguousarray(synth.rhs_uniform(
        mesh.nglobal, 100, ncomp=nc, dirichlet=mesh.boundary).T)).cuda()
    log(f"setup {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    ut, st = op.pcg_solve(b, rtol=rtol, maxit=maxit)      # kappa = 1 target
    log(f"target solve: {st['iters']} iterations, converged {st['converged']}, "
        f"rel.res {max(st['rel_res']):.2e}, {time.perf_counter() - t0:.1f} s")
    k_t = torch.from_numpy(kap).cuda().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = poisson_solve(op, k_t, b, rtol=rtol, maxit=maxit)
    L = mass_norm_loss(op, u, ut)
    L.backward()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    log(f"forward + loss + adjoint gradient: {t_fb:.2f} s, loss {L.item():.6e}")
    g = k_t.grad.cpu().numpy()
    u0 = u.detach()

    def loss_at(kk):
        op.set_coeff(torch.from_numpy(kk).cuda())
        us, st = op.pcg_solve(b, x=u0.clone(), rtol=1e-15, maxit=maxit)
        d = us - ut
        return 0.5 * torch.sum(d * op.apply(B.MASS, d, masked=False)).item(), st["iters"]

    # Richardson-extrapolated central differences: D(h) = (L(k+h d) - L(k-h d)) / 2h,
    # R = (4 D(h/2) - D(h)) / 3 has an O(h^4) truncation error, so h can be
    # large enough that the rounding noise of L (solves to 1e-15) stays small.
    h = 4e-3
    worst, worst_scaled, fds = 0.0, 0.0, []
    gnorm = float(np.linalg.norm(g))
    t0 = time.perf_counter()
    for j in range(args.fd_directions):
        dlt = synth.fd_direction(kap.shape, 1000 + j)
        D = []
        for hh in (h, h / 2):
            lp, i1 = loss_at(kap + hh * dlt)
            lm, i2 = loss_at(kap - hh * dlt)
            D.append((lp - lm) / (2 * hh))
        fd = (4 * D[1] - D[0]) / 3
        an = float(np.sum(g * dlt))
        err = abs(fd - an) / abs(an)
        scaled = abs(fd - an) / (gnorm * float(np.linalg.norm(dlt)))
        worst, worst_scaled = max(worst, err), max(worst_scaled, scaled)
        fds.append([an, fd, err])
        log(f"FD direction {j}: adjoint {an:.12e} fd {fd:.12e} rel.err {err:.2e} "
            f"({i1} iterations per solve, {time.perf_counter() - t0:.1f} s)")
    t_fd = time.perf_counter() - t0
    op.close()
    return {"workload": "variable-kappa Poisson N=5 E=32x32x32 (n=4,096,000 per rhs), 8 rhs, "
                        "kappa = exp(16-mode field), loss 1/2|u-u_t|_M^2, adjoint gradient, "
                        f"{args.fd_directions} directions, Richardson-extrapolated central differences "
                        "(h = 4e-3, 2e-3; warm-started solves to 1e-15)",
            "loss": L.item(), "forward_backward_s": t_fb, "fd_seconds": t_fd,
            "fd_max_rel_err": worst, "fd_max_err_scaled_by_norms": worst_scaled,
            "fd_pass_1e-6_relative": worst <= 1e-6, "directions": fds}


def workload_sweep13(args):
    """BP1 and BP3 (GL q=N+2), N=1..8, E=2^k with n in [1e4, cap]: DOFs/s curves,
    r_max and n_0.8 per (BP, N)."""
    out = []
    cap = 4e7
    for bp in args.sweep_bp:
        for N in args.sweep_n:
            pts = []
            for k in range(0, 30):
                E = 2 ** k
                n = N ** 3 * E
                if n < 1e4:
                    continue
                if n > cap or E > 2 ** 24:
                    break
                rec = run_fixed(bp, N, synth_grid(k), 1, steps=100, warmup=5)
                pts.append((n, rec["DOFs_per_s"], rec["apply_frac_hbm"], rec["iter_alg_frac_hbm"]))
            rmax, n08, t08 = n08_from_sweep([(a, b) for a, b, _, _ in pts])
            best = max(pts, key=lambda t: t[1])
            log(f"BP{bp} N={N}: r_max {rmax:.3e} n_0.8 {n08:.3e} (apply {best[2]:.2f}, iter {best[3]:.2f} of HBM)")
            out.append({"bp": bp, "N": N, "r_max": rmax, "n_0.8": n08, "t_0.8_s": t08,
                        "apply_frac_hbm_at_rmax": best[2], "iter_frac_hbm_at_rmax": best[3],
                        "points": [[a, b] for a, b, _, _ in pts]})
    return {"workload": f"BP1/BP3 sweep, N=1..8, E=2^k <= 2^24 with 1e4 <= N^3 E <= {cap:.0e}, "
                        "100 fixed PCG iterations each, rhs uniform seed 0", "results": out}


def workload_helmholtz(args):
    """H = A + beta B (eq. (hm2), beta = 1) against the stiffness alone: BP5-type
    (GLL, term fused into the kernel) at N=7, E=64^3 and BP3-type (GL, a second
    kernel) at N=7, E=48^3; 100 fixed Jacobi-PCG iterations each."""
    rows = []
    for bp, grid in ((5, (64, 64, 64)), (3, (48, 48, 48))):
        a = run_fixed(bp, 7, grid, 1)
        h = run_fixed(bp, 7, grid, 1, helm_beta=1.0)
        h["ratio_vs_stiffness"] = h["DOFs_per_s"] / a["DOFs_per_s"]
        log(f"BP{bp}-type N=7: stiffness {a['DOFs_per_s']:.3e}, Helmholtz {h['DOFs_per_s']:.3e} "
            f"DOFs/s (operator {a['apply_avg_ms']:.3f} vs {h['apply_avg_ms']:.3f} ms)")
        rows += [a, h]
    return {"workload": "Helmholtz H = A + B_beta (beta = 1) vs stiffness, N=7, 100 fixed PCG "
                        "iterations, rhs uniform seed 0", "unit": "DOFs/s", "records": rows}


def workload_bk(args):
    """The bake-off kernels on their own (bp_apply_local, w_L = A_L u_L with no
    gather or scatter): E = 2^k elements, N from --sweep-n, per launch time,
    TFLOP/s from the section 5 flop counts, bandwidth of G + u_L + w_L, and
    time per point n_L = N^3 E with the 2x line of the single-GPU BK5 study
    (section 8)."""
    import numpy as np
    import torch

    from paper_2004_06722_amd import model
    bp = args.bk
    which = 3 if bp in (3, 4, 5, 6) else 1
    curves = []
    for N in args.sweep_n:
        pts = []
        for k in range(0, 19):
            E = 2 ** k
            if (N + 1) ** 3 * E > 1.5e8:
                break
            op, _, info = build_problem(bp, N, k)
            nl_words = E * (N + 1) ** 3
            uL = torch.from_numpy(np.random.default_rng(k).uniform(-1.0, 1.0, nl_words)).cuda()
            w = torch.empty_like(uL)
            for _ in range(3):
                op.apply_local(which, uL, out=w)
            reps = 20 if E >= 1024 else 200
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                op.apply_local(which, uL, out=w)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            op.close()
            nl = N ** 3 * E
            fl = model.apply_flops_per_element(bp, N) * E
            by = model.local_apply_bytes(bp, N, E)
            pts.append({"E": E, "n_L": nl, "ms": ms, "TFLOPs": fl / (ms * 1e-3) / 1e12,
                        "GBs": by / (ms * 1e-3) / 1e9, "frac_hbm": by / (ms * 1e-3) / 1e9 /
                        model.HBM_PEAK_GBS, "ns_per_point": ms * 1e6 / nl})
        best = max(pts, key=lambda r: r["TFLOPs"])
        log(f"BK{bp} N={N}: peak {best['TFLOPs']:.2f} TFLOP/s, {best['GBs']:.0f} GB/s "
            f"({100 * best['frac_hbm']:.0f}% HBM) at E={best['E']}; "
            f"min {min(r['ns_per_point'] for r in pts):.3f} ns/point")
        curves.append({"N": N, "points": pts})
    tmin = min(r["ns_per_point"] for c in curves for r in c["points"])
    for c in curves:
        # smallest n_L from which the time per point stays within 2x the minimum
        ok = [r for r in c["points"] if r["ns_per_point"] <= 2 * tmin]
        c["n_L_2x"] = min((r["n_L"] for r in ok), default=None)
    return {"workload": f"BK{bp} alone (bp_apply_local), E = 2^k <= 2^18 with (N+1)^3 E <= 1.5e8, "
                        "mean of 20-200 launches after 3 warm-up launches, u_L uniform[-1,1]",
            "min_ns_per_point": tmin, "curves": curves}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=5, help="timed solves (median reported)")
    ap.add_argument("--N", type=int, default=7)
    ap.add_argument("--k", type=int, default=18, help="E = 2^k elements (default 64^3)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the E = 2^k sweep for n_0.8")
    ap.add_argument("--sweep-k", default="5:17", help="sweep E = 2^k for k in lo:hi")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy", action="store_true", help="run only the counter calibration copy")
    ap.add_argument("--fp32-iters", type=int, default=0,
                    help="profiling aid: also run this many FP32 inner CG iterations")
    ap.add_argument("--fd-directions", type=int, default=32, help="adjoint workload: FD directions")
    ap.add_argument("--sweep-bp", type=int, nargs="+", default=[1, 3], help="sweep13: which BPs")
    ap.add_argument("--sweep-n", type=int, nargs="+", default=list(range(1, 9)),
                    help="sweep13: which orders N")
    ap.add_argument("--cg", default="standard", choices=["standard", "single-reduction"],
                    help="PCG recurrences of the bp5 workload and its sweep")
    ap.add_argument("--vector-bps", type=int, nargs="+", default=[2, 4, 6],
                    help="vector workload: which vector BPs (each with its scalar BP)")
    ap.add_argument("--bk", type=int, default=5, choices=[1, 3, 5],
                    help="bk workload: which bake-off kernel")
    ap.add_argument("--workload", default="bp5",
                    choices=["bp5", "vector", "mixed", "adjoint", "sweep13", "bk", "helmholtz",
                             "stream"],
                    help="bp5: the headline line; the others print their own record")
    args = ap.parse_args()
    if args.calib_copy:
        calib_copy()
        return
    if args.workload != "bp5":
        import torch
        torch.cuda.set_device(0)
        fn = {"vector": workload_vector, "mixed": workload_mixed, "adjoint": workload_adjoint,
              "sweep13": workload_sweep13, "bk": workload_bk,
              "helmholtz": workload_helmholtz, "stream": workload_stream}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU decomposition is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2004_06722_amd.bp as B
    from paper_2004_06722_amd import model
    from paper_2004_06722_amd._lib import BP_OPT_TIME_APPLY
    torch.cuda.set_device(0)
    bp, N, k = 5, args.N, args.k

    log(f"setup BP{bp} N={N} E=2^{k}")
    t0 = time.perf_counter()
    op, b, info = build_problem(bp, N, k)
    log(f"setup done in {time.perf_counter() - t0:.1f} s (operator {info['operator_setup_s']:.2f} s)"
        f": n={info['n']} unique={info['n_unique']}")
    op.set_cg_variant(args.cg == "single-reduction")
    # the headline: repeated solves of exactly `steps` iterations, no
    # per-launch events
    walls, loops, st = time_solve(op, b, args.steps, args.warmup, reps=args.reps)
    loop_s, wall = median(loops), median(walls)
    # the operator's average launch from a separate solve with an event pair
    # (without the system-scope fence) around every operator launch
    op.set_option(BP_OPT_TIME_APPLY, 1)
    _, _, st_ev = time_solve(op, b, args.steps, 0)
    op.set_option(BP_OPT_TIME_APPLY, 0)
    if args.fp32_iters:
        op.close()
        op, b, info = build_problem(bp, N, k, fp32=True)
        op.pcg_solve_mixed(b, outer_rtol=0.0, inner_rtol=0.0, max_outer=1,
                           max_inner=args.fp32_iters)
        torch.cuda.synchronize()
        log(f"ran {args.fp32_iters} FP32 inner iterations")
    log(f"timed {args.reps} x {args.steps} iterations: loop (median) {loop_s * 1e3:.2f} ms, "
        f"wall (median) {wall * 1e3:.2f} ms; loops "
        + ", ".join(f"{x * 1e3:.2f}" for x in loops))
    n, E = info["n"], info["E"]
    value = args.steps * n / loop_s
    apply_avg_ms = st_ev["apply_ms"] / max(st_ev["apply_count"], 1)
    ab = model.apply_bytes(bp, N, E)
    achieved = ab / (apply_avg_ms * 1e-3) / 1e9
    it_bytes = model.iteration_bytes(bp, N, E)
    kname = f"k_stiff_colloc<{N + 1}, double, false, false>"
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": loop_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded perturbed brick mesh, uniform[-1,1] rhs)",
        "config": {"workload": f"BP5 scalar Poisson, GLL q=N+1, N={N}, E={info['grid'][0]}x"
                               f"{info['grid'][1]}x{info['grid'][2]}, Jacobi-PCG fixed "
                               f"{args.steps} iterations",
                   "cg": args.cg,
                   "N": N, "E": E, "n": n, "n_unique": info["n_unique"]},
        "roofline": {"bound": "hbm", "kernel": kname,
                     "achieved": achieved, "peak": model.HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / model.HBM_PEAK_GBS, "traffic": measured_traffic(kname),
                     "bytes_per_launch": ab, "avg_launch_ms": apply_avg_ms},
        "iteration": {"algorithmic_GBs": it_bytes * args.steps / loop_s / 1e9,
                      "frac_hbm": it_bytes * args.steps / loop_s / 1e9 / model.HBM_PEAK_GBS,
                      "fp64_TFLOPs": model.iteration_flops(bp, N, E) * args.steps / loop_s / 1e12,
                      "DOFs_per_s_unique": args.steps * info["n_unique"] / loop_s},
        "timing": {"protocol": f"{args.warmup} warm-up iterations, then {args.reps} solves of "
                               f"exactly {args.steps} fixed iterations; value from the median "
                               "device time of the iterations (HIP events on the solve's stream "
                               "before the first and after the last iteration); wall = host "
                               "clock around each solve call, with its set-up",
                   "loop_ms": [x * 1e3 for x in loops], "wall_ms": [x * 1e3 for x in walls],
                   "spread": (max(loops) - min(loops)) / loop_s,
                   "DOFs_per_s_wall": args.steps * n / wall,
                   "operator_events_solve_ms": st_ev["ms"]},
    }
    op.close()
    del b
    torch.cuda.empty_cache()

    if not args.no_sweep:
        lo, hi = (int(x) for x in args.sweep_k.split(":"))
        pts = [(n, value)]
        for kk in range(lo, min(hi, k - 1) + 1):
            o2, b2, inf2 = build_problem(bp, N, kk)
            o2.set_cg_variant(args.cg == "single-reduction")
            _, l2, _ = time_solve(o2, b2, 100, 10, reps=3)
            r = 100 * inf2["n"] / median(l2)
            pts.append((inf2["n"], r))
            log(f"sweep E=2^{kk}: n={inf2['n']} {r:.3e} DOFs/s")
            o2.close()
            del b2
        rmax, n08, t08 = n08_from_sweep(pts)
        result["sweep"] = {"points": [[a, b_] for a, b_ in sorted(pts)], "r_max": rmax,
                           "n_0.8": n08, "t_0.8_s": t08,
                           "note": "BP5 N=7, E=2^k, 100 iterations each (median device "
                                   "time of 3 solves, as the headline); n = N^3 E; n_0.8 is "
                                   "log-interpolated where DOFs/s first reaches 0.8 r_max"}
    if not args.no_cpu:
        log("timing the CPU oracle")
        result["cpu_baseline"] = cpu_baseline(N)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
