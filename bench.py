"""Benchmark of the MI355X spectral-element Poisson solver (one GPU).

Workload (default): unit cube split into 56^3 trilinear hexahedra, interior
vertices perturbed by +-15% of h (seed 1506), element ids randomly permuted,
order N = 7 (60,698,457 global nodes), manufactured right-hand side of
u = sin(pi x) sin(pi y) sin(pi z), homogeneous Dirichlet boundary.

Timed region: `--steps` back-to-back FP64 operator applications y = A u
(element kernel + shared-node gather) with every input resident in HBM,
bracketed by device synchronisations; HIP events around each kernel on the
launch stream give the per-kernel durations used for the roofline entry.
After the timed region, time-to-tolerance of the PCG solve (||b - A x|| /
||b|| <= 1e-10, true residual) is measured in plain FP64 and in the
FP32-refined form: one untimed warm-up solve per form, then the median of
`--pcg-reps` solves, and once more with the aggregation-AMG coarse solver
(`pcg.amg_coarse_solver`).  Then a solve with one kappa per element and a Neumann
face (`coefficients`), and the heat-equation run (Section 6.2) on a
synthetic rod of 62,500 hexahedra at N = 7: 70 backward Euler steps, each a
PCG solve to 1e-10, in FP64 and FP32-refined form (`heat` in the output).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
FP64_PEAK_TFS = 78.6  # MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
METRIC = "Ax GDOF/s + PCG time-to-1e-10 residual, FP32-refined vs FP64, N=7"
COUNTERS = os.path.join(ROOT, "profiles", "ax_cube56_N7_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1506_05996_amd", "csrc", "sem_kernels.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes_ax(n_local, n_global, s=8):
    """Bytes the operator must move with stored geometry: six G factors and a
    32-bit index per local node, the input and output global vectors once."""
    return n_local * (6 * s + 4) + 2 * s * n_global


def algorithmic_flops_ax(n_local, N, geometry_on_the_fly):
    """Flops per apply: the sum-factorised operator, 12(N+1) + 18 per local
    node; rebuilding the factors from the vertices adds 104 per local node
    (Jacobian columns 18, cross products 27, determinant 5, scale 2, six dot
    products with the scale 36, and the lane's plane-independent parts, 129
    per lane, shared by the N+1 nodes of its pencil: 16)."""
    return n_local * (12 * (N + 1) + 18 + (104 if geometry_on_the_fly else 0))


def pcg_iteration_bytes(E, N, n_local, n_global, coarse_entries, s):
    """Algorithmic HBM bytes of one PCG iteration as the path runs it, with the
    fine-level vectors in s-byte floats and the coarse factor in FP64: the
    operator with the factors rebuilt from the vertices (input gather and
    entity records per local node, 24 vertex doubles per element, the gather
    of the shared nodes), the patch solves (index, residual gather and
    correction per patch node, an index per outside slot), the sum of the
    corrections with the shared-node gather, the restriction, both coarse
    sweeps, and the r and p/x vector updates."""
    patch = E * (N + 3) ** 3
    outside = E * ((N + 3) ** 3 - (N + 1) ** 3)
    shared = n_local - E * (N - 1) ** 3
    op = n_local * (s + 4) + 192 * E + 2 * s * n_global
    fine = patch * (4 + 2 * s) + 4 * outside
    assemble = s * patch + s * n_local + 2 * s * shared
    coarse = s * n_local + 64 * E + 8 * coarse_entries
    vectors = 3 * s * n_global + 5 * s * n_global
    return op + fine + assemble + coarse + vectors


def pcg_roofline(E, N, n_local, n_global, coarse_entries, info, time_s, refined):
    """Time-to-tolerance against the HBM roofline: the iterations' algorithmic
    bytes at the 8 TB/s peak over the measured solve time."""
    if refined:
        inner = info["iterations"] * pcg_iteration_bytes(E, N, n_local, n_global, coarse_entries, 4)
        # each outer step: FP64 operator, true residual, scaling to FP32, FP64 update of x
        outer = (info["outer"] + 1) * (n_local * 12 + 192 * E + 16 * n_global + 56 * n_global)
        total = inner + outer
    else:
        total = info["iterations"] * pcg_iteration_bytes(E, N, n_local, n_global, coarse_entries, 8)
    floor_s = total / (HBM_PEAK_GBS * 1e9)
    return {"bound": "hbm", "algorithmic_bytes": int(total), "floor_s": round(floor_s, 4),
            "frac": round(floor_s / time_s, 4)}


def traffic_from_counters(kernel):
    """HBM bytes per apply from committed rocprofv3 counter runs, when they
    were taken on the current kernel source for this element kernel; else None."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as f:
        c = json.load(f)
    if c.get("kernel_hash") != kernel_hash() or c.get("element_kernel") != kernel:
        return None
    return c.get("bytes_per_apply")


def cpu_baseline(mesh, N, n_global, budget_s=10.0, sample_elems=4096):
    """The FP64 oracle's operator, timed on the host on a sample of the
    workload's elements; scaled to GDOF/s of the full workload."""
    import numpy as np

    from oracle.problem import Problem

    S = min(sample_elems, mesh.n_elem)
    P = Problem(mesh.vtx, mesh.hex[:S], N, fine=False, coarse=False)
    u = np.random.default_rng(1507).uniform(-1, 1, P.num.n_global)
    P.A(u)
    reps, t0 = 0, time.perf_counter()
    while True:
        P.A(u)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    t = el / reps
    t_full = t * mesh.n_elem / S
    return {"value": n_global / t_full / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle apply_A on the first {S} of {mesh.n_elem} elements of the same mesh "
                      f"(N={N}), {reps} reps in {el:.1f} s, {t * 1e3:.1f} ms/apply, scaled by elements"}


def run_batch(args):
    """64 independent solves of uneven size and order in one batched call
    (FP64 and FP32-refined, to a relative residual of 1e-10), against the same
    instances solved one after another through sem_pcg_solve."""
    import numpy as np
    import torch

    import meshgen
    from paper_1506_05996_amd import sem

    dev = torch.device("cuda:0")
    inst = meshgen.batch_instances(64)
    t0 = time.time()
    B = sem.Batch([(d["mesh"].vtx, d["mesh"].hex, d["N"]) for d in inst])
    setup_s = time.time() - t0
    total = int(sum(B.n_global))
    log(f"[bench] batch: 64 instances, {total} DOFs, orders {sorted(set(d['N'] for d in inst))}, "
        f"set-up {setup_s:.1f} s")
    bs = []
    for d in inst:
        H = sem.Mesh(d["mesh"].vtx, d["mesh"].hex, d["N"], host_only=True)
        b = d["rhs"].copy()
        b[H.boundary_mask().astype(bool)] = 0.0
        H.close()
        bs.append(torch.tensor(b, device=dev))
    res = {}
    for name, mode in (("fp64", sem.SOLVE_FP64), ("fp32_refined", sem.SOLVE_FP32_REFINED)):
        B.solve(bs, mode=mode, rtol=1e-10, max_iter=2000, inner_rtol=args.inner_rtol, max_outer=40)  # warm-up
        times = []
        for _ in range(max(1, args.pcg_reps)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            xs, infos, status = B.solve(bs, mode=mode, rtol=1e-10, max_iter=2000, inner_rtol=args.inner_rtol,
                                        max_outer=40)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        its = [i["iterations"] for i in infos]
        res[name] = {"time_s": round(float(np.median(times)), 4), "status": status,
                     "iterations_max": max(its), "iterations_mean": round(float(np.mean(its)), 1),
                     "rel_residual_max": max(i["rel_residual"] for i in infos)}
        log(f"[bench] batch {name}: {res[name]}")
    # the same instances one after another
    if not args.no_serial:
        serial = 0.0
        for d, b in zip(inst, bs):
            M = sem.Mesh(d["mesh"].vtx, d["mesh"].hex, d["N"])
            M.solve(b, rtol=1e-10, max_iter=2000)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            M.solve(b, rtol=1e-10, max_iter=2000)
            torch.cuda.synchronize()
            serial += time.perf_counter() - t1
            M.close()
        res["fp64_one_by_one_s"] = round(serial, 4)
        res["batch_speedup_fp64"] = round(serial / res["fp64"]["time_s"], 3)
        log(f"[bench] one by one fp64: {serial:.3f} s")
    out = {"metric": "batched PCG time-to-1e-10, 64 instances (DOF/s, FP64)",
           "value": round(total / res["fp64"]["time_s"], 1), "unit": "DOF/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batch64", "instances": 64, "total_dofs": total, "setup_s": round(setup_s, 2),
                      "orders": [d["N"] for d in inst], "k": [d["k"] for d in inst]},
           "pcg": res}
    print(json.dumps(out), flush=True)


def run_amg(M, b, dev, args):
    """The coarse solve P_0 as one K-cycle of the aggregation AMG instead of the
    exact inverse: hierarchy, time per application of P_0 (HIP events over 20
    replays of the captured cycle), and PCG to 1e-10 with it in both forms."""
    import numpy as np
    import torch

    from paper_1506_05996_amd import sem

    t0 = time.time()
    M.set_coarse_solver(sem.COARSE_AMG)
    setup = time.time() - t0
    sizes, _ = M.amg_hierarchy()
    R = torch.tensor(np.random.default_rng(1508).uniform(-1, 1, M.n_vertices), device=dev)
    Z = torch.empty_like(R)
    M.coarse_solve(R, Z)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(20):
        M.coarse_solve(R, Z)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 20
    M.set_coarse_solver(sem.COARSE_EXACT)
    M.coarse_solve(R, Z)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(20):
        M.coarse_solve(R, Z)
    ev1.record()
    torch.cuda.synchronize()
    ms_exact = ev0.elapsed_time(ev1) / 20
    M.set_coarse_solver(sem.COARSE_AMG)
    res = {"levels": [int(v) for v in sizes], "setup_s": round(setup, 2), "ms_per_P0": round(ms, 3),
           "ms_per_exact_coarse_solve": round(ms_exact, 3)}
    for name, mode in (("fp64", sem.SOLVE_FP64), ("fp32_refined", sem.SOLVE_FP32_REFINED)):
        kw = dict(mode=mode, rtol=1e-10, max_iter=2000, inner_rtol=args.inner_rtol, max_outer=40)
        M.solve(b, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = M.solve(b, **kw)
        torch.cuda.synchronize()
        res[name] = {"time_s": round(time.perf_counter() - t0, 4), "iterations": info["iterations"],
                     "outer": info["outer"], "rel_residual": info["rel_residual"]}
        log(f"[bench] AMG coarse solver {name}: {res[name]}")
    M.set_coarse_solver(sem.COARSE_EXACT)
    log(f"[bench] AMG: levels {res['levels']}, P_0 {ms:.3f} ms vs exact {ms_exact:.3f} ms")
    return res


def run_coefficients(M, mesh, dev, args):
    """Per-element coefficients and Neumann data on the same mesh: kappa_e
    log-uniform in [0.1, 10] (seed 1507; 1 on the elements with a face on
    z = Lz), c_e = 0, Dirichlet on every face but z = Lz, Neumann g = 1 there,
    source s = 1.  The operator timed, then PCG to 1e-10 in FP64 and
    FP32-refined form (one warm-up solve each)."""
    import numpy as np
    import torch

    import meshgen
    from paper_1506_05996_amd import sem

    faces = meshgen.top_faces(mesh)
    kap = 10.0 ** np.random.default_rng(1507).uniform(-1.0, 1.0, mesh.n_elem)
    kap[faces[:, 0]] = 1.0
    t0 = time.time()
    M.set_element_coefficients(kap, None)
    x = M.node_coords()
    Lx, Ly, Lz = mesh.lengths
    top = np.abs(x[:, 2] - Lz) <= 1e-12
    side = ((np.abs(x[:, 0]) <= 1e-12) | (np.abs(x[:, 0] - Lx) <= 1e-12)
            | (np.abs(x[:, 1]) <= 1e-12) | (np.abs(x[:, 1] - Ly) <= 1e-12))
    dirichlet = (M.boundary_mask().astype(bool) & ~(top & ~side)).astype(np.uint8)
    del x, top, side
    M.set_dirichlet(dirichlet)
    b = M.lumped_mass() + M.boundary_face_mass(faces)  # s = 1, kappa g = 1 on the Neumann faces
    b[dirichlet.astype(bool)] = 0.0
    setup = time.time() - t0
    bd = torch.tensor(b, device=dev)
    del b, dirichlet
    u = torch.tensor(np.random.default_rng(1506).uniform(-1, 1, M.n_global), device=dev)
    y = torch.empty_like(u)
    for _ in range(3):
        M.apply_A(u, y)
    te, tg = M.time_apply_A(u, y, 20)
    del u, y
    res = {"kappa": "per element, log-uniform in [0.1, 10]", "neumann_faces": int(len(faces)),
           "setup_s": round(setup, 2), "ms_ax_kernel": round(te, 4), "ms_gs_kernel": round(tg, 4)}
    for name, mode in (("fp64", sem.SOLVE_FP64), ("fp32_refined", sem.SOLVE_FP32_REFINED)):
        kw = dict(mode=mode, rtol=1e-10, max_iter=4000, inner_rtol=args.inner_rtol, max_outer=40)
        M.solve(bd, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, info = M.solve(bd, **kw)
        torch.cuda.synchronize()
        r = bd - M.apply_A(xs)
        res[name] = {"time_s": round(time.perf_counter() - t0, 4), "iterations": info["iterations"],
                     "outer": info["outer"],
                     "true_rel_residual": float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(bd))}
        log(f"[bench] coefficients {name}: {res[name]}")
    return res


def run_node_coefficients(M, mesh, dev, args):
    """kappa at every node on the same mesh: kappa(x) = 1 + 0.5 sin(2 pi x/Lx)
    sin(2 pi y/Ly) sin(2 pi z/Lz), c = 0, Dirichlet on the whole boundary,
    source s = 1.  The operator (factors scaled by kappa, read from memory)
    timed, then PCG to 1e-10 in FP64 and FP32-refined form (one warm-up solve
    each).  Constant coefficients are restored afterwards."""
    import numpy as np
    import torch

    from paper_1506_05996_amd import sem

    t0 = time.time()
    Lx, Ly, Lz = mesh.lengths
    xl = M.node_coords()[M.numbering().reshape(M.n_elem, -1)]  # [E, (N+1)^3, 3]
    kap = 1.0 + 0.5 * (np.sin(2 * np.pi * xl[..., 0] / Lx) * np.sin(2 * np.pi * xl[..., 1] / Ly)
                       * np.sin(2 * np.pi * xl[..., 2] / Lz))
    del xl
    M.set_dirichlet(M.boundary_mask())
    M.set_node_coefficients(kap, None)
    del kap
    b = M.lumped_mass()
    b[M.boundary_mask().astype(bool)] = 0.0
    setup = time.time() - t0
    bd = torch.tensor(b, device=dev)
    del b
    u = torch.tensor(np.random.default_rng(1506).uniform(-1, 1, M.n_global), device=dev)
    y = torch.empty_like(u)
    for _ in range(3):
        M.apply_A(u, y)
    te, tg = M.time_apply_A(u, y, 20)
    del u, y
    res = {"kappa": "per node, 1 + 0.5 sin sin sin", "setup_s": round(setup, 2),
           "ms_ax_kernel": round(te, 4), "ms_gs_kernel": round(tg, 4)}
    for name, mode in (("fp64", sem.SOLVE_FP64), ("fp32_refined", sem.SOLVE_FP32_REFINED)):
        kw = dict(mode=mode, rtol=1e-10, max_iter=4000, inner_rtol=args.inner_rtol, max_outer=40)
        M.solve(bd, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, info = M.solve(bd, **kw)
        torch.cuda.synchronize()
        r = bd - M.apply_A(xs)
        res[name] = {"time_s": round(time.perf_counter() - t0, 4), "iterations": info["iterations"],
                     "outer": info["outer"],
                     "true_rel_residual": float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(bd))}
        log(f"[bench] node coefficients {name}: {res[name]}")
    M.set_coefficients(1.0, 0.0)
    return res


def run_heat(args, dev):
    """The heat-equation run of Section 6.2 on the synthetic rod: 70 backward
    Euler steps (kappa = 1e-2, dt = 0.04, c = 1/dt, moving source), each a PCG
    solve to 1e-10 started from the previous step, in FP64 and in the
    FP32-refined form.  Sources are generated on the device before the timed
    loop; one untimed step per form first (coefficient set-up, coarse
    refactorisation, work vectors)."""
    import numpy as np
    import torch

    import meshgen
    from paper_1506_05996_amd import sem

    H = meshgen.HEAT
    t0 = time.time()
    mesh, N = meshgen.workload_mesh("rod625_N7")
    M = sem.Mesh(mesh.vtx, mesh.hex, N)
    setup_s = time.time() - t0
    ng = M.n_global
    x = torch.tensor(M.node_coords(), device=dev)
    steps, dt, kappa = H["steps"], H["dt"], H["kappa"]
    qs = [meshgen.heat_source(x, dt * (s + 1), mesh.lengths, exp=torch.exp) for s in range(steps)]
    del x
    log(f"[bench] heat: rod {mesh.n_elem} hexes, N={N}, n_global={ng}, setup {setup_s:.1f} s")
    res = {"workload": "rod625_N7", "hexes": mesh.n_elem, "order": N, "n_global": ng, "steps": steps,
           "dt": dt, "kappa": kappa, "rtol": 1e-10, "setup_s": round(setup_s, 2)}
    finals = {}
    for name, mode in (("fp64", sem.SOLVE_FP64), ("fp32_refined", sem.SOLVE_FP32_REFINED)):
        kw = dict(mode=mode, rtol=1e-10, max_iter=2000, inner_rtol=args.inner_rtol, max_outer=40)
        u = torch.zeros(ng, dtype=torch.float64, device=dev)
        M.heat_step(u, dt, kappa, q=qs[0], **kw)  # warm-up (result discarded)
        u.zero_()
        its = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            u, info = M.heat_step(u, dt, kappa, q=qs[s], u_next=u, **kw)
            its += info["iterations"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        finals[name] = u
        res[name] = {"time_s": round(el, 3), "ms_per_step": round(el / steps * 1e3, 2), "iterations": its,
                     "u_max": float(u.max())}
        log(f"[bench] heat {name}: {res[name]}")
    res["speedup_fp32_refined"] = round(res["fp64"]["time_s"] / res["fp32_refined"]["time_s"], 3)
    d = finals["fp32_refined"] - finals["fp64"]
    res["fp32_refined_vs_fp64_rel_l2"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(finals["fp64"]))
    del qs, finals
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cube56_N7")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--pcg-reps", type=int, default=3, help="timed solves per mode (median), after one warm-up")
    ap.add_argument("--inner-rtol", type=float, default=3e-3, help="refined form: tolerance of each FP32 inner solve")
    ap.add_argument("--no-serial", action="store_true", help="batch64: skip the one-by-one comparison")
    ap.add_argument("--no-heat", action="store_true", help="skip the heat-equation run on the rod")
    ap.add_argument("--no-amg", action="store_true", help="skip the PCG runs with the AMG coarse solver")
    ap.add_argument("--no-coef", action="store_true",
                    help="skip the per-element-coefficient / Neumann solve on the main mesh")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection run: 3 FP64 applies and 3 copies of a vector of known size, no timing")
    ap.add_argument("--fine-precond", type=int, default=0, metavar="K",
                    help="profiling run: K applications of the patch-solve preconditioner (FP64, then FP32), no timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        run_batch(args)
        return

    import numpy as np
    import torch

    import meshgen
    from paper_1506_05996_amd import sem

    dev = torch.device("cuda:0")
    t0 = time.time()
    mesh, N = meshgen.workload_mesh(args.workload)
    lengths = mesh.lengths
    log(f"[bench] mesh {args.workload}: {mesh.n_elem} hexes, N={N} ({time.time() - t0:.1f} s)")
    t0 = time.time()
    M = sem.Mesh(mesh.vtx, mesh.hex, N)
    setup_s = time.time() - t0
    log(f"[bench] setup: n_global={M.n_global} n_local={M.n_local} in {setup_s:.1f} s")
    ng, nl = M.n_global, M.n_local

    u = torch.tensor(np.random.default_rng(1506).uniform(-1, 1, ng), device=dev)
    y = torch.empty_like(u)
    if args.counters:
        # rocprofv3 --pmc runs: the operator, then a plain device copy of
        # n_global doubles (known bytes) that calibrates the counters
        for _ in range(3):
            M.apply_A(u, y)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(u)
        torch.cuda.synchronize()
        log(f"[bench] counters run done: copy bytes per launch {8 * ng} read + {8 * ng} written")
        return
    if args.fine_precond > 0:
        # rocprofv3 runs of the patch solves alone (sem_precond with the fine part only)
        for dt in (torch.float64, torch.float32):
            ud, yd = u.to(dt), y.to(dt)
            for _ in range(args.fine_precond):
                M.precond(ud, yd, pc=sem.PC_FINE)
        torch.cuda.synchronize()
        log(f"[bench] fine-preconditioner run done: {args.fine_precond} applications per dtype")
        return
    for _ in range(args.warmup):
        M.apply_A(u, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_elem, ms_gs = M.time_apply_A(u, y, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = ng / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] Ax: {ms_per_step:.3f} ms/apply wall, kernels {ms_elem:.3f} + {ms_gs:.3f} ms")

    balg = algorithmic_bytes_ax(nl, ng)
    tile = M.tile(sem.SEM_F64)
    geo = tile == sem.TILE_GEO
    if geo:
        # the element kernel rebuilds the factors: arithmetic-bound, FP64 vector peak
        falg = algorithmic_flops_ax(nl, N, True)
        achieved = falg / (ms_elem * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_PEAK_TFS, 4),
                    "traffic": traffic_from_counters("ax_kernel<7, double, 1, true, false>"),
                    "kernel": "ax_kernel, factors rebuilt from the element vertices (tile %d)" % tile,
                    "ms_ax_kernel": round(ms_elem, 4), "ms_gs_kernel": round(ms_gs, 4),
                    "algorithmic_flops": falg}
    else:
        achieved = balg / ((ms_elem + ms_gs) * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_from_counters("ax_kernel<7, double, %d, false, false>" % tile),
                    "kernel": "sem_apply_A = ax_kernel (stored factors, tile %d) + gs_kernel" % tile,
                    "ms_ax_kernel": round(ms_elem, 4), "ms_gs_kernel": round(ms_gs, 4),
                    "algorithmic_bytes": balg}
    # the whole application measured against the stored-factor HBM bound
    # (algorithmic bytes B_alg / time / 8 TB/s)
    roofline["frac_of_stored_factor_hbm_bound"] = round(balg / ((ms_elem + ms_gs) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    if geo:
        # the stored-factor kernel on the same mesh, for its HBM roofline
        M.set_tile(1)
        for _ in range(args.warmup):
            M.apply_A(u, y)
        se, sg = M.time_apply_A(u, y, args.steps)
        M.set_tile(tile)
        ach = balg / ((se + sg) * 1e-3) / 1e9
        roofline["stored_factor_kernel"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                                            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                            "ms_ax_kernel": round(se, 4), "ms_gs_kernel": round(sg, 4),
                                            "algorithmic_bytes": balg}
        log(f"[bench] stored-factor kernel: {se:.3f} + {sg:.3f} ms, {ach / HBM_PEAK_GBS:.3f} of HBM peak")

    pcg = None
    if not args.no_pcg:
        m_n = M.lumped_mass()
        x_n = M.node_coords()
        mask = M.boundary_mask().astype(bool)
        bh = m_n * meshgen.manufactured_s(x_n, lengths)
        bh[mask] = 0.0
        ue = meshgen.manufactured_u(x_n, lengths)
        ue[mask] = 0.0
        del x_n
        b = torch.tensor(bh, device=dev)
        ue_d = torch.tensor(ue, device=dev)
        mN = torch.tensor(m_n, device=dev)
        pcg = {}
        for name, mode in (("fp64", sem.SOLVE_FP64), ("fp32_refined", sem.SOLVE_FP32_REFINED)):
            times, info = [], None
            kw = dict(mode=mode, rtol=1e-10, max_iter=2000, inner_rtol=args.inner_rtol, max_outer=40)
            M.solve(b, **kw)  # warm-up: work vectors, graph capture of the coarse sweeps
            for _ in range(max(1, args.pcg_reps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = M.solve(b, **kw)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            # true residual in FP64 and error against the exact solution
            r = b - M.apply_A(x)
            res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
            err = x - ue_d
            emax = float(err.abs().max())
            el2 = float(torch.sqrt((mN * err * err).sum()))
            pcg[name] = {"time_s": round(float(np.median(times)), 4), "iterations": info["iterations"],
                         "outer": info["outer"], "true_rel_residual": res, "err_max_vs_exact": emax,
                         "err_l2m_vs_exact": el2, "reps": len(times)}
            if mode == sem.SOLVE_FP64:
                x64 = x.clone()
            else:
                pcg[name]["rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
            pcg[name]["roofline"] = pcg_roofline(mesh.n_elem, N, nl, ng, sum(M.coarse_factor_size()), info,
                                                 pcg[name]["time_s"], mode == sem.SOLVE_FP32_REFINED)
            log(f"[bench] PCG {name}: {pcg[name]}")
        pcg["speedup_fp32_refined"] = round(pcg["fp64"]["time_s"] / pcg["fp32_refined"]["time_s"], 3)
        if not args.no_amg:
            pcg["amg_coarse_solver"] = run_amg(M, b, dev, args)
        del b, ue_d, mN, x64

    coefs = None
    if not args.no_coef:
        coefs = run_coefficients(M, mesh, dev, args)
        coefs["per_node"] = run_node_coefficients(M, mesh, dev, args)

    heat = None
    if not args.no_heat:
        del u, y
        heat = run_heat(args, dev)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU baseline (oracle) ...")
        cpu = cpu_baseline(mesh, N, ng)
        log(f"[bench] CPU baseline: {cpu}")

    out = {"metric": METRIC, "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "hexes": mesh.n_elem, "order": N, "n_global": ng,
                      "perturbation": mesh.meta.get("perturb"), "seed": 1506, "step": "one FP64 apply of A",
                      "setup_s": round(setup_s, 2)},
           "roofline": roofline, "pcg": pcg, "coefficients": coefs, "heat": heat, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
