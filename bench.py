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
Further sections of the same line: `stream` (the device's copy/triad/read
bandwidth with the library's own streaming kernels), `box20x8_N15` (20^3
hexahedra stretched 8:1, N = 15: the FP64 and FP32 matrix-core operators
against the vector kernel, PCG in FP64 and FP32-refined form, the latter with
inner tolerance 1e-3), `batch64` (64 instances of orders 3..8 solved in one
batched call against one by one) and
`cube4_N4` (the small cube: FP64 latency to 1e-8, the refined form to 1e-10
with a sweep of its inner tolerance).  `cpu_baseline` times the FP64 oracle on
the host: its operator on a sample of the 56^3 mesh, and its PCG.

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


def kernel_text(src: str, name: str) -> str:
    """Definition of kernel `name` in the kernel header: from its template line
    to the closing brace in column 0."""
    i = src.index("\n" + name + "(")
    start = src.rfind("\ntemplate", 0, i)
    end = src.index("\n}\n", i) + 3
    return src[start:end]


def kernel_hash(element_kernel: str = "ax_line_kernel") -> str:
    """Hash of what the operator counters measure: the helpers ahead of the
    first kernel, the element kernel and the shared-node gather kernel (edits
    elsewhere in the header leave counters taken on these valid)."""
    with open(KERNEL_SRC) as f:
        src = f.read()
    pre = src[:src.index("__global__")]
    name = element_kernel.split("<")[0]
    text = pre + kernel_text(src, name) + kernel_text(src, "gs_kernel")
    return hashlib.sha256(text.encode()).hexdigest()[:16]


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
    if c.get("element_kernel") != kernel or c.get("kernel_hash") != kernel_hash(kernel):
        return None
    return c.get("bytes_per_apply")


def host_info():
    """Host description for the CPU baseline: model name, cores available to
    this process, and a one-thread numpy triad a = b + 0.5 c over 3 x 256 MiB."""
    import numpy as np

    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    n = 1 << 25
    b, c = np.ones(n), np.full(n, 2.0)
    a = np.empty(n)
    best = 1e30
    for _ in range(5):
        t0 = time.perf_counter()
        np.multiply(c, 0.5, out=a)
        np.add(a, b, out=a)
        best = min(best, time.perf_counter() - t0)
    # multiply reads c, writes a; add reads a and b, writes a
    return {"cpu_model": model, "nproc": cores, "triad_gbs_1thread": round(5 * 8 * n / best / 1e9, 2)}


def cpu_baseline(mesh, N, n_global, gpu_pcg_iterations=None, budget_s=10.0, sample_elems=4096):
    """The FP64 oracle timed on the host, one thread (numpy einsum and vector
    operations; BLAS pinned to one thread): its operator on a sample of the
    workload's elements, scaled to GDOF/s of the full workload; its PCG on the
    4^3, N = 4 cube to 1e-8 in full; and one PCG iteration (operator, two-scale
    preconditioner, vector updates) on a 12^3-hex sample of the 56^3, N = 7
    workload, scaled by elements and by the GPU's FP64 iteration count to an
    estimated time to 1e-10 at full size."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import meshgen
    from oracle.problem import Problem

    with threadpool_limits(limits=1):
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
        out = {"value": n_global / t_full / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle apply_A on the first {S} of {mesh.n_elem} elements of the same mesh "
                         f"(N={N}), {reps} reps in {el:.1f} s, {t * 1e3:.1f} ms/apply, scaled by elements"}
        # PCG, config 1 in full
        m1, N1 = meshgen.workload_mesh("cube4_N4")
        t0 = time.perf_counter()
        P1 = Problem(m1.vtx, m1.hex, N1)
        b1 = P1.load(lambda x: meshgen.manufactured_s(x, m1.lengths))
        t1 = time.perf_counter()
        _, it1, _, _ = P1.solve(b1, rtol=1e-8)
        t2 = time.perf_counter()
        out["pcg_cube4_N4"] = {"setup_s": round(t1 - t0, 3), "time_s": round(t2 - t1, 4), "iterations": it1,
                               "rtol": 1e-8}
        # one PCG iteration on a 12^3-hex sample of the N = 7 workload
        ms, Ns = meshgen.cube_mesh(12, perturb=0.15, seed=1506, permute=True), N
        t0 = time.perf_counter()
        Ps = Problem(ms.vtx, ms.hex, Ns)
        setup = time.perf_counter() - t0
        bs = Ps.load(lambda x: meshgen.manufactured_s(x, ms.lengths))
        t0 = time.perf_counter()
        _, its, _, _ = Ps.solve(bs, rtol=1e-30, max_iter=3)
        per_it = (time.perf_counter() - t0) / max(its, 1)
        est = {"sample": f"12^3 hexes, N={Ns}, {Ps.num.n_global} DOFs, {its} iterations timed after a "
                         f"{setup:.1f} s set-up", "s_per_iteration_sample": round(per_it, 3),
               "s_per_iteration_scaled": round(per_it * mesh.n_elem / ms.n_elem, 1)}
        if gpu_pcg_iterations:
            est["gpu_fp64_iterations"] = gpu_pcg_iterations
            est["time_s_estimated"] = round(per_it * mesh.n_elem / ms.n_elem * gpu_pcg_iterations, 1)
        out["pcg_cube56_N7_estimate"] = est
    out.update(host_info())
    return out


def run_batch(args):
    """--workload batch64: the batch section alone, as its own JSON line."""
    res, total, setup_s, inst = batch_section(args)
    out = {"metric": "batched PCG time-to-1e-10, 64 instances (DOF/s, FP64)",
           "value": round(total / res["fp64"]["time_s"], 1), "unit": "DOF/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batch64", "instances": 64, "total_dofs": total, "setup_s": round(setup_s, 2),
                      "orders": [d["N"] for d in inst], "k": [d["k"] for d in inst]},
           "pcg": res}
    print(json.dumps(out), flush=True)


def batch_section(args):
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
    B.close()
    return res, total, setup_s, inst


def run_stream(dev):
    """Copy, triad and read bandwidth of the library's streaming probes over
    three arrays of 2^28 doubles (2 GiB each)."""
    from paper_1506_05996_amd import sem

    r = sem.stream_bench(n=1 << 28, reps=10, device=dev.index or 0)
    out = {k.replace("_gbs", "_tbs"): round(v / 1e3, 3) for k, v in r.items()}
    out["arrays"] = "3 x 2^28 FP64"
    log(f"[bench] stream: {out}")
    return out


def operator_rooflines(M, u, dt_bytes, steps, warmup, tiles):
    """Per tile: element and gather kernel times (HIP events), GDOF/s and the
    HBM fraction of the stored-factor algorithmic bytes at this precision."""
    from paper_1506_05996_amd import sem

    ng, nl = M.n_global, M.n_local
    dtype = sem.SEM_F64 if dt_bytes == 8 else sem.SEM_F32
    keep = M.tile(dtype)
    y = u.new_empty(u.shape)
    out = {}
    for name, t in tiles:
        M.set_tile(t, dtype)
        for _ in range(warmup):
            M.apply_A(u, y)
        te, tg = M.time_apply_A(u, y, steps)
        balg = algorithmic_bytes_ax(nl, ng, dt_bytes)
        ach = balg / ((te + tg) * 1e-3) / 1e9
        out[name] = {"ms_ax_kernel": round(te, 4), "ms_gs_kernel": round(tg, 4),
                     "gdofs": round(ng / ((te + tg) * 1e-3) / 1e9, 2),
                     "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes": balg}}
    M.set_tile(keep, dtype)
    return out


def solve_section(M, b, ue, mN, kw_common, reps, modes=(("fp64", 0), ("fp32_refined", 1))):
    """PCG to the given tolerance in each mode: one warm-up, median of reps,
    FP64 true residual, error against the exact solution (max and m-weighted
    L2), refined against FP64."""
    import numpy as np
    import torch

    res, x64 = {}, None
    for name, mode in modes:
        kw = dict(kw_common, mode=mode)
        M.solve(b, **kw)
        times = []
        for _ in range(max(1, reps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = M.solve(b, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        r = b - M.apply_A(x)
        err = x - ue
        res[name] = {"time_s": round(float(np.median(times)), 4), "iterations": info["iterations"],
                     "outer": info["outer"],
                     "true_rel_residual": float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)),
                     "err_max_vs_exact": float(err.abs().max()),
                     "err_l2m_vs_exact": float(torch.sqrt((mN * err * err).sum())), "reps": len(times)}
        if x64 is None:
            x64 = x.clone()
        else:
            res[name]["rel_l2_vs_fp64"] = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
    if "fp64" in res and "fp32_refined" in res:
        res["speedup_fp32_refined"] = round(res["fp64"]["time_s"] / res["fp32_refined"]["time_s"], 3)
    return res


def manufactured_rhs(M, lengths, dev):
    import torch

    import meshgen

    m_n = M.lumped_mass()
    x_n = M.node_coords()
    mask = M.boundary_mask().astype(bool)
    bh = m_n * meshgen.manufactured_s(x_n, lengths)
    bh[mask] = 0.0
    ue = meshgen.manufactured_u(x_n, lengths)
    ue[mask] = 0.0
    return (torch.tensor(bh, device=dev), torch.tensor(ue, device=dev), torch.tensor(m_n, device=dev))


def run_order15(args, dev):
    """20^3 hexahedra stretched 8:1 in z, N = 15: the operator with the FP64
    and FP32 matrix-core kernels against the vector kernel, each against the
    HBM roofline of its precision; PCG to 1e-10 in FP64 and FP32-refined form
    (the autotuned tiles: matrix-core kernels in both)."""
    import numpy as np
    import torch

    import meshgen
    from paper_1506_05996_amd import sem

    t0 = time.time()
    mesh, N = meshgen.workload_mesh("box20x8_N15")
    M = sem.Mesh(mesh.vtx, mesh.hex, N)
    setup_s = time.time() - t0
    log(f"[bench] box20x8_N15: n_global={M.n_global}, setup {setup_s:.1f} s, tiles {M.tile(0)} / {M.tile(1)}")
    res = {"workload": "box20x8_N15", "hexes": mesh.n_elem, "order": N, "n_global": M.n_global,
           "setup_s": round(setup_s, 2), "tile_fp64": M.tile(sem.SEM_F64), "tile_fp32": M.tile(sem.SEM_F32)}
    u = torch.tensor(np.random.default_rng(1506).uniform(-1, 1, M.n_global), device=dev)
    tiles = (("mfma", sem.TILE_MFMA), ("line_rebuilt", sem.TILE_LINE_GEO), ("line_stored", sem.TILE_LINE),
             ("vector", 1))
    res["ax_fp64"] = operator_rooflines(M, u, 8, 20, 3, tiles)
    res["ax_fp32"] = operator_rooflines(M, u.float(), 4, 20, 3, tiles)
    del u
    log(f"[bench] box20x8_N15 Ax fp64 {res['ax_fp64']}")
    log(f"[bench] box20x8_N15 Ax fp32 {res['ax_fp32']}")
    b, ue, mN = manufactured_rhs(M, mesh.lengths, dev)
    res["inner_rtol"] = args.inner_rtol_n15
    res["pcg"] = solve_section(M, b, ue, mN, dict(rtol=1e-10, max_iter=4000, inner_rtol=args.inner_rtol_n15,
                                                  max_outer=40), args.pcg_reps)
    log(f"[bench] box20x8_N15 PCG {res['pcg']}")
    M.close()
    return res


def run_small(args, dev):
    """The 4^3-hex cube at N = 4: FP64 PCG to 1e-8 (latency), the refined form
    to 1e-10 for inner tolerances 1e-2 .. 1e-5, and FP64 to 1e-10 beside it."""
    import meshgen
    from paper_1506_05996_amd import sem

    mesh, N = meshgen.workload_mesh("cube4_N4")
    M = sem.Mesh(mesh.vtx, mesh.hex, N)
    b, ue, mN = manufactured_rhs(M, mesh.lengths, dev)
    common = dict(max_iter=1000, max_outer=40)
    res = {"workload": "cube4_N4", "n_global": M.n_global,
           "fp64_rtol1e-8": solve_section(M, b, ue, mN, dict(common, rtol=1e-8), 5, (("fp64", 0),))["fp64"],
           "fp64_rtol1e-10": solve_section(M, b, ue, mN, dict(common, rtol=1e-10), 5, (("fp64", 0),))["fp64"]}
    sweep = {}
    for it in (1e-2, 1e-3, 1e-4, 1e-5):
        sweep[f"{it:g}"] = solve_section(M, b, ue, mN, dict(common, rtol=1e-10, inner_rtol=it), 5,
                                         (("fp32_refined", sem.SOLVE_FP32_REFINED),))["fp32_refined"]
    res["fp32_refined_inner_rtol"] = sweep
    log(f"[bench] cube4_N4 {res}")
    M.close()
    return res


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
    ap.add_argument("--inner-rtol-n15", type=float, default=1e-3,
                    help="refined form on the N = 15 box: tolerance of each FP32 inner solve")
    ap.add_argument("--no-serial", action="store_true", help="batch64: skip the one-by-one comparison")
    ap.add_argument("--no-heat", action="store_true", help="skip the heat-equation run on the rod")
    ap.add_argument("--no-amg", action="store_true", help="skip the PCG runs with the AMG coarse solver")
    ap.add_argument("--no-coef", action="store_true",
                    help="skip the per-element-coefficient / Neumann solve on the main mesh")
    ap.add_argument("--no-n15", action="store_true", help="skip the N = 15 box section")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch section")
    ap.add_argument("--no-small", action="store_true", help="skip the 4^3, N = 4 cube section")
    ap.add_argument("--tile", type=int, default=0,
                    help="counters/profiling runs: force this operator tile in both precisions (0: autotuned)")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection run: 3 FP64 applies and 3 copies of a vector of known size, no timing")
    ap.add_argument("--fine-precond", type=int, default=0, metavar="K",
                    help="profiling run: K applications of the patch-solve preconditioner (FP64, then FP32), no timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library solves each mesh on one "
              f"device and has no multi-GPU path", file=sys.stderr)
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
        # rocprofv3 --pmc runs: the operator in both precisions; the FP64 ->
        # FP32 conversion of u (n_global entries: 8 B read, 4 B written each,
        # known bytes) calibrates the counters
        if args.tile:
            M.set_tile(args.tile, sem.SEM_F64)
            M.set_tile(args.tile, sem.SEM_F32)
        log(f"[bench] counters run: tiles {M.tile(sem.SEM_F64)} / {M.tile(sem.SEM_F32)}")
        for _ in range(3):
            M.apply_A(u, y)
        u32, y32 = u.float(), y.float()
        for _ in range(3):
            M.apply_A(u32, y32)
        torch.cuda.synchronize()
        log(f"[bench] counters run done: calibration (FP64 -> FP32 conversion) {8 * ng} bytes read + "
            f"{4 * ng} written per launch")
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
    # the device's streaming bandwidth and every operator kernel on this mesh
    # (FP64 and FP32; the stored-factor ones against the HBM roofline of their
    # algorithmic bytes), before the timed region
    stream = run_stream(dev)
    tiles = (("stored_plane", 1), ("stored_line", sem.TILE_LINE), ("rebuilt_plane", sem.TILE_GEO),
             ("rebuilt_line", sem.TILE_LINE_GEO))
    kernels = {"fp64": operator_rooflines(M, u, 8, args.steps, args.warmup, tiles),
               "fp32": operator_rooflines(M, u.float(), 4, args.steps, args.warmup, tiles)}
    for dt in ("fp64", "fp32"):
        log(f"[bench] operator kernels {dt}: " + ", ".join(
            f"{k} {v['ms_ax_kernel']:.3f}+{v['ms_gs_kernel']:.3f} ms ({v['gdofs']} GDOF/s)" for k, v in kernels[dt].items()))

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
    geo = tile in (sem.TILE_GEO, sem.TILE_LINE_GEO)
    kname = {sem.TILE_GEO: ("ax_kernel", "ax_kernel<7, double, 1, true, false>"),
             sem.TILE_LINE_GEO: ("ax_line_kernel", "ax_line_kernel<7, double, 1, true, false>"),
             sem.TILE_LINE: ("ax_line_kernel", "ax_line_kernel<7, double, 1, false, false>")}.get(
        tile, ("ax_kernel", "ax_kernel<7, double, %d, false, false>" % tile))
    if geo:
        # the element kernel rebuilds the factors: arithmetic-bound, FP64 vector peak
        falg = algorithmic_flops_ax(nl, N, True)
        achieved = falg / (ms_elem * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_PEAK_TFS, 4),
                    "traffic": traffic_from_counters(kname[1]),
                    "kernel": "%s, factors rebuilt from the element vertices (tile %d)" % (kname[0], tile),
                    "ms_ax_kernel": round(ms_elem, 4), "ms_gs_kernel": round(ms_gs, 4),
                    "algorithmic_flops": falg}
    else:
        achieved = balg / ((ms_elem + ms_gs) * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_from_counters(kname[1]),
                    "kernel": "sem_apply_A = %s (stored factors, tile %d) + gs_kernel" % (kname[0], tile),
                    "ms_ax_kernel": round(ms_elem, 4), "ms_gs_kernel": round(ms_gs, 4),
                    "algorithmic_bytes": balg}
    # the whole application measured against the stored-factor HBM bound
    # (algorithmic bytes B_alg / time / 8 TB/s)
    roofline["frac_of_stored_factor_hbm_bound"] = round(balg / ((ms_elem + ms_gs) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    st = min((kernels["fp64"][k] for k in ("stored_plane", "stored_line")), key=lambda r: r["ms_ax_kernel"])
    roofline["stored_factor_kernel"] = dict(st["roofline"], ms_ax_kernel=st["ms_ax_kernel"],
                                            ms_gs_kernel=st["ms_gs_kernel"])
    roofline["frac_of_stored_factor_bound_at_copy_rate"] = round(
        balg / ((ms_elem + ms_gs) * 1e-3) / 1e12 / stream["copy_tbs"], 4)

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
    del u, y
    if not args.no_heat:
        heat = run_heat(args, dev)

    order15 = None if args.no_n15 else run_order15(args, dev)
    batch = None
    if not args.no_batch:
        bres, btotal, bsetup, binst = batch_section(args)
        batch = {"workload": "batch64", "instances": len(binst), "total_dofs": btotal, "setup_s": round(bsetup, 2),
                 "orders": [d["N"] for d in binst], "k": [d["k"] for d in binst],
                 "dofs_per_s_fp64": round(btotal / bres["fp64"]["time_s"], 1), "pcg": bres}
    small = None if args.no_small else run_small(args, dev)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU baseline (oracle) ...")
        cpu = cpu_baseline(mesh, N, ng, gpu_pcg_iterations=pcg["fp64"]["iterations"] if pcg else None)
        log(f"[bench] CPU baseline: {cpu}")

    out = {"metric": METRIC, "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "hexes": mesh.n_elem, "order": N, "n_global": ng,
                      "perturbation": mesh.meta.get("perturb"), "seed": 1506, "step": "one FP64 apply of A",
                      "setup_s": round(setup_s, 2)},
           "roofline": roofline, "stream_copy_tbs": stream["copy_tbs"], "stream": stream,
           "operator_kernels": kernels, "pcg": pcg, "coefficients": coefs, "heat": heat,
           "box20x8_N15": order15, "batch64": batch, "cube4_N4": small, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
