"""Benchmark: multigrid CGKS on the bump-channel workload, one MI355X.

Workload: inviscid steady channel [0,3]x[0,1]x[0,0.5] with the Gaussian bump
0.05 exp(-25 (x-1.5)^2) on the lower wall, seeded mixed mesh of about 189k
cells (tet, pyramid, prism, hex), inflow Mach 0.5, slip walls, far field at
both ends, 3-level V-cycle with random-hash agglomeration (seed 1, 3 passes per
level), FP64.  One step = one V-cycle, i.e. the whole hot path: fine smoothing
(local step, HWENO, BGK flux at every face Gauss point, gradient update), the
fine residual at the smoothed state, restriction, KFVS forcing and sweeps on
two coarse levels, prolongation and the residual-norm read.

Reported `value`: fine CGKS residual evaluations per second over the timed
steps (each V-cycle evaluates the fine residual twice).  Extra fields: the
isolated cgks_residual rate, time and cycles to a 1e-10 residual drop in FP64
and in mixed precision (on this mesh, which stalls, and on the same channel
meshed with hexahedra only, which converges), the roofline of the face-flux
kernel, adjoint timings on this state with a gradient check against converged
finite differences on a small channel, and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic operations per face Gauss point of the fine flux kernel (inviscid steady mode, FP64),
# counted by instantiating the kernel's per-point source with a counting scalar
# (paper_2402_02075_amd/csrc/flopcount.hip; quadrilateral faces, face sum included).
FLOPS_PER_GP = 3775.75
FP64_PEAK_TFLOPS = 78.6       # MI355X dense FP64 vector
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the same face kernel on this workload, from two rocprofv3 counter passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors read off a 1 GiB copy and fill in the same runs).
# Set to None whenever the face kernel changes until the counters are taken again.
FACE_HBM_BYTES_PER_LAUNCH = 452.9e6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(cg, mg, precision=0):
    m = mg.bump_channel()
    S = cg.Solver(precision=precision)
    t0 = time.perf_counter()
    S.set_mesh(m)
    t_mesh = time.perf_counter() - t0
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        S.set_bc(tag, cg.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        S.set_bc(tag, cg.BC_SLIP)
    t0 = time.perf_counter()
    sizes = S.agglomerate()
    t_agg = time.perf_counter() - t0
    return m, S, sizes, t_mesh, t_agg


def cpu_baseline(mg, budget_s=15.0):
    """The CPU oracle as it stands on a bounded sample of the same workload."""
    import oracle as om
    m = mg.bump_channel()
    M = om.Mesh(m)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, om.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, om.BC_SLIP)
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=3, amp=0.03)
    G = np.zeros((15, m.n_cells))
    al = np.ones(m.n_cells)
    par = om.params()

    def rate(budget):
        rng = np.random.default_rng(0)
        n_sub = 256
        elapsed, done = 0.0, 0
        while elapsed < budget and done < m.n_cells:
            sub = rng.choice(m.n_cells, n_sub, replace=False)
            t0 = time.perf_counter()
            M.residual(par, W, G, al, sub=sub)
            elapsed += time.perf_counter() - t0
            done += n_sub
            if elapsed < 1.0:
                n_sub *= 2
        return done / elapsed, done, elapsed

    cells_per_s, done, elapsed = rate(budget_s)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": cells_per_s / m.n_cells, "unit": "residual evals/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} randomly chosen cells of the {m.n_cells}-cell bump channel (oracle residual on a cell "
                     f"subset, {elapsed:.1f} s), scaled to whole-mesh evaluations"}
    # the same oracle on one core (its OpenMP loop limited to one thread)
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        c1, d1, e1 = rate(budget_s / 3)
        gomp.omp_set_num_threads(threads)
        out["single_core"] = {"value": c1 / m.n_cells, "cores": 1,
                              "sample": f"{d1} cells, {e1:.1f} s, scaled to whole-mesh evaluations"}
    except OSError:
        pass
    return out


def hex_convergence(cg, mg, max_cycles):
    """Time to a 1e-10 drop, FP64, mixed and FP64 with the implicit coarse smoother, on the same
    channel meshed with hexahedra only (96 x 32 x 16 = 49,152 cells), where the scheme converges
    to round-off."""
    import torch
    m = mg.bump_channel(n_prism=0, n_pyr=0)
    res = {"cells": m.n_cells, "mesh": "bump channel 96x32x16, hexahedra only"}
    Wref = None
    # FP64, mixed precision, and FP64 with the implicit coarse smoother (backward Euler with
    # point relaxation on the coarse levels, 2 sweeps at CFL 0.25)
    for prec, smoother, key in ((0, 0, "fp64"), (1, 0, "mixed"), (0, 1, "implicit_coarse")):
        S = cg.Solver(precision=prec, coarse_smoother=smoother, relax_sweeps=2, cfl_implicit=0.25)
        S.set_mesh(m)
        prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
        for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
            S.set_bc(tag, cg.BC_FARFIELD, prim)
        for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
            S.set_bc(tag, cg.BC_SLIP)
        S.agglomerate()
        W0, G0 = mg.uniform_state(m.n_cells)
        W = torch.from_numpy(W0).cuda()
        G = torch.from_numpy(G0).cuda()
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, ok = S.vcycle(W, G, al, max_cycles, 1e-10)
        torch.cuda.synchronize()
        dt_c = time.perf_counter() - t0
        res[key] = {"seconds": dt_c, "cycles": int(len(h)), "reached": bool(ok), "final_drop": float(h[-1] / h[0])}
        F = S.wall_force(W, G, al, mg.TAG_WALL_BOTTOM).cpu().numpy()
        res[key]["lower_wall_force"] = [float(x) for x in F]
        if Wref is None:
            Wref = W.clone()
        else:
            d = (W - Wref)[0].abs()
            res[f"{key}_vs_fp64"] = {"density_max_abs_diff": float(d.max()),
                                     "density_l2_diff": float(torch.sqrt((d * d).mean()))}
        log(f"hex channel {key}: {len(h)} cycles {dt_c:.2f}s drop {h[-1] / h[0]:.3e}")
    return res


def shock_regime(cg, mg, cycles):
    """Viscous sphere at Re 300 (on D = 1), Mach 1.2 (bow shock) and 0.95, adiabatic no-slip wall,
    Riemann far field at r = 20: V-cycles from the free stream on a synthetic 286,720-cell
    prism/tet sphere (first layer 0.023 D); drop reached, cost per cycle and drag coefficient, with
    the paper's drag coefficients on its own 665,914-cell meshes as context."""
    import torch
    m = mg.sphere_shell(level=4, n_layers=24, n_prism=8, first_h=0.023)
    res = {"cells": m.n_cells, "mesh": "sphere shell, icosphere level 4, 24 layers (8 prism), r 0.5..20"}
    paper_cd = {1.2: 1.296, 0.95: 0.963}
    for mach in (1.2, 0.95):
        S = cg.Solver(viscous=1, mu=mach / 300.0, prandtl=0.72)
        S.set_mesh(m)
        S.set_bc(mg.TAG_SPHERE, cg.BC_NOSLIP_ADIABATIC)
        S.set_bc(mg.TAG_FARFIELD, cg.BC_FARFIELD, np.array([1.0, mach, 0.0, 0.0, 1.0 / 1.4]))
        S.agglomerate()
        W0, G0 = mg.uniform_state(m.n_cells, vel=(mach, 0.0, 0.0))
        W = torch.from_numpy(W0).cuda()
        G = torch.from_numpy(G0).cuda()
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, ok = S.vcycle(W, G, al, cycles, 1e-10)
        torch.cuda.synchronize()
        dt_c = time.perf_counter() - t0
        F = S.wall_force(W, G, al, mg.TAG_SPHERE).cpu().numpy()
        cd = float(F[0] / (0.5 * mach * mach * np.pi / 4.0))
        res[f"mach_{mach}"] = {"cycles": int(len(h)), "seconds": dt_c, "ms_per_cycle": 1e3 * dt_c / max(len(h), 1),
                               "final_drop": float(h[-1] / h[0]), "min_drop": float(h.min() / h[0]),
                               "reached_1e-10": bool(ok), "Cd": cd, "Cd_paper": paper_cd[mach],
                               "min_alpha": float(al.min())}
        log(f"sphere Mach {mach}: {len(h)} cycles {dt_c:.2f}s drop {h[-1] / h[0]:.2e} Cd {cd:.4f}")
        S.close()
    return res


def sphere_throughput(cg, mg, levels):
    """Throughput on the larger synthetic meshes: the viscous sphere (Mach 0.2, Re 100 on D, Pr 0.72,
    adiabatic no-slip wall, Riemann far field at r = 20) on the icosphere-level-5 mesh (1.47M cells)
    and level 6 (6.14M cells): isolated residual evaluations in FP64 and with the FP32 Gauss-point
    flux, and V-cycles, on a state developed by 200 V-cycles."""
    import torch
    res = {}
    shape = {5: (32, 12), 6: (33, 12)}
    for lev in levels:
        nl, npr = shape[lev]
        m = mg.sphere_shell(level=lev, n_layers=nl, n_prism=npr)
        S = cg.Solver(viscous=1, mu=2e-3, prandtl=0.72)
        t0 = time.perf_counter()
        S.set_mesh(m)
        t_mesh = time.perf_counter() - t0
        S.set_bc(mg.TAG_SPHERE, cg.BC_NOSLIP_ADIABATIC)
        S.set_bc(mg.TAG_FARFIELD, cg.BC_FARFIELD, np.array([1.0, 0.2, 0.0, 0.0, 1.0 / 1.4]))
        t0 = time.perf_counter()
        sizes = S.agglomerate()
        t_agg = time.perf_counter() - t0
        W0, G0 = mg.uniform_state(m.n_cells, vel=(0.2, 0.0, 0.0))
        W = torch.from_numpy(W0).cuda()
        G = torch.from_numpy(G0).cuda()
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
        S.vcycle(W, G, al, 200, 0.0)
        out = {"cells": m.n_cells, "faces": S.n_faces, "gauss_points": S.n_gp, "level_cells": [int(x) for x in sizes],
               "setup_s": {"mesh_and_geometry": t_mesh, "agglomeration": t_agg}}
        for prec, key in ((0, "fp64"), (1, "fp32_flux")):
            S.set_params(precision=prec)
            for _ in range(3):
                S.residual(W, G, al)
            torch.cuda.synchronize()
            S.timing_start()
            t0 = time.perf_counter()
            n_iso = 20
            for _ in range(n_iso):
                S.residual(W, G, al)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / n_iso
            face_ms, face_n = S.timing_stop()
            out[f"residual_evals_per_s_{key}"] = 1.0 / dt
            out[f"face_kernel_ms_{key}"] = face_ms / max(face_n, 1)
        S.set_params(precision=0)
        S.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.vcycle(W, G, al, 20, 0.0)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / 20
        out["vcycle_ms"] = ms
        out["residual_evals_per_s_in_vcycles"] = 2.0 / (ms * 1e-3)
        out["cells_evals_per_s"] = out["residual_evals_per_s_in_vcycles"] * m.n_cells
        res[f"icosphere_level_{lev}"] = out
        log(f"sphere level {lev}: {m.n_cells} cells, residual {1e3 / out['residual_evals_per_s_fp64']:.2f} ms "
            f"(FP32 flux {1e3 / out['residual_evals_per_s_fp32_flux']:.2f} ms), V-cycle {ms:.2f} ms")
        S.close()
        del W, G, al
        torch.cuda.empty_cache()
    return res


def explicit_vs_vcycle(cg, mg, cap):
    """The paper's multigrid comparison (single-level explicit CGKS against the 3-level V-cycle):
    iterations and time to residual drops of 1e-4 ... 1e-10 on the hexahedral channel
    (48 x 16 x 8 = 6,144 cells); the explicit scheme is the same solver with one level."""
    import torch
    m = mg.bump_channel(48, 16, 8, n_prism=0, n_pyr=0)
    res = {"cells": m.n_cells, "mesh": "bump channel 48x16x8, hexahedra only",
           "paper_context": {"iteration_ratio": "1/8 to 1/25 (spheres, M6 wing)", "cpu_time_speedup": "2.67 to 9.54"}}
    for levels, key in ((3, "vcycle"), (1, "explicit")):
        S = cg.Solver(levels=levels)
        S.set_mesh(m)
        prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
        for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
            S.set_bc(tag, cg.BC_FARFIELD, prim)
        for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
            S.set_bc(tag, cg.BC_SLIP)
        S.agglomerate()
        W0, G0 = mg.uniform_state(m.n_cells)
        W = torch.from_numpy(W0).cuda()
        G = torch.from_numpy(G0).cuda()
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, ok = S.vcycle(W, G, al, cap, 1e-10)
        torch.cuda.synchronize()
        dt_c = time.perf_counter() - t0
        hh = h / h[0]
        first = {}
        for lvl in (1e-4, 1e-6, 1e-8, 1e-10):
            idx = np.flatnonzero(hh <= lvl)
            first[f"{lvl:.0e}"] = int(idx[0]) + 1 if len(idx) else None
        res[key] = {"iterations": int(len(h)), "seconds": dt_c, "reached_1e-10": bool(ok),
                    "ms_per_iteration": 1e3 * dt_c / len(h), "iterations_to_drop": first}
        log(f"{key}: {len(h)} iterations {dt_c:.2f}s drop {hh[-1]:.2e}")
        S.close()
    v, e = res["vcycle"], res["explicit"]
    if v["reached_1e-10"] and e["reached_1e-10"]:
        res["iteration_ratio"] = v["iterations"] / e["iterations"]
        res["time_speedup"] = e["seconds"] / v["seconds"]
    return res


def hierarchy_study(cg, mg, max_cycles):
    """Cycle and coarsening variants on the hexahedral channel (48 x 16 x 8 = 6,144 cells): time and
    cycles to a 1e-10 drop for the 3-level V-cycle, the W-cycle, 2/4/5 levels, 2 and 4 agglomeration
    passes, one post-sweep per level, and skewness thresholds delta 0.1 and 0.5."""
    import torch
    m = mg.bump_channel(48, 16, 8, n_prism=0, n_pyr=0)
    variants = [("v3", {}), ("w3", {"cycle_gamma": 2}), ("v2", {"levels": 2}), ("v4", {"levels": 4}),
                ("v5", {"levels": 5}), ("w4", {"levels": 4, "cycle_gamma": 2}), ("passes2", {"passes": 2}),
                ("passes4", {"passes": 4}), ("post1", {"nu_post": [1] * 8}),
                ("skew_delta_0.1", {"skew_delta": 0.1}), ("skew_delta_0.5", {"skew_delta": 0.5})]
    res = {"cells": m.n_cells, "mesh": "bump channel 48x16x8, hexahedra only"}
    for key, kw in variants:
        S = cg.Solver(**kw)
        S.set_mesh(m)
        prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
        for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
            S.set_bc(tag, cg.BC_FARFIELD, prim)
        for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
            S.set_bc(tag, cg.BC_SLIP)
        sizes = S.agglomerate()
        W0, G0 = mg.uniform_state(m.n_cells)
        W = torch.from_numpy(W0).cuda()
        G = torch.from_numpy(G0).cuda()
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, ok = S.vcycle(W, G, al, max_cycles, 1e-10)
        torch.cuda.synchronize()
        dt_c = time.perf_counter() - t0
        res[key] = {"levels": [int(x) for x in sizes], "cycles": int(len(h)), "seconds": dt_c, "reached": bool(ok),
                    "final_drop": float(h[-1] / h[0]), "ms_per_cycle": 1e3 * dt_c / max(len(h), 1)}
        log(f"hierarchy {key}: levels {list(sizes)} {len(h)} cycles {dt_c:.2f}s drop {h[-1] / h[0]:.2e}")
        S.close()
    return res


def adjoint_measurements(cg, mg, S, W, G, al):
    """Linearisation and vector-Jacobian-product timings on the benchmark state, and the
    adjoint gradients of the lower-wall x-force against converged finite differences on a
    small all-hexahedral channel (768 cells)."""
    import torch
    from paper_2402_02075_amd import adjoint as ad
    out = {}
    N = W.shape[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.linearize(W, G, al)
    torch.cuda.synchronize()
    out["linearize_s"] = time.perf_counter() - t0
    g = torch.Generator(device="cuda").manual_seed(1)
    w = [torch.randn(*sh, dtype=torch.float64, device="cuda", generator=g) for sh in ((5, N), (15, N), (N,))]
    S.vjp_residual(*w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        S.vjp_residual(*w)
    torch.cuda.synchronize()
    out["vjp_residual_ms"] = (time.perf_counter() - t0) / 20 * 1e3
    t0 = time.perf_counter()
    r = S.adjoint_solve(mg.TAG_WALL_BOTTOM, max_iter=20, tol=0.0)
    out["adjoint_iteration_ms"] = (time.perf_counter() - t0) / max(r["iterations"], 1) * 1e3
    out["tape_bytes"] = int(8 * (451 * 4 * S.n_faces + 1650 * N))

    # gradient check on a channel that converges to round-off
    def mesh_fn(a):
        return mg.bump_channel(24, 8, 4, n_prism=0, n_pyr=0, amp=a)

    amp, mach, h = 0.05, 0.5, 1e-5
    m = mesh_fn(amp)
    Sc = ad.channel_solver(m, mach)
    t0 = time.perf_counter()
    Wc, Gc, ac, hist, _ = ad.converge(Sc, m, cycles=30000, tol=1e-14)
    t_primal = time.perf_counter() - t0
    t0 = time.perf_counter()
    gr = ad.gradients(mesh_fn, amp, mach, Wc, Gc, ac, max_iter=30000, tol=1e-12)
    t_adj = time.perf_counter() - t0
    fd = {}
    for name, mf, mp in (("Mach", lambda s_: mesh_fn(amp), lambda s_: mach + s_),
                         ("A", lambda s_: mesh_fn(amp + s_), lambda s_: mach)):
        J = []
        for sgn in (1.0, -1.0):
            Sx = ad.channel_solver(mf(sgn * h), mp(sgn * h))
            Wx, Gx, ax = Wc.clone(), Gc.clone(), ac.clone()
            Sx.vcycle(Wx, Gx, ax, 20000, 1e-12)
            J.append(float(Sx.wall_force(Wx, Gx, ax, mg.TAG_WALL_BOTTOM)[0]))
        fd[name] = (J[0] - J[1]) / (2 * h)
    out["gradient_check"] = {
        "workload": "bump channel 24x8x4 hexahedra (768 cells), Mach 0.5, J = lower-wall x-force",
        "primal_cycles": int(len(hist)), "primal_drop": float(hist[-1] / hist[0]), "primal_s": t_primal,
        "adjoint_iterations": int(gr["adjoint_iterations"]), "adjoint_s": t_adj,
        "dJ_dMach": {"adjoint": gr["dJ_dMach"], "fd": fd["Mach"],
                     "rel_err": abs(gr["dJ_dMach"] - fd["Mach"]) / abs(fd["Mach"])},
        "dJ_dA": {"adjoint": gr["dJ_dA"], "fd": fd["A"], "rel_err": abs(gr["dJ_dA"] - fd["A"]) / abs(fd["A"])},
        "fd_step": h}
    log(f"adjoint: linearize {out['linearize_s']:.2f}s vjp {out['vjp_residual_ms']:.2f}ms "
        f"iteration {out['adjoint_iteration_ms']:.2f}ms; gradient rel err "
        f"{out['gradient_check']['dJ_dMach']['rel_err']:.2e} {out['gradient_check']['dJ_dA']['rel_err']:.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--develop", type=int, default=100, help="untimed V-cycles that develop the flow first")
    ap.add_argument("--converge", type=int, default=4000, help="max cycles for the time-to-1e-10 runs (0: skip)")
    ap.add_argument("--converge-hex", type=int, default=60000,
                    help="max cycles for the time-to-1e-10 runs on the all-hexahedral channel (0: skip)")
    ap.add_argument("--shock-cycles", type=int, default=8000,
                    help="V-cycles of the Mach 1.2 / 0.95 viscous sphere runs (0: skip)")
    ap.add_argument("--sphere-levels", default="5,6",
                    help="icosphere levels of the viscous-sphere throughput runs (5: 1.47M, 6: 6.14M cells; 0 skips)")
    ap.add_argument("--explicit-cap", type=int, default=200000,
                    help="max iterations of the explicit vs V-cycle comparison on a 6,144-cell channel (0: skip)")
    ap.add_argument("--hierarchy-study", type=int, default=0,
                    help="max cycles of the cycle/coarsening variant study on a 6,144-cell channel (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timings and gradient check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true", help="run a plain 1 GiB copy first (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; sharding the mesh over several GPUs is "
                                   "not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2402_02075_amd import cgks as cg
    from paper_2402_02075_amd import meshgen as mg
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    m, S, sizes, t_mesh, t_agg = build_workload(cg, mg)
    log(f"mesh {m.n_cells} cells {m.counts()} faces {S.n_faces} gp {S.n_gp} levels {sizes} "
        f"setup {t_mesh:.2f}s agglomeration {t_agg:.2f}s")
    N = m.n_cells
    W0, G0 = mg.uniform_state(N)
    W = torch.from_numpy(W0).cuda()
    G = torch.from_numpy(G0).cuda()
    al = torch.ones(N, dtype=torch.float64, device="cuda")
    # develop the flow so that reconstruction and compression-factor branches are realistic
    if args.develop:
        S.vcycle(W, G, al, args.develop, 0.0)
    S.vcycle(W, G, al, args.warmup, 0.0)
    torch.cuda.synchronize()
    evals_per_cycle = max(1, S.params.nu_pre[0]) + (1 if len(sizes) > 1 else 0) + S.params.nu_post[0]
    # timed V-cycles with the face kernel bracketed by events on the library's stream
    S.timing_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, _ = S.vcycle(W, G, al, args.steps, 0.0)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    face_ms, face_n = S.timing_stop()
    ms_per_step = 1e3 * t_steps / args.steps
    value = evals_per_cycle * args.steps / t_steps
    # the same V-cycle with the implicit coarse smoother (not the headline: cost per cycle only)
    S.set_params(coarse_smoother=1)
    Wi, Gi, ai = W.clone(), G.clone(), al.clone()
    S.vcycle(Wi, Gi, ai, 3, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.vcycle(Wi, Gi, ai, 20, 0.0)
    torch.cuda.synchronize()
    ms_implicit = 1e3 * (time.perf_counter() - t0) / 20
    S.set_params(coarse_smoother=0)
    del Wi, Gi, ai
    # isolated residual evaluations
    R = torch.empty(5, N, dtype=torch.float64, device="cuda")
    Gn = torch.empty(15, N, dtype=torch.float64, device="cuda")
    an = torch.empty(N, dtype=torch.float64, device="cuda")
    for _ in range(3):
        S.residual(W, G, al)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_iso = 20
    for _ in range(n_iso):
        S.residual(W, G, al)
    torch.cuda.synchronize()
    iso = n_iso / (time.perf_counter() - t0)
    face_avg_ms = face_ms / max(face_n, 1)
    achieved_tflops = FLOPS_PER_GP * S.n_gp / (face_avg_ms * 1e-3) / 1e12
    out = {
        "metric": "CGKS residual evals/s + time to 1e-10 residual, FP64 vs FP32-mixed, 1 GPU",
        "value": value, "unit": "residual evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3-level V-cycle CGKS, inviscid bump channel, Mach 0.5, seeded mixed mesh",
                   "cells": N, "faces": S.n_faces, "gauss_points": S.n_gp, "level_cells": sizes,
                   "cell_types": m.counts(), "fine_evals_per_step": evals_per_cycle},
        "residual_evals_per_s_isolated": iso,
        "ms_per_step_implicit_coarse_smoother": ms_implicit,
        "cells_evals_per_s": value * N,
        "setup_s": {"mesh_and_geometry": t_mesh, "agglomeration": t_agg},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP64_PEAK_TFLOPS, "traffic": FACE_HBM_BYTES_PER_LAUNCH,
                     "traffic_unit": "bytes per launch",
                     "kernel": "k_face<double, steady> (BGK flux at face Gauss points)",
                     "avg_ms": face_avg_ms, "launches": face_n, "flops_per_gp": FLOPS_PER_GP},
    }
    # time to a 1e-10 drop from the uniform start, FP64 then mixed
    if args.converge:
        for prec, key in ((0, "fp64"), (1, "mixed")):
            S.set_params(precision=prec)
            Wc = torch.from_numpy(W0).cuda()
            Gc = torch.from_numpy(G0).cuda()
            ac = torch.ones(N, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h, ok = S.vcycle(Wc, Gc, ac, args.converge, 1e-10)
            torch.cuda.synchronize()
            dt_c = time.perf_counter() - t0
            out[f"time_to_1e-10_{key}"] = {"seconds": dt_c, "cycles": int(len(h)), "reached": bool(ok),
                                           "final_drop": float(h[-1] / h[0]) if len(h) else None}
            if key == "fp64":
                Wref = Wc.clone()
            else:
                d = (Wc - Wref)[0].abs()
                out["mixed_vs_fp64"] = {"density_max_abs_diff": float(d.max()),
                                        "density_l2_diff": float(torch.sqrt((d * d).mean()))}
            log(f"{key}: {len(h)} cycles {dt_c:.2f}s drop {h[-1] / h[0]:.3e}")
        S.set_params(precision=0)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_measurements(cg, mg, S, W, G, al)
    if args.converge_hex:
        out["time_to_1e-10_hex_channel"] = hex_convergence(cg, mg, args.converge_hex)
    if args.sphere_levels not in ("", "0"):
        out["sphere_throughput"] = sphere_throughput(cg, mg, [int(x) for x in args.sphere_levels.split(",")])
    if args.explicit_cap:
        out["explicit_vs_vcycle"] = explicit_vs_vcycle(cg, mg, args.explicit_cap)
    if args.hierarchy_study:
        out["hierarchy_study"] = hierarchy_study(cg, mg, args.hierarchy_study)
    if args.shock_cycles:
        out["shock_regime_sphere"] = shock_regime(cg, mg, args.shock_cycles)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
