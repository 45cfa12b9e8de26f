"""Writes adjoint_oracle_fd.json: the oracle's own sensitivities of the lower-wall x-force J on a
small converged hexahedral bump channel, by central differences with step 1e-6 of J at converged
perturbed states (the discrete-adjoint check of the library against the oracle).

Mesh: the bump channel generator at 12 x 4 x 2 hexahedra (96 cells), bump amplitude A = 0.05,
inflow Mach M = 0.5 (rho = 1, p = 1/gamma, so c = 1 and u = M), far field at inlet and outlet,
slip walls, 3-level V-cycles (hash seed 1, 3 passes).  Each of the four states (M +- h, A +- h)
is converged by oracle V-cycles from the free stream until the drop of the residual norm stops
improving (its minimum unchanged for 3,000 cycles) or 40,000 cycles.

Calls only the oracle and the seeded input generators.  Run from the repository root:
    python tests/golden/make_adjoint_oracle_fd.py
(four processes; about 15 minutes on 8 cores).
"""
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

DIMS = (12, 4, 2)
AMP, MACH, STEP = 0.05, 0.5, 1e-6
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_oracle_fd.json")


def converged_force(args):
    os.environ["OMP_NUM_THREADS"] = "2"
    import oracle as om
    from paper_2402_02075_amd import meshgen as mg
    amp, mach = args
    m = mg.bump_channel(*DIMS, n_prism=0, n_pyr=0, amp=amp)
    M = om.Mesh(m)
    prim = np.array([1.0, mach, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, om.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, om.BC_SLIP)
    H = om.Hierarchy(M, levels=3, passes=3, seed=1)
    par = om.params()
    W, G = mg.uniform_state(m.n_cells, vel=(mach, 0.0, 0.0))
    al = np.ones(m.n_cells)
    h0 = best = None
    since = 0
    k = 0
    t0 = time.perf_counter()
    while k < 40000 and since < 3000:
        r = H.vcycle(par, W, G, al)
        k += 1
        h0 = r if h0 is None else h0
        if best is None or r < best:
            best, since = r, 0
        else:
            since += 1
    J = float(M.wall_force(par, W, G, al, mg.TAG_WALL_BOTTOM)[0])
    return {"amp": amp, "mach": mach, "cycles": k, "first_norm": h0, "min_norm": best, "last_norm": r,
            "J": J, "seconds": time.perf_counter() - t0}


def main():
    cases = [(AMP, MACH + STEP), (AMP, MACH - STEP), (AMP + STEP, MACH), (AMP - STEP, MACH)]
    with Pool(4) as p:
        res = p.map(converged_force, cases)
    out = {
        "mesh": f"bump channel {DIMS[0]}x{DIMS[1]}x{DIMS[2]} hexahedra, A = {AMP}, M = {MACH}",
        "step": STEP,
        "runs": res,
        "dJ_dMach": (res[0]["J"] - res[1]["J"]) / (2 * STEP),
        "dJ_dA": (res[2]["J"] - res[3]["J"]) / (2 * STEP),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
