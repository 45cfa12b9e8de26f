"""Writes vcycle_fixed_point.json: the state the oracle's 3-level V-cycle converges to on the
12 x 4 x 2 hexahedral bump channel (96 cells, bump amplitude 0.05, inflow Mach 0.5, far field at
inlet and outlet, slip walls, hash seed 1, 3 passes), from the free stream until the residual norm
stops improving (its minimum unchanged for 3,000 cycles) or 40,000 cycles.

Calls only the oracle and the seeded input generators.  Run from the repository root:
    python tests/golden/make_vcycle_fixed_point.py
(about 20 minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "vcycle_fixed_point.json")


def main():
    import oracle as om
    from paper_2402_02075_amd import meshgen as mg
    m = mg.bump_channel(12, 4, 2, n_prism=0, n_pyr=0, amp=0.05)
    M = om.Mesh(m)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, om.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, om.BC_SLIP)
    H = om.Hierarchy(M, levels=3, passes=3, seed=1)
    par = om.params()
    W, G = mg.uniform_state(m.n_cells)
    al = np.ones(m.n_cells)
    hist = []
    best, since = None, 0
    t0 = time.perf_counter()
    while len(hist) < 40000 and since < 3000:
        r = H.vcycle(par, W, G, al)
        hist.append(r)
        if best is None or r < best:
            best, since = r, 0
        else:
            since += 1
        if len(hist) % 2000 == 0:
            print(f"{len(hist)} cycles, drop {r / hist[0]:.3e}, {time.perf_counter() - t0:.0f} s", flush=True)
    out = {"mesh": "bump channel 12x4x2 hexahedra, A = 0.05, M = 0.5", "cycles": len(hist),
           "first_norm": hist[0], "min_norm": best, "last_norm": hist[-1],
           "W": W.tolist(), "G": G.tolist(), "alpha": al.tolist()}
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"{len(hist)} cycles, minimum drop {best / hist[0]:.3e}")


if __name__ == "__main__":
    main()
