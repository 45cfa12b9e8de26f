"""GPU parity of agglomeration, coarse KFVS, transfers and the V-cycle.

Agglomeration is integer work decided by a floating-point predicate: given
identical graph arrays (the oracle's geometry fed to both sides) the coarse map,
coarse volumes and first moments must be bit-identical, at small and at full
bump-channel size.  Coarse operators and the V-cycle are FP64 and compared
with the residual bound of the fine tests.
"""
import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

from gpu_common import assert_residual_close, flux_scale, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def cg(torch):
    from paper_2402_02075_amd import cgks
    return cgks


def _bcs():
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    out = [(mg.TAG_INLET, 3, prim), (mg.TAG_OUTLET, 3, prim)]
    for t in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        out.append((t, 1, None))
    return out


def _pair(oracle, cg, m, **par):
    M = oracle.Mesh(m)
    S = cg.Solver(**par)
    S.set_mesh(m)
    for tag, kind, prim in _bcs():
        M.set_bc(tag, kind, prim)
        S.set_bc(tag, kind, prim)
    return M, S


def _oracle_graph(oracle, M):
    vol, cen, _ = M.cells()
    F = M.faces()
    sel = (F["fr"] >= 0) & np.all(F["shift"] == 0, axis=1)
    return oracle.Graph(vol, vol[:, None] * cen, F["fl"][sel], F["fr"][sel], F["area"][sel], F["fmom"][sel],
                        F["avec"][sel])


@pytest.mark.parametrize("size", ["small", "full"])
def test_agglomeration_bit_exact(oracle, cg, torch, size):
    m = mg.bump_channel(24, 12, 6, n_prism=2, n_pyr=3, jitter=0.05, seed=1) if size == "small" else mg.bump_channel()
    say(f"[gpu] agglomerate_graph {size} cells={m.n_cells}")
    M = oracle.Mesh(m)
    g = _oracle_graph(oracle, M)
    S = cg.Solver()
    for passes in (1, 3):
        f2c_o, cg_o, st_o = oracle.agglomerate_graph(g, seed=1, passes=passes)
        dev = lambda a, dt=np.float64: to_dev(torch, np.ascontiguousarray(a, dtype=dt))
        f2c, Vc, Pc, nc, mc, st = S.agglomerate_graph(dev(g.V), dev(g.P), dev(g.a, np.int32), dev(g.b, np.int32),
                                                      dev(g.S), dev(g.M), dev(g.A), passes)
        assert nc == len(cg_o.V) and mc == len(cg_o.a)
        np.testing.assert_array_equal(f2c.cpu().numpy(), f2c_o)
        np.testing.assert_array_equal(Vc.cpu().numpy(), cg_o.V)   # bit-identical sums
        np.testing.assert_array_equal(Pc.cpu().numpy(), cg_o.P)
        np.testing.assert_array_equal(st, st_o[:passes])


def test_agglomeration_other_seed_and_determinism(oracle, cg, torch):
    m = mg.bump_channel(20, 10, 6, n_prism=2, n_pyr=3, jitter=0.05, seed=4)
    M = oracle.Mesh(m)
    g = _oracle_graph(oracle, M)
    S = cg.Solver(seed=7)
    dev = lambda a, dt=np.float64: to_dev(torch, np.ascontiguousarray(a, dtype=dt))
    args = (dev(g.V), dev(g.P), dev(g.a, np.int32), dev(g.b, np.int32), dev(g.S), dev(g.M), dev(g.A), 3)
    say("[gpu] agglomerate seed 7 twice")
    a = S.agglomerate_graph(*args)[0].cpu().numpy()
    b = S.agglomerate_graph(*args)[0].cpu().numpy()
    np.testing.assert_array_equal(a, b)
    f2c_o, _, _ = oracle.agglomerate_graph(g, seed=7, passes=3)
    np.testing.assert_array_equal(a, f2c_o)


@pytest.fixture(scope="module")
def hier(oracle, cg, torch):
    m = mg.bump_channel(24, 12, 6, n_prism=2, n_pyr=3, jitter=0.05, seed=1, amp=0.05)
    say(f"[gpu] hierarchy cells={m.n_cells}")
    M, S = _pair(oracle, cg, m)
    sizes = S.agglomerate()
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    return m, M, S, H, sizes


def test_hierarchy_maps_match_oracle(hier):
    m, M, S, H, sizes = hier
    for l in (1, 2):
        L = H.level(l)
        assert sizes[l] == L["n"]
        np.testing.assert_array_equal(S.level_map(l).cpu().numpy(), L["f2c"])


def test_kfvs_restrict_prolong(oracle, torch, hier):
    m, M, S, H, sizes = hier
    par = oracle.params()
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=9, amp=0.08)
    rng = np.random.default_rng(2)
    R = rng.normal(size=W.shape) * 1e-3
    Wd, Rd = to_dev(torch, W), to_dev(torch, R)
    for l in (1, 2):
        if l == 1:
            Wf, Rf, Wfd, Rfd = W, R, Wd, Rd
        Wc, Rc = S.restrict(l, Wfd, Rfd)
        oWc, oRc = H.restrict(l, Wf, Rf)
        np.testing.assert_allclose(Wc.cpu().numpy(), oWc, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(Rc.cpu().numpy(), oRc, rtol=1e-13, atol=1e-17)
        Rk = S.kfvs_residual(l, Wc).cpu().numpy()
        oRk = H.kfvs_residual(par, l, oWc)
        Lv = H.level(l)
        surf = np.zeros(Lv["n"])
        nA = np.linalg.norm(Lv["A"], axis=1)
        np.add.at(surf, Lv["a"], nA)
        np.add.at(surf, Lv["b"], nA)
        surf += 1.0  # boundary faces
        assert_residual_close(Rk, oRk, surf, flux_scale(oWc), what=f"kfvs level {l}")
        dW = rng.normal(size=oWc.shape) * 1e-4
        Wp = Wfd.clone()
        S.prolong(l, to_dev(torch, dW), Wp)
        np.testing.assert_allclose(Wp.cpu().numpy(), H.prolong(l, dW, Wfd.cpu().numpy()), rtol=0, atol=0)
        Wf, Rf, Wfd, Rfd = oWc, oRc, Wc, Rc


def test_vcycle_matches_oracle(oracle, torch, hier):
    m, M, S, H, sizes = hier
    par = oracle.params()
    W, G = mg.uniform_state(m.n_cells)
    al = np.ones(m.n_cells)
    Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)
    say("[gpu] vcycle x3")
    hist, conv = S.vcycle(Wd, Gd, ad, 3, 1e-30)
    ohist = [H.vcycle(par, W, G, al) for _ in range(3)]
    np.testing.assert_allclose(hist, ohist, rtol=1e-10)
    # 1e-12 relative to the magnitude of each conserved quantity: density, the momentum vector
    # (one scale for its three components: the transverse ones are near zero), energy (about 2.3)
    mom = np.abs(W[1:4]).max()
    scale = np.array([np.abs(W[0]).max(), mom, mom, mom, np.abs(W[4]).max()])[:, None]
    np.testing.assert_allclose(Wd.cpu().numpy() / scale, W / scale, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ad.cpu().numpy(), al, rtol=1e-9)


def test_vcycle_queued_equals_checked(oracle, torch, hier):
    """Without a tolerance the cycles are queued with their norms kept on the device: the state
    and the history must be those of the loop that reads every norm, and the oracle's."""
    m, M, S, H, sizes = hier
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=21, amp=0.05)
    G = np.zeros((15, m.n_cells))
    al = np.ones(m.n_cells)
    out = {}
    for tol in (1e-300, 0.0):
        Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)
        say(f"[gpu] vcycle x4 tol={tol}")
        hist, conv = S.vcycle(Wd, Gd, ad, 4, tol)
        assert not conv and len(hist) == 4
        out[tol] = (hist, Wd.cpu().numpy(), Gd.cpu().numpy(), ad.cpu().numpy())
    for a, b in zip(out[1e-300], out[0.0]):
        np.testing.assert_array_equal(a, b)
    par = oracle.params()
    Wo, Go, ao = W.copy(), G.copy(), al.copy()
    ohist = [H.vcycle(par, Wo, Go, ao) for _ in range(4)]
    np.testing.assert_allclose(out[0.0][0], ohist, rtol=1e-10)


def test_vcycle_stop_inside_a_batch(torch, hier):
    """A tolerance reached in the middle of a batch of queued cycles: the call must stop after
    exactly that cycle, with the state of a run of that many cycles."""
    m, M, S, H, sizes = hier
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=22, amp=0.05)
    G = np.zeros((15, m.n_cells))
    al = np.ones(m.n_cells)

    def run(n, tol):
        Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)
        hist, conv = S.vcycle(Wd, Gd, ad, n, tol)
        return hist, conv, Wd.cpu().numpy(), Gd.cpu().numpy(), ad.cpu().numpy()

    full = run(40, 0.0)[0]
    drop = full / full[0]
    tol = drop[21]
    k_stop = int(np.nonzero(drop <= tol)[0][0])
    say(f"[gpu] stop inside a batch at cycle {k_stop}")
    assert k_stop > 0 and k_stop % 16 != 15  # not the last cycle of a batch of 16
    hist, conv, Ws, Gs, As = run(40, tol)
    assert conv and len(hist) == k_stop + 1
    np.testing.assert_array_equal(hist, full[:k_stop + 1])
    _, _, Wr, Gr, Ar = run(k_stop + 1, 0.0)
    np.testing.assert_array_equal(Ws, Wr)
    np.testing.assert_array_equal(Gs, Gr)
    np.testing.assert_array_equal(As, Ar)


def test_vcycle_converges_faster_than_explicit(cg, torch, hier):
    m, M, S, H, sizes = hier
    W, G = mg.uniform_state(m.n_cells)
    res = {}
    for mode in ("explicit", "vcycle"):
        Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, np.ones(m.n_cells))
        if mode == "vcycle":
            hist, _ = S.vcycle(Wd, Gd, ad, 60, 1e-30)
        else:
            rn = S.empty(1)
            hist = []
            for _ in range(60):
                S.step(Wd, Gd, ad, -1.0, rn)
                hist.append(rn.item())
        res[mode] = hist[-1] / hist[0]
    say(f"[gpu] drop after 60: {res}")
    assert res["vcycle"] < res["explicit"]


def test_converged_state_equals_the_oracle_fixed_point(cg, torch):
    """On the 12 x 4 x 2 hexahedral channel the library's V-cycle, run from the free stream to a
    1e-14 drop, ends at the state the oracle's V-cycle converged to (a stored oracle run,
    tests/golden/vcycle_fixed_point.json), within 1e-11 of each component's size: the two solve
    the same discrete equations, and the fixed point does not depend on the path to it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "vcycle_fixed_point.json")) as f:
        gold = json.load(f)
    m = mg.bump_channel(12, 4, 2, n_prism=0, n_pyr=0, amp=0.05)
    S = cg.Solver()
    S.set_mesh(m)
    for tag, kind, prim in _bcs():
        S.set_bc(tag, kind, prim)
    S.agglomerate()
    W0, G0 = mg.uniform_state(m.n_cells)
    W, G = to_dev(torch, W0), to_dev(torch, G0)
    al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
    h, ok = S.vcycle(W, G, al, 40000, 1e-14)
    say(f"[gpu] converged state vs oracle fixed point: {len(h)} cycles, drop {h[-1] / h[0]:.2e}")
    assert ok
    Wo = np.array(gold["W"])
    d = np.abs(W.cpu().numpy() - Wo).max(axis=1) / np.abs(Wo).max(axis=1)
    say("    max difference per component: " + " ".join(f"{x:.2e}" for x in d))
    assert d.max() < 1e-11
