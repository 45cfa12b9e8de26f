"""Internal locality order of the cells (GPU).

The library stores cells by element type and along the Hilbert curve through their centroids,
and moves cell arrays between that order and the caller's at the ABI.  On a mesh whose cells are
listed in a random order:
the residual, gradients and compression factor equal the oracle's (which works in the caller's
order), and equal those of a context that keeps the caller's order to rounding; the exchange in
the internal order (cell_order 2) gives the same values permuted; the hierarchy, which hashes
caller ids (paper Sec. 4.1), equals the oracle's; V-cycles agree with the oracle's.  At full
bump-channel size the V-cycle of the shuffled mesh costs the same as that of the generator's
order (the internal layout is the same).
"""
import time

import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

from gpu_common import assert_residual_close, cell_flux_bound, cell_surface, channel_bcs, flux_scale, say, to_dev

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


@pytest.fixture(scope="module")
def shuffled():
    return mg.permute_cells(mg.bump_channel(16, 8, 4, n_prism=2, n_pyr=3, jitter=0.05, seed=2, amp=0.05), seed=3)


def _solver(cg, m, **kw):
    S = cg.Solver(**kw)
    S.set_mesh(m)
    channel_bcs(S.set_bc, cg.BC_FARFIELD, cg.BC_SLIP)
    return S


def _state(m, seed=4):
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=seed, amp=0.06)
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(15, m.n_cells)) * 0.15
    al = rng.uniform(0.7, 1.0, size=m.n_cells)
    return W, G, al


def test_shuffled_residual_matches_oracle(oracle, cg, torch, shuffled):
    m = shuffled
    say(f"[gpu] shuffled channel {m.n_cells} cells: residual vs oracle")
    S = _solver(cg, m)
    perm = S.cell_order()
    assert sorted(perm.tolist()) == list(range(m.n_cells))
    assert np.any(perm != np.arange(m.n_cells))
    M = oracle.Mesh(m)
    channel_bcs(M.set_bc, oracle.BC_FARFIELD, oracle.BC_SLIP)
    W, G, al = _state(m)
    R, Gn, an = S.residual(to_dev(torch, W), to_dev(torch, G), to_dev(torch, al))
    S.check()
    oR, oGn, oan, _ = M.residual(oracle.params(), W, G, al)
    surf = cell_surface(M.faces(), m.n_cells)
    assert_residual_close(R.cpu().numpy(), oR, cell_flux_bound(W, M.faces(), m.n_cells))
    np.testing.assert_allclose(an.cpu().numpy(), oan, rtol=1e-10)
    vol = M.cells()[0]
    gscale = np.abs(W).max(1).repeat(3)[:, None] * (surf / vol)[None, :]
    assert (np.abs(Gn.cpu().numpy() - oGn) / gscale).max() < 1e-12


def test_orders_agree(cg, torch, shuffled):
    m = shuffled
    W, G, al = _state(m, seed=6)
    out = {}
    for order in (0, 1, 2):
        S = _solver(cg, m, cell_order=order)
        perm = S.cell_order()
        if order == 0:
            np.testing.assert_array_equal(perm, np.arange(m.n_cells))
        ins = [W, G, al] if order < 2 else [W[:, perm], G[:, perm], al[perm]]
        R, Gn, an = S.residual(*[to_dev(torch, np.ascontiguousarray(a)) for a in ins])
        r = [R.cpu().numpy(), Gn.cpu().numpy(), an.cpu().numpy()]
        if order == 2:   # back to the caller's order
            inv = np.empty_like(perm)
            inv[perm] = np.arange(m.n_cells)
            r = [r[0][:, inv], r[1][:, inv], r[2][inv]]
            out["perm1"] = perm
        out[order] = r
        vol = S.geometry()[0].cpu().numpy()
        if order == 2:
            vol = vol[inv]
        out[f"vol{order}"] = vol
    say("[gpu] cell orders 0 / 1 / 2 on the shuffled channel")
    # orders 1 and 2 run identical kernels on identical data: bit-identical
    for a, b in zip(out[1], out[2]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(out["vol1"], out["vol2"])
    # order 0 sums faces in another order: equal to rounding
    fs = flux_scale(W)
    np.testing.assert_allclose(out[1][0], out[0][0], rtol=0, atol=1e-12 * fs.max())
    np.testing.assert_allclose(out[1][2], out[0][2], rtol=1e-12)
    np.testing.assert_allclose(out["vol1"], out["vol0"], rtol=1e-13)


def test_shuffled_hierarchy_and_vcycles_match_oracle(oracle, cg, torch, shuffled):
    m = shuffled
    say(f"[gpu] shuffled channel {m.n_cells} cells: hierarchy and 3 V-cycles vs oracle")
    S = _solver(cg, m)
    sizes = S.agglomerate()
    M = oracle.Mesh(m)
    channel_bcs(M.set_bc, oracle.BC_FARFIELD, oracle.BC_SLIP)
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    for l in (1, 2):
        L = H.level(l)
        assert sizes[l] == L["n"]
        np.testing.assert_array_equal(S.level_map(l).cpu().numpy(), L["f2c"])
    W, G, al = _state(m, seed=8)
    G[:] = 0.0
    al[:] = 1.0
    Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)
    h, _ = S.vcycle(Wd, Gd, ad, 3, 0.0)
    par = oracle.params()
    ho = [H.vcycle(par, W, G, al) for _ in range(3)]
    np.testing.assert_allclose(h, ho, rtol=1e-10)
    scale = np.abs(W).max(1)[:, None]
    assert (np.abs(Wd.cpu().numpy() - W) / scale).max() < 1e-12


def test_shuffled_full_size_costs_the_same(cg, torch):
    """189k-cell bump channel: V-cycle time of the shuffled mesh within 5 % of the generator's order
    (median of 5 batches of 20 queued cycles each, after 40 untimed cycles)."""
    m0 = mg.bump_channel()
    ms = mg.permute_cells(m0, seed=5)
    times = {}
    for key, m in (("ordered", m0), ("shuffled", ms)):
        S = _solver(cg, m)
        S.agglomerate()
        W0, G0 = mg.uniform_state(m.n_cells)
        W, G = to_dev(torch, W0), to_dev(torch, G0)
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
        S.vcycle(W, G, al, 40, 0.0)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.vcycle(W, G, al, 20, 0.0)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) / 20)
        times[key] = float(np.median(ts))
        S.close()
    say(f"[gpu] 189k channel V-cycle: ordered {1e3 * times['ordered']:.3f} ms, "
        f"shuffled {1e3 * times['shuffled']:.3f} ms")
    assert times["shuffled"] < 1.05 * times["ordered"]
