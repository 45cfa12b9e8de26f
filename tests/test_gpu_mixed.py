"""Mixed precision: FP32 flux evaluation and FP32 coarse levels, errors against the FP64 oracle.

* The fine residual with Gauss-point fluxes evaluated in FP32 (sums and outputs FP64)
  against the FP64 oracle: the error is stated in units of the cell's flux scale.
* The coarse KFVS operator in FP32 against the FP64 oracle, likewise.
* The mixed V-cycle (FP32 coarse levels, transfers and flux until the switch, then FP64
  flux) converges to the same discrete fixed point as the FP64 cycle: the coarse
  correction is proportional to the fine residual (delta form), so its FP32 rounding
  vanishes at convergence.
"""
import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

from gpu_common import assert_residual_close, cell_flux_bound, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ad(torch):
    from paper_2402_02075_amd import adjoint
    return adjoint


def _oracle_channel(oracle, m):
    M = oracle.Mesh(m)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, oracle.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, oracle.BC_SLIP)
    return M


MESH = lambda: mg.bump_channel(16, 10, 4, n_prism=2, n_pyr=3, jitter=0.08, seed=5, amp=0.05)


def test_fp32_flux_residual_error(oracle, torch, ad):
    m = MESH()
    say(f"[gpu] mixed fp32 flux residual cells={m.n_cells}")
    S = ad.channel_solver(m, 0.5, agglomerate=False)
    M = _oracle_channel(oracle, m)
    W, G = mg.smooth_state_and_gradients(mg.cell_node_mean(m), seed=21, amp=0.05)
    al = np.random.default_rng(21).uniform(0.6, 1.0, size=m.n_cells)
    Ro, Go, ao, _ = M.residual(oracle.params(), W, G, al)
    dev = [torch.from_numpy(a).cuda() for a in (W, G, al)]
    S.set_params(precision=1)
    R, Gn, an = (t.cpu().numpy() for t in S.residual(*dev))
    S.set_params(precision=0)
    R64 = S.residual(*dev)[0].cpu().numpy()
    bnd = cell_flux_bound(W, M.faces(), m.n_cells)
    ratio32 = assert_residual_close(R, Ro, bnd, tol=1e-5, what="R fp32")
    ratio64 = assert_residual_close(R64, Ro, bnd, tol=1e-12, what="R fp64")
    rel_alpha = float(np.abs(an - ao).max())
    say(f"    FP32 flux: max |R - R_oracle| / (sum_f S_f |F_f|) = {ratio32 * 1e-5:.2e} (FP64 path: {ratio64 * 1e-12:.2e}); "
        f"alpha max abs err {rel_alpha:.2e}")
    assert rel_alpha < 1e-5


def test_fp32_kfvs_error(oracle, torch, ad):
    """Each side restricts the same seeded fine state with its own restriction (the
    agglomerations are bit-identical), then the FP32 KFVS is compared with the FP64 oracle."""
    m = MESH()
    say(f"[gpu] mixed fp32 kfvs cells={m.n_cells}")
    S = ad.channel_solver(m, 0.5)
    M = _oracle_channel(oracle, m)
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    W = mg.random_smooth_state(mg.cell_node_mean(m), seed=22, amp=0.05)
    par = oracle.params()
    Wl, Wo = torch.from_numpy(W).cuda(), W
    for lev in (1, 2):
        Wl, _ = S.restrict(lev, Wl, torch.zeros_like(Wl))
        Wo, _ = H.restrict(lev, Wo, np.zeros_like(Wo))
        Ro = H.kfvs_residual(par, lev, Wo)
        S.set_params(precision=1)
        R32 = S.kfvs_residual(lev, Wl).cpu().numpy()
        S.set_params(precision=0)
        R64 = S.kfvs_residual(lev, Wl).cpu().numpy()
        den = np.abs(Ro).max(axis=1)
        err32 = np.abs(R32 - Ro).max(axis=1) / den
        err64 = np.abs(R64 - Ro).max(axis=1) / den
        say(f"    level {lev}: max |R - R_oracle| / max |R_oracle| per component, FP32 "
            + " ".join(f"{e:.2e}" for e in err32) + " | FP64 " + " ".join(f"{e:.2e}" for e in err64))
        assert err32.max() < 1e-5
        assert err64.max() < 1e-12


def test_mixed_vcycle_reaches_fp64_fixed_point(torch, ad):
    m = mg.bump_channel(24, 8, 4, n_prism=0, n_pyr=0)
    say(f"[gpu] mixed vcycle fixed point cells={m.n_cells}")
    out = {}
    for prec in (0, 1):
        S = ad.channel_solver(m, 0.5, precision=prec)
        W, G, al, hist, ok = ad.converge(S, m, cycles=30000, tol=1e-12)
        say(f"    precision {prec}: {len(hist)} cycles, drop {hist[-1] / hist[0]:.2e}")
        assert ok
        out[prec] = (W.cpu().numpy(), len(hist))
    d = np.abs(out[1][0] - out[0][0]).max(axis=1) / np.abs(out[0][0]).max(axis=1)
    say("    mixed vs FP64 converged state, max rel difference per component: " + " ".join(f"{x:.2e}" for x in d))
    assert d.max() < 1e-9


def test_mixed_switch_inside_a_batch(torch, ad):
    """The switch from the FP32 to the FP64 flux decided at a cycle inside a batch of queued
    cycles: the run must equal one that stops the mixed cycle after that cycle and continues in
    FP64 (same states bit for bit, same norms)."""
    m = mg.bump_channel(24, 8, 4, n_prism=0, n_pyr=0)
    W0, G0 = mg.uniform_state(m.n_cells)
    al0 = np.ones(m.n_cells)

    def dev():
        return (torch.from_numpy(W0.copy()).cuda(), torch.from_numpy(G0.copy()).cuda(),
                torch.from_numpy(al0.copy()).cuda())

    n = 40
    S = ad.channel_solver(m, 0.5, precision=1, mixed_switch=0.0)
    h, _ = S.vcycle(*dev(), n, 1e-300)
    drop = h / h[0]
    x = drop[9]
    s = int(np.nonzero(drop <= x)[0][0])
    say(f"[gpu] mixed switch inside a batch at cycle {s}")
    assert 0 < s < 15
    SA = ad.channel_solver(m, 0.5, precision=1, mixed_switch=x)
    WA, GA, aA = dev()
    hA, _ = SA.vcycle(WA, GA, aA, n, 1e-300)
    SB = ad.channel_solver(m, 0.5, precision=1, mixed_switch=0.0)
    WB, GB, aB = dev()
    hB1, _ = SB.vcycle(WB, GB, aB, s + 1, 1e-300)
    SB.set_params(precision=0)
    hB2, _ = SB.vcycle(WB, GB, aB, n - s - 1, 1e-300)
    np.testing.assert_array_equal(hA, np.concatenate([hB1, hB2]))
    for a, b in ((WA, WB), (GA, GB), (aA, aB)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_mixed_switch_by_the_stall_window(torch, ad):
    """The switch to the FP64 flux after `mixed_stall` cycles without a new minimum of the residual
    norm, decided inside a batch of queued cycles: the run equals one that stops the mixed cycle
    at that cycle and continues in FP64 (states bit for bit, same norms).  The switch cycle is read
    off the mixed run's own history (the first k with k - argmin(h[:k+1]) = mixed_stall)."""
    m = mg.bump_channel(24, 8, 4, n_prism=2, n_pyr=2, jitter=0.05, seed=3)
    W0, G0 = mg.uniform_state(m.n_cells)
    al0 = np.ones(m.n_cells)

    def dev():
        return (torch.from_numpy(W0.copy()).cuda(), torch.from_numpy(G0.copy()).cuda(),
                torch.from_numpy(al0.copy()).cuda())

    n, stall = 300, 5
    SA = ad.channel_solver(m, 0.5, precision=1, mixed_switch=0.0, mixed_stall=stall)
    WA, GA, aA = dev()
    hA, _ = SA.vcycle(WA, GA, aA, n, 1e-300)
    # the first cycle k at which the mixed run has gone `stall` cycles without a new minimum
    best, best_at, s = np.inf, 0, None
    for k, r in enumerate(hA):
        if r < best:
            best, best_at = r, k
        if k - best_at >= stall:
            s = k
            break
    say(f"[gpu] mixed switch by the stall window at cycle {s}")
    assert s is not None and 0 < s < n - 1
    SB = ad.channel_solver(m, 0.5, precision=1, mixed_switch=0.0, mixed_stall=10 ** 6)
    WB, GB, aB = dev()
    hB1, _ = SB.vcycle(WB, GB, aB, s + 1, 1e-300)
    SB.set_params(precision=0)
    hB2, _ = SB.vcycle(WB, GB, aB, n - s - 1, 1e-300)
    np.testing.assert_array_equal(hA, np.concatenate([hB1, hB2]))
    for a, b in ((WA, WB), (GA, GB), (aA, aB)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
