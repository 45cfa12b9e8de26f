"""GPU parity of the implicit coarse smoother (paper Sec. 4.3) against the oracle.

* ``cgks_coarse_implicit`` on both coarse levels of a mixed channel, at 0, 2 and 5
  relaxation sweeps, with a right-hand side large enough that the flux differences are
  nonlinear: FP64 within 1e-12 in units of the state it increments (1e-10 of the increment
  itself), FP32 within 1e-5 of the state.
* V-cycles with the implicit coarse smoother against the oracle's cycles.
* On the hexahedral channel the implicit-smoother cycle converges to the fixed point of the
  forward-Euler cycle (the coarse correction is proportional to the fine residual).
"""
import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

from gpu_common import say, to_dev

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


@pytest.fixture(scope="module")
def hier(oracle, cg, torch):
    m = mg.bump_channel(24, 12, 6, n_prism=2, n_pyr=3, jitter=0.05, seed=1, amp=0.05)
    say(f"[gpu] implicit smoother hierarchy cells={m.n_cells}")
    M = oracle.Mesh(m)
    S = cg.Solver()
    S.set_mesh(m)
    for tag, kind, prim in _bcs():
        M.set_bc(tag, kind, prim)
        S.set_bc(tag, kind, prim)
    sizes = S.agglomerate()
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    return m, M, S, H, sizes


@pytest.mark.parametrize("sweeps", [0, 2, 5])
def test_implicit_increment_matches_oracle(oracle, torch, hier, sweeps):
    m, M, S, H, sizes = hier
    W = mg.random_smooth_state(mg.cell_node_mean(m), seed=31, amp=0.08)
    Wd = to_dev(torch, W)
    Wo = W
    rng = np.random.default_rng(32)
    for l in (1, 2):
        Wd, _ = S.restrict(l, Wd, torch.zeros_like(Wd))
        Wo, _ = H.restrict(l, Wo, np.zeros_like(Wo))
        n = sizes[l]
        mom = np.abs(Wo[1:4]).max()
        wscale = np.array([np.abs(Wo[0]).max(), mom, mom, mom, np.abs(Wo[4]).max()])[:, None]
        # right-hand side sized so that the first iterate rhs/D is about 1e-3 of the state:
        # D_i from the oracle's diagonal-only increment of a unit right-hand side
        par0 = oracle.params(coarse_smoother=1, relax_sweeps=0, cfl_implicit=2.0)
        D = 1.0 / H.coarse_implicit(par0, l, Wo, np.ones((5, n)))[0]
        rhs = 1e-3 * rng.standard_normal((5, n)) * wscale * D[None, :]
        say(f"[gpu] implicit level {l} n={n} sweeps={sweeps}")
        out = {}
        for prec in (0, 1):
            S.set_params(coarse_smoother=1, relax_sweeps=sweeps, cfl_implicit=2.0, precision=prec)
            out[prec] = S.coarse_implicit(l, Wd, to_dev(torch, rhs)).cpu().numpy()
        S.set_params(coarse_smoother=0, precision=0)
        ref = H.coarse_implicit(oracle.params(coarse_smoother=1, relax_sweeps=sweeps, cfl_implicit=2.0), l, Wo, rhs)
        # The increment updates the state: it is compared in units of the state (density, one scale
        # for the momentum vector, energy), as the V-cycle's states are.  Relative to the increment
        # itself the error is larger: each sweep forms F(U + dU) - F(U), whose rounding is of order
        # eps |F|, and the right-hand side and the neighbour terms largely cancel.
        iscale = np.abs(ref).max(axis=1, keepdims=True)
        e64 = (np.abs(out[0] - ref) / wscale).max(axis=1)
        e32 = (np.abs(out[1] - ref) / wscale).max(axis=1)
        i64 = (np.abs(out[0] - ref) / iscale).max(axis=1)
        say("    vs state: FP64 " + " ".join(f"{e:.1e}" for e in e64) + " | FP32 " + " ".join(f"{e:.1e}" for e in e32)
            + " ; FP64 vs increment " + " ".join(f"{e:.1e}" for e in i64))
        assert e64.max() < 1e-12
        assert i64.max() < 1e-10
        assert e32.max() < 1e-5


def test_implicit_vcycle_matches_oracle(oracle, torch, hier):
    m, M, S, H, sizes = hier
    S.set_params(coarse_smoother=1, relax_sweeps=2, cfl_implicit=2.0)
    try:
        par = oracle.params(coarse_smoother=1, relax_sweeps=2, cfl_implicit=2.0)
        W, G = mg.uniform_state(m.n_cells)
        al = np.ones(m.n_cells)
        Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)
        say("[gpu] implicit-smoother vcycle x3")
        hist, _ = S.vcycle(Wd, Gd, ad, 3, 1e-30)
        ohist = [H.vcycle(par, W, G, al) for _ in range(3)]
        np.testing.assert_allclose(hist, ohist, rtol=1e-10)
        mom = np.abs(W[1:4]).max()
        scale = np.array([np.abs(W[0]).max(), mom, mom, mom, np.abs(W[4]).max()])[:, None]
        np.testing.assert_allclose(Wd.cpu().numpy() / scale, W / scale, rtol=0, atol=1e-12)
    finally:
        S.set_params(coarse_smoother=0)


def test_implicit_vcycle_reaches_explicit_fixed_point(cg, torch):
    from paper_2402_02075_amd import adjoint as ad
    m = mg.bump_channel(16, 6, 4, n_prism=0, n_pyr=0)
    say(f"[gpu] implicit vs explicit fixed point cells={m.n_cells}")
    out = {}
    for smoother in (0, 1):
        S = ad.channel_solver(m, 0.5, coarse_smoother=smoother, relax_sweeps=2, cfl_implicit=2.0)
        W, G, al, hist, ok = ad.converge(S, m, cycles=30000, tol=1e-12)
        say(f"    coarse smoother {smoother}: {len(hist)} cycles, drop {hist[-1] / hist[0]:.2e}")
        assert ok
        out[smoother] = W.cpu().numpy()
    d = np.abs(out[1] - out[0]).max(axis=1) / np.abs(out[0]).max(axis=1)
    say("    implicit vs explicit converged state, max rel difference: " + " ".join(f"{x:.1e}" for x in d))
    assert d.max() < 1e-9
