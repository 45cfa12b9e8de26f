"""GPU parity of the multigrid cycle variants against the oracle (mixed bump channel, FP64):
W-cycle (each coarser level visited twice per parent visit), four levels, post-sweeps on every
level.  Three cycles from the free stream; residual histories within 1e-10 and states within
1e-12 of each conserved quantity's magnitude, as for the V-cycle."""
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
def mesh():
    return mg.bump_channel(24, 12, 6, n_prism=2, n_pyr=3, jitter=0.05, seed=1, amp=0.05)


@pytest.mark.parametrize("variant", ["w_cycle", "four_levels", "post_sweeps", "w_implicit"])
def test_cycle_variant_matches_oracle(oracle, cg, torch, mesh, variant):
    m = mesh
    levels = 4 if variant == "four_levels" else 3
    gamma = 2 if variant in ("w_cycle", "w_implicit") else 1
    smoother = 1 if variant == "w_implicit" else 0
    post = [1] * 8 if variant == "post_sweeps" else [0] * 8
    say(f"[gpu] cycle variant {variant} cells={m.n_cells}")
    M = oracle.Mesh(m)
    S = cg.Solver(levels=levels, cycle_gamma=gamma, coarse_smoother=smoother, nu_post=post)
    S.set_mesh(m)
    for tag, kind, prim in _bcs():
        M.set_bc(tag, kind, prim)
        S.set_bc(tag, kind, prim)
    sizes = S.agglomerate()
    H = oracle.Hierarchy(M, levels=levels, passes=3, seed=1)
    assert list(sizes) == [H.size(l)[0] for l in range(levels)]
    par = oracle.params(cycle_gamma=gamma, coarse_smoother=smoother)
    W, G = mg.uniform_state(m.n_cells)
    al = np.ones(m.n_cells)
    Wd, Gd, ad = to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)
    hist, _ = S.vcycle(Wd, Gd, ad, 3, 1e-30)
    ohist = [H.vcycle(par, W, G, al, nu_pre=[1] * 8, nu_post=post) for _ in range(3)]
    np.testing.assert_allclose(hist, ohist, rtol=1e-10)
    mom = np.abs(W[1:4]).max()
    scale = np.array([np.abs(W[0]).max(), mom, mom, mom, np.abs(W[4]).max()])[:, None]
    err = np.abs(Wd.cpu().numpy() - W) / scale
    say(f"    levels {list(sizes)}; max state error per quantity " + " ".join(f"{e:.1e}" for e in err.max(axis=1)))
    assert err.max() < 1e-12
    np.testing.assert_allclose(ad.cpu().numpy(), al, rtol=1e-9)


def test_cycle_parameters_and_implicit_entry_point_errors(cg, torch, mesh):
    """Out-of-range cycle parameters and coarse levels are rejected with an error, not run."""
    S = cg.Solver()
    with pytest.raises(cg.CgksError):
        S.set_params(cycle_gamma=4)
    with pytest.raises(cg.CgksError):
        S.set_params(coarse_smoother=2)
    with pytest.raises(cg.CgksError):
        S.set_params(relax_sweeps=65)
    with pytest.raises(cg.CgksError):
        S.set_params(coarse_smoother=1, cfl_implicit=0.0)
    S.set_params(coarse_smoother=0, cfl_implicit=0.25, relax_sweeps=2, cycle_gamma=1)
    S.set_mesh(mesh)
    for tag, kind, prim in _bcs():
        S.set_bc(tag, kind, prim)
    sizes = S.agglomerate()
    W = to_dev(torch, mg.uniform_state(mesh.n_cells)[0])
    Wc, _ = S.restrict(1, W, torch.zeros_like(W))
    with pytest.raises(cg.CgksError):
        S.coarse_implicit(len(sizes), Wc, Wc)  # no such level
    with pytest.raises(cg.CgksError):
        S.coarse_implicit(0, W, W)  # the fine level has no coarse smoother
    # zero right-hand side: zero increment up to rounding (the flux differences F(U + 0) - F(U) are
    # formed with fused multiply-adds, so they need not cancel to the last bit)
    dU = S.coarse_implicit(1, Wc, torch.zeros_like(Wc))
    assert float(dU.abs().max()) < 1e-15
