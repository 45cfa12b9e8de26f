"""Oracle pins of the multigrid cycle variants (paper Sec. 4.2: pre/post sweeps, levels; the
W-cycle visits each coarser level twice per visit of its parent).

* With two levels, a W-cycle (two visits of level 1, each one sweep, same forcing, continuing
  from the level's state) is the same arithmetic as a V-cycle with two pre-sweeps on level 1:
  the results are bit-identical.
* The free stream is a fixed point of every cycle variant (W-cycle, four levels, post-sweeps,
  implicit coarse smoother).
* The state the V-cycle converges to on a small hexahedral channel (a stored oracle run) is a zero
  of the fine residual, so it is also the fixed point of the single-level explicit scheme: one
  forward-Euler step and one more V-cycle leave it unchanged (the coarse correction of the FAS
  cycle, Sec. 4.2, vanishes with the fine residual).
"""
import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg


def _channel(oracle, nx=12, ny=6, nz=4, amp=0.05):
    m = mg.bump_channel(nx, ny, nz, n_prism=0, n_pyr=0, amp=amp)
    M = oracle.Mesh(m)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, oracle.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, oracle.BC_SLIP)
    return m, M


def test_two_level_w_cycle_equals_v_cycle_with_two_coarse_sweeps(oracle):
    m, M = _channel(oracle)
    H = oracle.Hierarchy(M, levels=2, passes=3, seed=1)
    W0, G0 = mg.smooth_state_and_gradients(mg.cell_node_mean(m), seed=4, amp=0.03)
    out = {}
    for key, par, pre in (("w", oracle.params(cycle_gamma=2), [1, 1]), ("v", oracle.params(), [1, 2])):
        W, G, al = W0.copy(), G0.copy(), np.ones(m.n_cells)
        for _ in range(2):
            H.vcycle(par, W, G, al, nu_pre=pre + [1] * 6, nu_post=[0] * 8)
        out[key] = W
    np.testing.assert_array_equal(out["w"], out["v"])
    # and it is not the V-cycle with one coarse sweep
    W, G, al = W0.copy(), G0.copy(), np.ones(m.n_cells)
    for _ in range(2):
        H.vcycle(oracle.params(), W, G, al)
    assert np.abs(W - out["v"]).max() > 1e-8


@pytest.mark.parametrize("variant", ["w3", "levels4", "post", "implicit_w"])
def test_free_stream_is_a_fixed_point_of_every_cycle(oracle, variant):
    m, M = _channel(oracle, amp=0.0)  # flat walls: the uniform flow satisfies the slip condition
    levels = 4 if variant == "levels4" else 3
    H = oracle.Hierarchy(M, levels=levels, passes=2, seed=1)
    par = oracle.params(cycle_gamma=2 if variant in ("w3", "implicit_w") else 1,
                        coarse_smoother=1 if variant == "implicit_w" else 0)
    post = [1] * 8 if variant == "post" else [0] * 8
    W, G = mg.uniform_state(m.n_cells)
    al = np.ones(m.n_cells)
    W0 = W.copy()
    H.vcycle(par, W, G, al, nu_pre=[1] * 8, nu_post=post)
    np.testing.assert_allclose(W, W0, rtol=0, atol=1e-13)


def test_converged_vcycle_state_is_the_explicit_fixed_point(oracle):
    """The oracle V-cycle's converged state on the 12 x 4 x 2 hexahedral channel
    (tests/golden/vcycle_fixed_point.json, written by make_vcycle_fixed_point.py from oracle calls
    only) has a fine residual at round-off, and neither an explicit step nor a V-cycle moves it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "vcycle_fixed_point.json")) as f:
        gold = json.load(f)
    assert gold["min_norm"] / gold["first_norm"] < 1e-12
    m, M = _channel(oracle, 12, 4, 2)
    W, G, al = (np.array(gold[k], dtype=np.float64) for k in ("W", "G", "alpha"))
    par = oracle.params()
    # the fine residual at the converged state, against its size at the free stream
    W0, G0 = mg.uniform_state(m.n_cells)
    r0 = M.residual_norm(M.residual(par, W0, G0, np.ones(m.n_cells))[0])
    r = M.residual_norm(M.residual(par, W, G, al)[0])
    assert r0 > 0.0 and r / r0 < 1e-12, (r, r0)
    scale = np.abs(W).max(axis=1, keepdims=True)
    We, Ge, ae = W.copy(), G.copy(), al.copy()
    M.step_fe(par, We, Ge, ae)  # single-level explicit step
    assert (np.abs(We - W) / scale).max() < 1e-13
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    Wv, Gv, av = W.copy(), G.copy(), al.copy()
    H.vcycle(par, Wv, Gv, av)
    assert (np.abs(Wv - W) / scale).max() < 1e-13
