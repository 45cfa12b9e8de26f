"""Edge cases and error paths of the library on the GPU: empty, re-oriented and collapsed cells, a boundary
tag without a condition, a non-physical state (reported, then cleared), and a ragged mesh whose
cell count is no multiple of the 64-cell reconstruction groups."""
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


def _channel_bcs(S, cg, skip=()):
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        if tag not in skip:
            S.set_bc(tag, cg.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        if tag not in skip:
            S.set_bc(tag, cg.BC_SLIP)


def test_empty_reoriented_and_collapsed_meshes(cg, torch):
    say("[gpu] edge: empty, re-oriented and collapsed meshes")
    S = cg.Solver()
    m = mg.bump_channel(6, 4, 2, n_prism=0, n_pyr=0)
    with pytest.raises(cg.CgksError) as e:
        S.set_mesh(mg.Mesh(m.xyz, m.ctype[:0], m.cnode_ptr[:1], m.cnode[:0], m.bnode_ptr[:1], m.bnode[:0],
                           m.btag[:0], None))
    assert e.value.code == cg.E_ARG
    S.set_mesh(m)
    vol0 = S.geometry()[0].cpu().numpy()
    # a hexahedron given with the opposite orientation (bottom and top quadrilaterals swapped) is
    # the same cell: the library takes volumes orientation-free
    cnode = m.cnode.copy()
    a = m.cnode_ptr[3]
    cnode[a:a + 8] = m.cnode[a:a + 8][[4, 5, 6, 7, 0, 1, 2, 3]]
    S.set_mesh(mg.Mesh(m.xyz, m.ctype, m.cnode_ptr, cnode, m.bnode_ptr, m.bnode, m.btag, None))
    np.testing.assert_allclose(S.geometry()[0].cpu().numpy(), vol0, rtol=1e-13)
    # a collapsed hexahedron (top nodes = bottom nodes) has no volume and no matching faces
    cnode = m.cnode.copy()
    cnode[a + 4:a + 8] = m.cnode[a:a + 4]
    with pytest.raises(cg.CgksError) as e:
        S.set_mesh(mg.Mesh(m.xyz, m.ctype, m.cnode_ptr, cnode, m.bnode_ptr, m.bnode, m.btag, None))
    assert e.value.code == cg.E_MESH
    # the context stays usable with a valid mesh
    S.set_mesh(m)
    assert S.n_cells == m.n_cells


def test_boundary_tag_without_condition(cg, torch):
    say("[gpu] edge: boundary tag without a condition")
    m = mg.bump_channel(6, 4, 2, n_prism=0, n_pyr=0)
    S = cg.Solver()
    S.set_mesh(m)
    _channel_bcs(S, cg, skip=(mg.TAG_WALL_TOP,))
    W, G = mg.uniform_state(m.n_cells)
    Wd, Gd = to_dev(torch, W), to_dev(torch, G)
    S.geometry()  # geometry needs no boundary condition
    with pytest.raises(cg.CgksError) as e:
        S.residual(Wd, Gd)
    assert e.value.code == cg.E_STATE and str(mg.TAG_WALL_TOP) in str(e.value)
    S.set_bc(mg.TAG_WALL_TOP, cg.BC_SLIP)
    S.residual(Wd, Gd)
    S.check()


def test_nonphysical_state_is_reported_then_cleared(cg, torch):
    say("[gpu] edge: non-physical state")
    m = mg.bump_channel(12, 6, 4, n_prism=2, n_pyr=2, jitter=0.05, seed=3)
    S = cg.Solver()
    S.set_mesh(m)
    _channel_bcs(S, cg)
    W, G = mg.uniform_state(m.n_cells)
    Wbad = W.copy()
    Wbad[0, m.n_cells // 2] = -0.5  # negative density in one cell
    S.residual(to_dev(torch, Wbad), to_dev(torch, G))
    with pytest.raises(cg.CgksError) as e:
        S.check()
    assert e.value.code == cg.E_PHYS
    # the flag is cleared: a physical state evaluates cleanly afterwards
    R = S.residual(to_dev(torch, W), to_dev(torch, G))[0]
    S.check()
    assert np.isfinite(R.cpu().numpy()).all()
    # inside a batch of queued V-cycles the state is reported as well, and the flag cleared
    S.agglomerate()
    al = np.ones(m.n_cells)
    with pytest.raises(cg.CgksError) as e:
        S.vcycle(to_dev(torch, Wbad), to_dev(torch, G), to_dev(torch, al), 10, 1e-10)
    assert e.value.code == cg.E_PHYS
    hist, _ = S.vcycle(to_dev(torch, W), to_dev(torch, G), to_dev(torch, al), 3, 0.0)
    assert len(hist) == 3 and np.isfinite(hist).all()


def test_ragged_group_tail_matches_oracle(oracle, cg, torch):
    """130 cells: two full 64-cell reconstruction groups and a two-cell tail group, lane-map waves
    partly idle; the residual agrees with the oracle as on the larger meshes."""
    from gpu_common import assert_residual_close, cell_surface, flux_scale
    m = mg.bump_channel(13, 5, 2, n_prism=0, n_pyr=0)
    assert m.n_cells == 130
    say(f"[gpu] edge: ragged tail cells={m.n_cells}")
    M = oracle.Mesh(m)
    S = cg.Solver()
    S.set_mesh(m)
    _channel_bcs(S, cg)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, oracle.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, oracle.BC_SLIP)
    W, G = mg.smooth_state_and_gradients(mg.cell_node_mean(m), seed=5, amp=0.05)
    al = np.full(m.n_cells, 0.9)
    R, Gn, an = (t.cpu().numpy() for t in S.residual(to_dev(torch, W), to_dev(torch, G), to_dev(torch, al)))
    S.check()
    oR, oGn, oan, _ = M.residual(oracle.params(), W, G, al)
    F = M.faces()
    assert_residual_close(R, oR, cell_surface(F, m.n_cells), flux_scale(W), what="R ragged")
    np.testing.assert_allclose(an, oan, rtol=1e-10, atol=1e-14)
