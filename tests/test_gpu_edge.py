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
    from gpu_common import assert_residual_close, cell_flux_bound
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
    assert_residual_close(R, oR, cell_flux_bound(W, M.faces(), m.n_cells), what="R ragged")
    np.testing.assert_allclose(an, oan, rtol=1e-10, atol=1e-14)


def test_host_twins_equal_device_calls(cg, torch):
    """cgks_residual_host and cgks_vcycle_host (host arrays in the caller's order) give the device
    calls' results bit for bit, on a mesh whose cells are listed in a random order."""
    m = mg.permute_cells(mg.bump_channel(12, 6, 4, n_prism=2, n_pyr=2, jitter=0.05, seed=3, amp=0.05), seed=4)
    S = cg.Solver()
    S.set_mesh(m)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1.0 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        S.set_bc(tag, cg.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        S.set_bc(tag, cg.BC_SLIP)
    S.agglomerate()
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=6, amp=0.05)
    G = np.zeros((15, m.n_cells))
    al = np.ones(m.n_cells)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    R, Gn, an = S.residual(dev(W), dev(G), dev(al))
    Rh, Gnh, anh = S.residual_host(W, G, al)
    np.testing.assert_array_equal(Rh, R.cpu().numpy())
    np.testing.assert_array_equal(Gnh, Gn.cpu().numpy())
    np.testing.assert_array_equal(anh, an.cpu().numpy())
    Wd, Gd, ad = dev(W), dev(G), dev(al)
    h, _ = S.vcycle(Wd, Gd, ad, 5, 0.0)
    Wh, Gh, ah = W.copy(), G.copy(), al.copy()
    hh, _ = S.vcycle_host(Wh, Gh, ah, 5, 0.0)
    np.testing.assert_array_equal(hh, h)
    np.testing.assert_array_equal(Wh, Wd.cpu().numpy())
    np.testing.assert_array_equal(Gh, Gd.cpu().numpy())
    np.testing.assert_array_equal(ah, ad.cpu().numpy())


def test_batch_rollback_equals_checked_loop(cg, torch):
    """A state that turns non-physical a few cycles into a queued batch (a large CFL number on a
    perturbed channel): the batch call reports CGKS_E_PHYS with the cycles run and the state left
    bit-identical to a loop of single-cycle calls that stops at its first error (the batch restores
    its starting state and re-runs cycle by cycle)."""
    import ctypes as C
    m = mg.bump_channel(16, 6, 4, n_prism=2, n_pyr=2, jitter=0.05, seed=7, amp=0.05)
    S = cg.Solver()
    S.set_mesh(m)
    _channel_bcs(S, cg)
    S.agglomerate()
    x = mg.cell_node_mean(m)
    W0 = mg.random_smooth_state(x, seed=8, amp=0.05)
    G0 = np.zeros((15, m.n_cells))
    a0 = np.ones(m.n_cells)
    lib = cg.lib()
    found = None
    for cfl in (2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0):
        S.set_params(cfl=cfl)
        W, G, al = to_dev(torch, W0), to_dev(torch, G0), to_dev(torch, a0)
        j = None
        for k in range(16):
            try:
                S.vcycle(W, G, al, 1, 1e-10)
            except cg.CgksError as e:
                assert e.code == cg.E_PHYS
                j = k
                break
        if j is not None and 2 <= j <= 14:
            found = (cfl, j, W.clone(), G.clone(), al.clone())
            break
    assert found is not None, "no CFL number in the list fails inside the first batch"
    cfl, j, Wc, Gc, ac = found
    say(f"[gpu] rollback: CFL {cfl}, the checked loop fails in cycle {j + 1}")
    S.set_params(cfl=cfl)
    W, G, al = to_dev(torch, W0), to_dev(torch, G0), to_dev(torch, a0)
    hist = np.zeros(16)
    done = C.c_int32(-1)
    code = lib.cgks_vcycle(S.h, C.c_void_p(W.data_ptr()), C.c_void_p(G.data_ptr()), C.c_void_p(al.data_ptr()), 16,
                           1e-10, hist.ctypes.data_as(C.c_void_p), C.byref(done))
    assert code == cg.E_PHYS
    assert done.value == j
    bits = lambda t: t.contiguous().view(torch.int64)
    assert torch.equal(bits(W), bits(Wc)) and torch.equal(bits(G), bits(Gc)) and torch.equal(bits(al), bits(ac))
    # the flag is cleared afterwards: a physical state runs again
    S.set_params(cfl=0.5)
    h, _ = S.vcycle(to_dev(torch, W0), to_dev(torch, G0), to_dev(torch, a0), 3, 0.0)
    assert np.isfinite(h).all()
