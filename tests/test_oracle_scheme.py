"""Pins of the oracle's finite-volume scheme, reconstruction, agglomeration and
multigrid against facts fixed outside it (closed forms, invariants, brute force).

Paper: Sec. 2.2 (finite volume on hybrid meshes, face quadrature), Sec. 2.4
(gradient update), Sec. 3 (HWENO), Sec. 4.1 (agglomeration, Alg. 1),
Sec. 4.2 (restriction, forcing, correction, V-cycle).
"""
import os

import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def mixed(oracle):
    m = mg.periodic_mixed_box(6, jitter=0.15, seed=7)
    return m, oracle.Mesh(m)


@pytest.fixture(scope="module")
def channel(oracle):
    m = mg.bump_channel(12, 10, 4, n_prism=2, n_pyr=3, jitter=0.1, seed=3, amp=0.0)
    M = oracle.Mesh(m)
    return m, M


def _setup_channel_bc(oracle, M, U=(0.5, 0.0, 0.0)):
    prim = np.array([1.0, *U, 1 / 1.4])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, oracle.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, oracle.BC_SLIP)


# ------------------------------------------------------------------ geometry
def test_single_tet_volume_and_centroid(oracle):
    rng = np.random.default_rng(2)
    P = rng.normal(size=(4, 3))
    v = np.dot(np.cross(P[1] - P[0], P[2] - P[0]), P[3] - P[0]) / 6
    if v < 0:
        P[[1, 2]] = P[[2, 1]]
    m = mg.Mesh(P, np.array([4], np.uint8), np.array([0, 4]), np.arange(4), np.array([0, 3, 6, 9, 12]),
                np.array([0, 1, 3, 1, 2, 3, 2, 0, 3, 0, 2, 1]), np.ones(4, np.int32))
    M = oracle.Mesh(m)
    vol, cen, m2 = M.cells()
    assert vol[0] == pytest.approx(abs(v), rel=1e-13)
    np.testing.assert_allclose(cen[0], P.mean(axis=0), rtol=1e-13, atol=1e-14)
    # second moments of a tet: (V/20) (sum_i d_i d_i^T + (sum d)(sum d)^T) with d_i = P_i - c
    d = P - P.mean(axis=0)
    S = (d.T @ d + np.outer(d.sum(0), d.sum(0))) * abs(v) / 20
    np.testing.assert_allclose(m2[0], [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]], rtol=1e-12, atol=1e-15)


def test_closed_cells_and_divergence_volume(mixed):
    m, M = mixed
    vol, cen, _ = M.cells()
    F = M.faces()
    assert vol.sum() == pytest.approx(1.0, rel=1e-13)
    s = np.zeros((M.n_cells, 3))
    np.add.at(s, F["fl"], F["avec"])
    inner = F["fr"] >= 0
    np.add.at(s, F["fr"][inner], -F["avec"][inner])
    assert np.abs(s).max() < 1e-15
    # (1/3) sum x.n dS over the faces equals the quadrature volume; sum_k w S a.x n = V a (linear exactness)
    a = np.array([0.3, -1.1, 0.7])
    w = F["gpw"] * F["area"][:, None]
    dv = np.zeros(M.n_cells)
    ga = np.zeros((M.n_cells, 3))
    for side, sgn in ((F["fl"], 1.0), (F["fr"], -1.0)):
        sel = side >= 0
        X = F["gpx"] - (F["shift"][:, None, :] if sgn < 0 else 0.0)
        xn = np.einsum("fkd,fkd->fk", X, F["gpn"])
        np.add.at(dv, side[sel], sgn * (w * xn).sum(1)[sel] / 3)
        lin = np.einsum("fkd,d->fk", X, a)
        np.add.at(ga, side[sel], sgn * np.einsum("fk,fk,fkd->fd", w, lin, F["gpn"])[sel])
    np.testing.assert_allclose(dv, vol, rtol=1e-13)
    np.testing.assert_allclose(ga, vol[:, None] * a[None, :], rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------------ reconstruction
def _quadratic_data(M, coeff, x0=np.zeros(3)):
    """Exact cell averages and gradient averages of a global quadratic from cell moments."""
    vol, cen, m2 = M.cells()
    c = cen - x0
    xx, yy, zz, xy, yz, xz = (m2[:, i] / vol for i in range(6))
    a0, ax, ay, az, axx, ayy, azz, axy, ayz, axz = coeff
    avg = (a0 + ax * c[:, 0] + ay * c[:, 1] + az * c[:, 2] + axx * (xx + c[:, 0] ** 2) + ayy * (yy + c[:, 1] ** 2)
           + azz * (zz + c[:, 2] ** 2) + axy * (xy + c[:, 0] * c[:, 1]) + ayz * (yz + c[:, 1] * c[:, 2])
           + axz * (xz + c[:, 0] * c[:, 2]))
    gx = ax + 2 * axx * c[:, 0] + axy * c[:, 1] + axz * c[:, 2]
    gy = ay + 2 * ayy * c[:, 1] + axy * c[:, 0] + ayz * c[:, 2]
    gz = az + 2 * azz * c[:, 2] + ayz * c[:, 1] + axz * c[:, 0]
    return avg, np.stack([gx, gy, gz])


def test_linear_weights_reproduce_global_quadratics(oracle, channel):
    m, M = channel
    _setup_channel_bc(oracle, M)
    vol, cen, _ = M.cells()
    rng = np.random.default_rng(4)
    W = np.zeros((5, M.n_cells))
    G = np.zeros((15, M.n_cells))
    coeffs = []
    for q in range(5):
        cf = rng.normal(size=10) * 0.05
        cf[0] = (1.0, 0.3, 0.1, -0.1, 3.0)[q]
        coeffs.append(cf)
        W[q], g = _quadratic_data(M, cf)
        G[3 * q:3 * q + 3] = g
    # eps -> infinity gives the linear weights, R = p^2 (Sec. 3.4, Eq. weno-linear)
    coef = M.reconstruct(oracle.params(weno_eps=1e30), W, G, np.ones(M.n_cells))
    F = M.faces()
    nint = np.bincount(F["fl"][F["fr"] >= 0], minlength=M.n_cells) + np.bincount(F["fr"][F["fr"] >= 0],
                                                                               minlength=M.n_cells)
    full = nint >= 3
    assert full.mean() > 0.9
    for q in range(5):
        cf = coeffs[q]
        c = cen
        # expected monomial coefficients about each centroid
        exp = np.zeros((M.n_cells, 10))
        a0, ax, ay, az, axx, ayy, azz, axy, ayz, axz = cf
        exp[:, 0] = (a0 + ax * c[:, 0] + ay * c[:, 1] + az * c[:, 2] + axx * c[:, 0] ** 2 + ayy * c[:, 1] ** 2
                     + azz * c[:, 2] ** 2 + axy * c[:, 0] * c[:, 1] + ayz * c[:, 1] * c[:, 2] + axz * c[:, 0] * c[:, 2])
        exp[:, 1] = ax + 2 * axx * c[:, 0] + axy * c[:, 1] + axz * c[:, 2]
        exp[:, 2] = ay + 2 * ayy * c[:, 1] + axy * c[:, 0] + ayz * c[:, 2]
        exp[:, 3] = az + 2 * azz * c[:, 2] + ayz * c[:, 1] + axz * c[:, 0]
        exp[:, 4:] = [axx, ayy, azz, axy, ayz, axz]
        np.testing.assert_allclose(coef[full, q], exp[full], rtol=1e-9, atol=1e-11)


def test_reconstruction_is_scale_invariant(oracle, channel):
    """x -> s x with data rescaled: coefficients scale by s^-|k| (pins the |Omega|^(1/3) row scaling)."""
    m, M = channel
    _setup_channel_bc(oracle, M)
    vol, cen, _ = M.cells()
    W = mg.random_smooth_state(cen, seed=11, amp=0.2)
    G = np.zeros((15, M.n_cells))
    rng = np.random.default_rng(9)
    G[:] = rng.normal(size=G.shape) * 0.3
    par = oracle.params()
    c1 = M.reconstruct(par, W, G, np.full(M.n_cells, 0.9))
    s = 2.5
    m2 = mg.Mesh(m.xyz * s, m.ctype, m.cnode_ptr, m.cnode, m.bnode_ptr, m.bnode, m.btag)
    M2 = oracle.Mesh(m2)
    _setup_channel_bc(oracle, M2)
    c2 = M2.reconstruct(par, W, G / s, np.full(M.n_cells, 0.9))
    scale = np.array([1, s, s, s, s * s, s * s, s * s, s * s, s * s, s * s])
    np.testing.assert_allclose(c2 * scale, c1, rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------------ finite volume scheme
def test_free_stream_preservation_periodic(oracle, mixed):
    m, M = mixed
    W, G = mg.uniform_state(M.n_cells, vel=(0.5, 0.3, -0.2))
    for par in (oracle.params(), oracle.params(viscous=True, mu=0.01, prandtl=0.72)):
        R, Gn, an, dt = M.residual(par, W, G, np.ones(M.n_cells))
        F = M.faces()
        scale = np.zeros(M.n_cells)
        np.add.at(scale, F["fl"], F["area"])
        np.add.at(scale, F["fr"], F["area"])
        assert np.abs(R).max() <= 1e-13 * scale.max() * 2.0
        assert np.abs(Gn).max() < 1e-12
        assert np.all(an == 1.0)


def test_free_stream_preservation_walls_and_farfield(oracle, channel):
    m, M = channel
    _setup_channel_bc(oracle, M)
    W, G = mg.uniform_state(M.n_cells, vel=(0.5, 0.0, 0.0))
    R, Gn, an, dt = M.residual(oracle.params(), W, G, np.ones(M.n_cells))
    assert np.abs(R).max() < 1e-13
    assert np.abs(Gn).max() < 1e-12


def test_discrete_conservation_periodic_s2o4(oracle, mixed):
    m, M = mixed
    vol, cen, _ = M.cells()
    W = mg.random_smooth_state(cen, seed=5, amp=0.1)
    G = np.zeros((15, M.n_cells))
    al = np.ones(M.n_cells)
    par = oracle.params()
    dt = 0.5 * M.local_dt(par, W).min()
    tot0 = (W * vol).sum(1)
    for _ in range(3):
        M.step_s2o4(par, dt, W, G, al)
    np.testing.assert_allclose((W * vol).sum(1), tot0, rtol=0, atol=1e-14 * np.abs(tot0).max() * 10)


@pytest.mark.slow
def test_density_wave_third_order(oracle):
    """Smooth density wave on periodic hexahedra (8^3 -> 16^3): observed L1 order close to 3 (Sec. 3)."""
    par = oracle.params()
    T = 0.02
    errs = []
    for n in (8, 16):
        M = oracle.Mesh(mg.periodic_hex_cube(n))
        W, G = mg.density_wave_averages(n)
        al = np.ones(M.n_cells)
        dt0 = M.local_dt(par, W).min()
        ns = int(np.ceil(T / dt0))
        for _ in range(ns):
            M.step_s2o4(par, T / ns, W, G, al)
        We, _ = mg.density_wave_averages(n, T=T)
        errs.append(np.abs(W[0] - We[0]).mean())
    order = np.log2(errs[0] / errs[1])
    assert 2.6 < order < 3.6, errs


# ------------------------------------------------------------------ agglomeration
def test_hash_worked_example(oracle):
    with open(os.path.join(GOLDEN, "hash_worked_example.txt")) as f:
        line = [ln for ln in f if not ln.startswith("#")][0]
    kv = dict(t.split("=") for t in line.split())
    assert oracle.face_hash(int(kv["left"]), int(kv["right"]), int(kv["nf"])) == int(kv["formula"])
    assert (23 * (10 + 12) + 10 * 12) % 100 == int(kv["formula"]) != int(kv["printed"])


def test_skew_predicate_geometry(oracle):
    """Two unit cubes across x = 1: virtual centre on the face centre -> accept; lopsided in-plane -> reject."""
    A = np.array([1.0, 0, 0])
    S, M = 1.0, np.array([1.0, 0.5, 0.5])
    assert oracle.skew_accept(1, 1, [0.5, 0.5, 0.5], [1.5, 0.5, 0.5], S, M, A, 0.25, np.sin(np.deg2rad(10)))
    # centre displaced along the face plane by 0.6 -> d in-plane and long: reject
    assert not oracle.skew_accept(1, 1, [0.5, 1.1, 0.5], [1.5, 1.1, 0.5], S, M, A, 0.25, np.sin(np.deg2rad(10)))
    # displaced along the normal: angle 90 deg: accept
    assert oracle.skew_accept(1, 1, [0.0, 0.5, 0.5], [1.0, 0.5, 0.5], S, M, A, 0.25, np.sin(np.deg2rad(10)))


def _fine_graph(oracle, M):
    vol, cen, _ = M.cells()
    F = M.faces()
    sel = (F["fr"] >= 0) & np.all(F["shift"] == 0, axis=1)
    return oracle.Graph(vol, vol[:, None] * cen, F["fl"][sel], F["fr"][sel], F["area"][sel], F["fmom"][sel],
                        F["avec"][sel])


def _brute_force_agglomerate(g, seed, passes, delta, smin):
    """Plain-Python restatement of the pass (Sec. 4.1, Alg. 1 with the readings in the oracle header)."""
    n = len(g.V)
    V = [float(v) for v in g.V]
    P = [list(map(float, p)) for p in g.P]
    pairs = [(int(a), int(b), float(s), list(map(float, mm)), list(map(float, aa)))
             for a, b, s, mm, aa in zip(g.a, g.b, g.S, g.M, g.A)]
    f2c = list(range(n))
    for _ in range(passes):
        nf = len(pairs)
        seen, mate = set(), {}
        matched = set()
        for j, (a, b, s, mm, aa) in enumerate(pairs):
            h = (23 * seed * (a + b) + a * b) % nf
            if h in seen:
                continue
            seen.add(h)
            Vt = V[a] + V[b]
            Pt = [P[a][d] + P[b][d] for d in range(3)]
            e = [Vt * mm[d] - s * Pt[d] for d in range(3)]
            ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2]
            d2 = delta * delta
            ok = ee * ee * ee <= (d2 * d2 * d2) * (((Vt * Vt) * (Vt * Vt)) * ((Vt * Vt) * (Vt * Vt))) * ((s * s) * (s * s) * (s * s))
            if not ok:
                ea = e[0] * aa[0] + e[1] * aa[1] + e[2] * aa[2]
                A2 = aa[0] * aa[0] + aa[1] * aa[1] + aa[2] * aa[2]
                ok = ea * ea >= smin * smin * ee * A2
            if ok and a not in matched and b not in matched:
                matched.update((a, b))
                mate[b] = a
        new = {}
        k = 0
        for i in range(len(V)):
            if i not in mate:
                new[i] = k
                k += 1
        for i in mate:
            new[i] = new[mate[i]]
        V2, P2 = [0.0] * k, [[0.0] * 3 for _ in range(k)]
        for i in range(len(V)):
            if i not in mate:
                V2[new[i]] = V[i]
                P2[new[i]] = list(P[i])
        for b_, a_ in mate.items():
            V2[new[b_]] = V[a_] + V[b_]
            P2[new[b_]] = [P[a_][d] + P[b_][d] for d in range(3)]
        groups = {}
        for j, (a, b, s, mm, aa) in enumerate(pairs):
            x, y = new[a], new[b]
            if x == y:
                continue
            sg = 1.0 if x < y else -1.0
            key = (min(x, y), max(x, y))
            G = groups.setdefault(key, [0.0, [0.0] * 3, [0.0] * 3])
            G[0] += s
            for d in range(3):
                G[1][d] += mm[d]
                G[2][d] += sg * aa[d]
        pairs = [(a, b, G[0], G[1], G[2]) for (a, b), G in sorted(groups.items())]
        f2c = [new[c] for c in f2c]
        V, P = V2, P2
    return np.array(f2c), len(V)


def test_agglomeration_matches_brute_force(oracle, channel):
    m, M = channel
    g = _fine_graph(oracle, M)
    for seed in (1, 7):
        f2c, cg, stats = oracle.agglomerate_graph(g, seed=seed, passes=3)
        bf, nc = _brute_force_agglomerate(g, seed, 3, 0.25, np.sin(np.deg2rad(10.0)))
        assert nc == len(cg.V)
        np.testing.assert_array_equal(f2c, bf)


def test_agglomeration_invariants(oracle):
    m = mg.bump_channel(24, 16, 8, n_prism=2, n_pyr=4, jitter=0.05, seed=1)
    M = oracle.Mesh(m)
    g = _fine_graph(oracle, M)
    P = 3
    f2c, cg, stats = oracle.agglomerate_graph(g, seed=1, passes=P)
    nc = len(cg.V)
    # partition: every fine cell in exactly one coarse cell, ids dense
    assert f2c.min() == 0 and f2c.max() == nc - 1 and len(np.unique(f2c)) == nc
    sizes = np.bincount(f2c)
    assert sizes.max() <= 2 ** P
    assert g.V.shape[0] / nc > 2.5
    # volumes and first moments add up
    np.testing.assert_allclose(cg.V.sum(), g.V.sum(), rtol=1e-13)
    np.testing.assert_allclose(np.bincount(f2c, weights=g.V), cg.V, rtol=1e-13)
    # numbering by smallest member id
    first = np.full(nc, np.iinfo(np.int64).max)
    np.minimum.at(first, f2c, np.arange(len(f2c)))
    assert np.all(np.diff(first) > 0)
    # each coarse cell is connected through fine interior faces
    parent = np.arange(len(f2c))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in zip(g.a, g.b):
        if f2c[a] == f2c[b]:
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(len(f2c))])
    assert len(np.unique(roots)) == nc
    # coarse area vectors close each coarse cell together with the boundary
    # determinism
    f2c2, _, _ = oracle.agglomerate_graph(g, seed=1, passes=P)
    np.testing.assert_array_equal(f2c, f2c2)


# ------------------------------------------------------------------ multigrid
def test_transfer_invariants_and_fas_fixed_point(oracle, channel):
    m, M = channel
    _setup_channel_bc(oracle, M)
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    vol, cen, _ = M.cells()
    L1, L2 = H.level(1), H.level(2)
    assert L1["V"].sum() == pytest.approx(vol.sum(), rel=1e-13)
    assert L2["V"].sum() == pytest.approx(vol.sum(), rel=1e-13)
    assert L1["n"] < M.n_cells and L2["n"] < L1["n"]
    W, G = mg.uniform_state(M.n_cells)
    Wc, Rc = H.restrict(1, W, np.zeros_like(W))
    np.testing.assert_allclose(Wc, np.repeat(W[:, :1], L1["n"], axis=1), rtol=1e-14)
    par = oracle.params()
    # coarse KFVS of a uniform free stream vanishes
    assert np.abs(H.kfvs_residual(par, 1, Wc)).max() < 1e-13
    # the free stream is a fixed point of the V-cycle
    al = np.ones(M.n_cells)
    W0 = W.copy()
    H.vcycle(par, W, G, al)
    np.testing.assert_allclose(W, W0, rtol=0, atol=1e-13)


def test_vcycle_accelerates_convergence(oracle):
    """Paper Sec. 5: the V-cycle needs far fewer iterations than explicit CGKS (sanity band only)."""
    m = mg.bump_channel(24, 12, 6, n_prism=2, n_pyr=3, jitter=0.05, seed=1, amp=0.05)
    M = oracle.Mesh(m)
    _setup_channel_bc(oracle, M)
    par = oracle.params(cfl=0.5)
    H = oracle.Hierarchy(M, levels=3, passes=3, seed=1)
    res = {}
    for mode in ("explicit", "vcycle"):
        W, G = mg.uniform_state(M.n_cells)
        al = np.ones(M.n_cells)
        hist = []
        for it in range(40):
            if mode == "explicit":
                hist.append(M.step_fe(par, W, G, al))
            else:
                hist.append(H.vcycle(par, W, G, al))
        res[mode] = hist[-1] / hist[0]
    assert res["vcycle"] < res["explicit"]


# ------------------------------------------------------------------ wall force
def _face_area_vectors(m, tag):
    """Area vectors of the boundary faces with `tag` from their nodes (exact for a bilinear quad)."""
    out = []
    for b in range(m.btag.shape[0]):
        if m.btag[b] != tag:
            continue
        x = m.xyz[m.bnode[m.bnode_ptr[b]:m.bnode_ptr[b + 1]]]
        if x.shape[0] == 3:
            a = 0.5 * np.cross(x[1] - x[0], x[2] - x[0])
        else:
            a = 0.5 * np.cross(x[2] - x[0], x[3] - x[1])
        out.append(a)
    return np.array(out)


def test_wall_force_rest_state_is_pressure_times_area(oracle):
    """Gas at rest: every face flux is p n exactly, so the force on the curved lower wall is
    p times the sum of its face area vectors (computed here from the nodes)."""
    m = mg.bump_channel(12, 8, 4, n_prism=2, n_pyr=3, jitter=0.1, seed=5, amp=0.05)
    M = oracle.Mesh(m)
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET, mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, oracle.BC_SLIP)
    p0, gam = 0.8, 1.4
    W = np.zeros((5, m.n_cells))
    W[0] = 1.0
    W[4] = p0 / (gam - 1)
    G = np.zeros((15, m.n_cells))
    F = M.wall_force(oracle.params(), W, G, None, mg.TAG_WALL_BOTTOM)
    A = _face_area_vectors(m, mg.TAG_WALL_BOTTOM)
    A *= -np.sign(A[:, 1])[:, None]  # out of the gas: downwards through the lower wall
    ref = p0 * A.sum(axis=0)
    assert ref[1] == pytest.approx(-1.5 * p0, rel=1e-12)  # projected area of the wall
    np.testing.assert_allclose(F, ref, rtol=0, atol=1e-13 * p0 * 1.5)


def test_wall_force_uniform_flow_flat_wall(oracle, channel):
    """Uniform stream tangent to a flat slip wall: the ghost state equals the interior state, the
    flux is the Euler flux, and its momentum part through the wall is p n: F = (0, -p A, 0)."""
    m, M = channel
    _setup_channel_bc(oracle, M)
    W, G = mg.uniform_state(m.n_cells)
    F = M.wall_force(oracle.params(), W, G, None, mg.TAG_WALL_BOTTOM)
    p = 1 / 1.4
    np.testing.assert_allclose(F, [0.0, -1.5 * p, 0.0], rtol=0, atol=1e-13)
    # upper wall: normal +y
    Ft = M.wall_force(oracle.params(), W, G, None, mg.TAG_WALL_TOP)
    np.testing.assert_allclose(Ft, [0.0, 1.5 * p, 0.0], rtol=0, atol=1e-13)
