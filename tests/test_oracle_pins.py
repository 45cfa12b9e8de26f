"""Further pins of the oracle against facts fixed outside it.

* Eq. (2nd-flux) with unequal, non-zero slopes on both sides and a collision time of the order of
  the step, evaluated by brute-force quadrature in velocity space (Gauss-Legendre on each half
  space, Gauss-Hermite elsewhere) and in time (Gauss-Legendre over the step), with the micro-slopes,
  time slopes, interface state and its slopes (Eqs. co, compatibility2 and the half-space slopes of
  g^c) solved from quadrature moments: pins the closed-form time integrals (the te^{-t/tau_n}
  integral of the kinetic and equilibrium slope terms), the interface value and the assembly.
* Sec. 3.4 by hand on a cube cell with quadratic data: beta_1 = min(beta_GG, beta_LS), beta_2 with
  the weights |Omega|^{2|alpha|/3 - 1}, the normalisation, the global indicator and the nonlinear
  weights, and the final polynomial R = w2 P2 + w1 P1.
* Sec. 3.3: the compression factor of one Gauss point from primitive variables.
* Far-field ghost states keep the outgoing Riemann invariant of the interior, the incoming one of the
  free stream, and the upwind entropy and tangential velocity; wall ghost gradients are those of the
  mirrored (slip) or reversed (no-slip) linear field.
* Sec. 4.3 (lambda) and Secs. 1, 4.2 (local time stepping): the local step of a cube, and the coarse
  steps of agglomerates from their outer faces.
"""
import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)


def cons(rho, u, p, gamma=GAMMA):
    u = np.asarray(u, float)
    return np.array([rho, *(rho * u), p / (gamma - 1) + 0.5 * rho * u @ u])


def prim(W, gamma=GAMMA):
    rho = W[0]
    U = W[1:4] / rho
    p = (gamma - 1) * (W[4] - 0.5 * rho * U @ U)
    return rho, U, p


# ------------------------------------------------------------------ velocity-space quadrature
class MaxwellGrid:
    """Quadrature of the unit-density Maxwellian with velocity U and lambda = rho/(2p) in the
    variables (u, v, w, xi_1, xi_2) (K = 2 internal degrees of freedom), over u > 0, u < 0 or
    all u.  Half spaces use Gauss-Legendre in u on [0, |U| + 14 sigma]; everything else
    Gauss-Hermite."""

    def __init__(self, U, lam, half=0, nu=160, nh=14, nx=8):
        s = 1.0 / np.sqrt(lam)
        if half == 0:
            x, w = np.polynomial.hermite.hermgauss(48)
            u, wu = U[0] + x * s, w / np.sqrt(np.pi)
        else:
            top = abs(U[0]) + 14.0 * s
            x, w = np.polynomial.legendre.leggauss(nu)
            u = 0.5 * top * (x + 1.0)
            wu = 0.5 * top * w * np.sqrt(lam / np.pi) * np.exp(-lam * (half * u - U[0]) ** 2)
            u = half * u
        xh, wh = np.polynomial.hermite.hermgauss(nh)
        v, wv = U[1] + xh * s, wh / np.sqrt(np.pi)
        ww_, www = U[2] + xh * s, wh / np.sqrt(np.pi)
        xx, wx = np.polynomial.hermite.hermgauss(nx)
        xi, wxi = xx * s, wx / np.sqrt(np.pi)
        G = np.meshgrid(u, v, ww_, xi, xi, indexing="ij")
        Wt = np.einsum("a,b,c,d,e->abcde", wu, wv, www, wxi, wxi)
        self.u, self.v, self.w = G[0].ravel(), G[1].ravel(), G[2].ravel()
        self.xi2 = (G[3] ** 2 + G[4] ** 2).ravel()
        self.wt = Wt.ravel()
        self.psi = np.stack([np.ones_like(self.u), self.u, self.v, self.w,
                             0.5 * (self.u ** 2 + self.v ** 2 + self.w ** 2 + self.xi2)])
        self.vel = (self.u, self.v, self.w)

    def mom(self, f):
        """<psi f> for a weight array f over the grid."""
        return self.psi @ (self.wt * f)

    def mat(self, f):
        """<psi psi^T f>."""
        return (self.psi * (self.wt * f)) @ self.psi.T


def _lam(W):
    rho, U, p = prim(W)
    return rho, U, rho / (2 * p)


def _slopes(rho, U, lam, dW):
    """Micro-slopes from rho <psi psi^T> a_j = dW_j and the time slope from <(A + a.u) psi> = 0."""
    g = MaxwellGrid(U, lam)
    M = rho * g.mat(np.ones_like(g.u))
    a = np.stack([np.linalg.solve(M, dW[j]) for j in range(3)])
    rhs = -sum(rho * g.mat(g.vel[j]) @ a[j] for j in range(3))
    A = np.linalg.solve(M, rhs)
    return a, A


def flux_by_quadrature(Wl, dWl, Wr, dWr, dt, mu=0.0, eps=0.01, C=1.0):
    """Time-averaged flux over [0, dt], its integral over [0, dt/2] and the interface values at dt
    and dt/2 of Eq. (2nd-flux), everything by quadrature (local frame, normal = x)."""
    rl, Ul, ll = _lam(Wl)
    rr, Ur, lr = _lam(Wr)
    al, Al = _slopes(rl, Ul, ll, dWl)
    ar, Ar = _slopes(rr, Ur, lr, dWr)
    gl, gr = MaxwellGrid(Ul, ll, +1), MaxwellGrid(Ur, lr, -1)
    one_l, one_r = np.ones_like(gl.u), np.ones_like(gr.u)
    Wc = rl * gl.mom(one_l) + rr * gr.mom(one_r)
    # interface slopes: kinetic-weighted half-space moments of the two side slopes
    dWc = np.stack([rl * gl.mat(one_l) @ al[j] + rr * gr.mat(one_r) @ ar[j] for j in range(3)])
    rc, Uc, lc = _lam(Wc)
    ac, Ac = _slopes(rc, Uc, lc, dWc)
    gc = MaxwellGrid(Uc, lc, 0)
    pl, pr, pc = prim(Wl)[2], prim(Wr)[2], prim(Wc)[2]
    jump = C * abs((pl - pr) / (pl + pr)) * dt
    tau = mu / pc if mu > 0 else 0.0
    taun = tau + jump if mu > 0 else eps * dt + jump

    def sl(g, a):  # (a . u) as a function on the grid: sum_j (a_j . psi) u_j
        return sum((a[j] @ g.psi) * g.vel[j] for j in range(3))

    # moment vectors of each term of f(0, t) against psi and u psi
    terms = {
        "gc": (rc, gc, np.ones_like(gc.u)),
        "gc_a": (rc, gc, sl(gc, ac)),
        "gc_A": (rc, gc, Ac @ gc.psi),
    }
    mom_v, mom_f = {}, {}
    for k, (rho, g, f) in terms.items():
        mom_v[k] = rho * g.mom(f)
        mom_f[k] = rho * g.mom(g.u * f)
    kin = {"k": (np.ones_like(gl.u), np.ones_like(gr.u)), "k_a": (sl(gl, al), sl(gr, ar)),
           "k_A": (Al @ gl.psi, Ar @ gr.psi)}
    for k, (fl, fr) in kin.items():
        mom_v[k] = rl * gl.mom(fl) + rr * gr.mom(fr)
        mom_f[k] = rl * gl.mom(gl.u * fl) + rr * gr.mom(gr.u * fr)

    def coeffs(t):
        e = np.exp(-t / taun)
        return {"gc": 1 - e, "gc_a": (t + tau) * e - tau, "gc_A": t - tau + tau * e,
                "k": e, "k_a": -(tau + t) * e, "k_A": -tau * e}

    def value(t):
        c = coeffs(t)
        return sum(c[k] * mom_v[k] for k in c)

    def integral(T, n=40):
        x, w = np.polynomial.legendre.leggauss(n)
        ts, ws = 0.5 * T * (x + 1), 0.5 * T * w
        out = np.zeros(5)
        for t, wt in zip(ts, ws):
            c = coeffs(t)
            out += wt * sum(c[k] * mom_f[k] for k in c)
        return out

    Fint = integral(dt)
    return dict(F=Fint / dt, Fint=Fint, Fhalf=integral(0.5 * dt), Wdt=value(dt), Whalf=value(0.5 * dt), Wc=Wc)


@pytest.mark.parametrize("viscous", [False, True])
def test_flux_by_velocity_and_time_quadrature(oracle, viscous):
    rng = np.random.default_rng(11)
    Wl = cons(1.1, [0.25, 0.1, -0.05], 1.0)
    Wr = cons(0.85, [0.15, -0.1, 0.1], 0.8)
    dWl = rng.normal(size=(3, 5)) * 0.3
    dWr = rng.normal(size=(3, 5)) * 0.3
    dt = 0.04
    if viscous:
        mu = 0.004     # tau = mu / p_c ~ 0.1 dt
        par = oracle.params(viscous=True, mu=mu, prandtl=1.0, c_tau=1.0)
        ref = flux_by_quadrature(Wl, dWl, Wr, dWr, dt, mu=mu, C=1.0)
    else:
        # C = 4: tau_n ~ 0.45 dt, so exp(-t/tau_n) and t exp(-t/tau_n) both matter over the step
        par = oracle.params(c_tau=4.0)
        ref = flux_by_quadrature(Wl, dWl, Wr, dWr, dt, eps=0.01, C=4.0)
    out = oracle.gks_point(Wl, dWl, Wr, dWr, dt, par)
    for key in ("F", "Wdt", "Whalf", "Wc"):
        np.testing.assert_allclose(out[key], ref[key], rtol=2e-11, atol=2e-12, err_msg=key)
    for key in ("Fint", "Fhalf"):
        np.testing.assert_allclose(out[key], ref[key], rtol=2e-11, atol=2e-13, err_msg=key)
    # the time-dependent terms really matter in this case: the interface value moves over the step
    assert np.abs(ref["Wdt"] - ref["Wc"]).max() > 1e-3


# ------------------------------------------------------------------ HWENO weights by hand
def test_weno_weights_by_hand(oracle):
    """Cube cell (side h) of a uniform hexahedral mesh, quadratic data per component
    Q = q + b.(x - x0) + (x - x0)^T H (x - x0)/2: p^2 = Q (linear weights reproduce quadratics),
    Green-Gauss and least-squares gradients of the averages are both b, so with the previous
    compression factor alpha < 1, beta_GG = alpha^2 |b|^2 V^(2/3) < beta_LS and beta_1 = beta_GG.
    Integrals over the cube: int |grad Q|^2 = V |b|^2 + h^5/12 |H|_F^2; second derivatives are
    constant, each distinct one counted once."""
    n = 4
    h = 1.0 / n
    m = mg.periodic_hex_cube(n)
    M = oracle.Mesh(m)
    vol, cen, _ = M.cells()
    i0 = 1 + n * (1 + n * 2)          # interior cell (1, 1, 2): all six neighbours without a period shift
    x0 = cen[i0]
    rng = np.random.default_rng(5)
    qs = np.array([1.0, 0.3, -0.02, 0.0, 2.6])
    bs = rng.normal(size=(5, 3)) * np.array([0.4, 0.3, 0.05, 0.02, 0.8])[:, None]
    Hs = []
    for c in range(5):
        B = rng.normal(size=(3, 3)) * [1.5, 1.0, 0.3, 0.2, 2.0][c]
        Hs.append(0.5 * (B + B.T))
    N = m.n_cells
    W = np.zeros((5, N))
    G = np.zeros((15, N))
    d = cen - x0
    for c in range(5):
        H = Hs[c]
        W[c] = qs[c] + d @ bs[c] + 0.5 * np.einsum("ni,ij,nj->n", d, H, d) + h * h / 24 * np.trace(H)
        for e in range(3):
            G[3 * c + e] = bs[c][e] + d @ H[e]
    alpha = np.ones(N)
    a0 = 0.6
    alpha[i0] = a0
    par = oracle.params()
    coef = oracle.Mesh(m).reconstruct(par, W, G, alpha)[i0]     # (5, 10) about the centroid
    V = h ** 3
    g1, g2, eps = 0.5, 0.5, 1e-5
    for c in range(5):
        q, b, H = qs[c], bs[c], Hs[c]
        Qbar = q + h * h / 24 * np.trace(H)
        # polynomials in the monomial basis 1, dx, dy, dz, dx^2, dy^2, dz^2, dxdy, dydz, dxdz
        p2 = np.array([q, *b, H[0, 0] / 2, H[1, 1] / 2, H[2, 2] / 2, H[0, 1], H[1, 2], H[0, 2]])
        p1 = np.array([Qbar, *(a0 * b), 0, 0, 0, 0, 0, 0])
        b1 = min(V ** (2 / 3) * a0 * a0 * (b @ b), V ** (2 / 3) * (b @ b))
        second = H[0, 0] ** 2 + H[1, 1] ** 2 + H[2, 2] ** 2 + H[0, 1] ** 2 + H[1, 2] ** 2 + H[0, 2] ** 2
        b2 = V ** (-1 / 3) * (V * (b @ b) + h ** 5 / 12 * (H * H).sum()) + V ** (1 / 3) * V * second
        den = Qbar ** 2 + b1 + 1e-40
        t1, t2 = b1 / den, b2 / den
        sig = abs(t2 - t1)
        w1 = g1 * (1 + (sig / (eps + t1)) ** 2)
        w2 = g2 * (1 + (sig / (eps + t2)) ** 2)
        w1, w2 = w1 / (w1 + w2), w2 / (w1 + w2)
        R = w2 * (p2 - g1 * p1) / g2 + w1 * p1
        np.testing.assert_allclose(coef[c], R, rtol=1e-10, atol=1e-12 * np.abs(R).max(), err_msg=f"component {c}")
        if c in (0, 4):
            assert abs(w1 - g1) > 0.05   # the weights are genuinely nonlinear in this case


# ------------------------------------------------------------------ compression factor
def test_compression_factor_by_hand(oracle):
    """alpha_pk = 1/(1 + A^2), A = |dp|/p_l + |dp|/p_r + (Ma_n,l - Ma_n,r)^2 + (Ma_t,l - Ma_t,r)^2
    with Ma_t from the tangential speed (both tangential components non-zero)."""
    rl, ul, vl, wl, pl = 1.2, 0.4, 0.3, -0.2, 1.1
    rr, ur, vr, wr, pr = 0.9, 0.1, -0.1, 0.25, 0.7
    cl, cr = np.sqrt(GAMMA * pl / rl), np.sqrt(GAMMA * pr / rr)
    A = abs(pl - pr) / pl + abs(pl - pr) / pr + (ul / cl - ur / cr) ** 2 + \
        (np.hypot(vl, wl) / cl - np.hypot(vr, wr) / cr) ** 2
    got = oracle.cf_point(cons(rl, [ul, vl, wl], pl), cons(rr, [ur, vr, wr], pr))
    assert got == pytest.approx(1.0 / (1.0 + A * A), rel=1e-14)
    # equal states: no compression; a rotation of the tangential plane leaves it unchanged
    assert oracle.cf_point(cons(rl, [ul, vl, wl], pl), cons(rl, [ul, vl, wl], pl)) == 1.0
    th = 0.8
    rot = lambda v, w: (np.cos(th) * v - np.sin(th) * w, np.sin(th) * v + np.cos(th) * w)
    got2 = oracle.cf_point(cons(rl, [ul, *rot(vl, wl)], pl), cons(rr, [ur, *rot(vr, wr)], pr))
    assert got2 == pytest.approx(got, rel=1e-13)


# ------------------------------------------------------------------ boundary ghost states
def _invariants(W, n, gamma=GAMMA):
    rho, U, p = prim(W)
    c = np.sqrt(gamma * p / rho)
    un = U @ n
    return un + 2 * c / (gamma - 1), un - 2 * c / (gamma - 1), p / rho ** gamma, U - un * n


@pytest.mark.parametrize("case", ["subsonic_outflow", "subsonic_inflow", "supersonic_inflow", "supersonic_outflow"])
def test_farfield_ghost_riemann_invariants(oracle, case):
    """Outward normal n.  Subsonic: the ghost keeps the interior's outgoing invariant u_n + 2c/(g-1)
    and the free stream's incoming one u_n - 2c/(g-1); entropy and tangential velocity come from
    the upwind side (interior for outflow, free stream for inflow).  Supersonic: the upwind state."""
    n = np.array([0.6, 0.0, 0.8])
    t = np.array([0.8, 0.0, -0.6])
    far = np.array([1.0, 0.5 * n[0] + 0.1 * t[0], 0.05, 0.5 * n[2] + 0.1 * t[2], 1 / GAMMA])
    Wf = cons(far[0], far[1:4], far[4])
    if case == "subsonic_outflow":
        Wi = cons(1.05, 0.4 * n + 0.2 * t + [0, -0.1, 0], 0.75)
    elif case == "subsonic_inflow":
        far = np.array([1.0, *(-0.5 * n + 0.1 * t), 1 / GAMMA])
        Wf = cons(far[0], far[1:4], far[4])
        Wi = cons(0.95, -0.4 * n - 0.2 * t + [0, 0.1, 0], 0.68)
    elif case == "supersonic_inflow":
        far = np.array([1.0, *(-1.6 * n + 0.2 * t), 1 / GAMMA])
        Wf = cons(far[0], far[1:4], far[4])
        Wi = cons(1.3, -1.5 * n, 0.9)
    else:
        Wi = cons(1.0, 1.7 * n + 0.3 * t, 1 / GAMMA)
    Wg, Gg = oracle.bc_ghost(oracle.BC_FARFIELD, n, Wi, np.ones(15), prim=far)
    assert np.all(Gg == 0.0)
    if case.startswith("supersonic"):
        np.testing.assert_allclose(Wg, Wf if case == "supersonic_inflow" else Wi, rtol=1e-14)
        return
    Rp_i, _, s_i, ut_i = _invariants(Wi, n)
    _, Rm_f, s_f, ut_f = _invariants(Wf, n)
    Rp_g, Rm_g, s_g, ut_g = _invariants(Wg, n)
    assert Rp_g == pytest.approx(Rp_i, rel=1e-13)
    assert Rm_g == pytest.approx(Rm_f, rel=1e-13)
    up_s, up_t = (s_i, ut_i) if case == "subsonic_outflow" else (s_f, ut_f)
    assert s_g == pytest.approx(up_s, rel=1e-12)
    np.testing.assert_allclose(ut_g, up_t, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind", ["slip", "noslip"])
def test_wall_ghost_gradients_are_the_mirrored_field(oracle, kind):
    """A linear interior field W(x) = W0 + G (x - xf) near a wall through xf with normal n: the
    ghost field is x -> ghost(W(R x)) (R the mirror across the wall plane), linear as well, and its
    gradient at the wall must be the ghost gradient.  Checked with exact differences of the linear
    map (the ghost state is linear in W for both wall kinds)."""
    k = oracle.BC_SLIP if kind == "slip" else oracle.BC_NOSLIP
    n = np.array([0.36, 0.48, 0.8])
    R = np.eye(3) - 2 * np.outer(n, n)
    rng = np.random.default_rng(8)
    W0 = cons(1.1, [0.3, -0.2, 0.1], 0.9)
    Gm = rng.normal(size=(5, 3)) * 0.2        # Gm[c, d] = dW_c/dx_d
    _, Gg = oracle.bc_ghost(k, n, W0, Gm.reshape(15))
    Gg = Gg.reshape(5, 3)
    h = 0.5
    for d in range(3):
        x = np.zeros(3)
        x[d] = h
        Wp, _ = oracle.bc_ghost(k, n, W0 + Gm @ (R @ x), None)
        Wm, _ = oracle.bc_ghost(k, n, W0 - Gm @ (R @ x), None)
        np.testing.assert_allclose((Wp - Wm) / (2 * h), Gg[:, d], rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ local and coarse time steps
@pytest.mark.parametrize("viscous", [False, True])
def test_local_dt_of_a_cube(oracle, viscous):
    """Cube of side h, uniform state: sum_p lambda_p S_p = h^2 (2(|u|+|v|+|w|) + 6c) + 12 mu h / rho."""
    n = 5
    h = 1.0 / n
    m = mg.periodic_hex_cube(n)
    M = oracle.Mesh(m)
    rho, u, p = 1.3, np.array([0.4, -0.25, 0.1]), 0.8
    W = np.repeat(cons(rho, u, p)[:, None], m.n_cells, 1)
    mu = 0.01 if viscous else 0.0
    par = oracle.params(cfl=0.7, viscous=viscous, mu=mu)
    c = np.sqrt(GAMMA * p / rho)
    ref = 0.7 * h ** 3 / (h * h * (2 * np.abs(u).sum() + 6 * c) + 12 * mu * h / rho)
    np.testing.assert_allclose(M.local_dt(par, W), ref, rtol=1e-13)


def test_coarse_dt_of_agglomerates(oracle):
    """Coarse step (R14): CFL |Omega_c| / sum over the agglomerate's outer faces of (|U.A| + c S), with
    A the summed area vectors and S the summed fine areas; for a uniform stream along x the faces'
    area vectors of one coarse face never have opposite x components, so the sum is
    c (outer fine area) + |u| (x-projected outer fine area), computed here from the fine faces."""
    m = mg.layered_box(8, 6, 4, lengths=(2.0, 1.5, 1.0), jitter=0.0)
    M = oracle.Mesh(m)
    H = oracle.Hierarchy(M, levels=2, passes=2, seed=1)
    lev = H.level(1)
    f2c = lev["f2c"]
    F = M.faces()
    rho, u, p = 1.0, 0.5, 1 / GAMMA
    c = np.sqrt(GAMMA * p / rho)
    nc = lev["n"]
    area = np.zeros(nc)
    xproj = np.zeros(nc)
    for f in range(M.n_faces):
        L, Rr = F["fl"][f], F["fr"][f]
        cl = f2c[L]
        if Rr >= 0 and f2c[Rr] == cl:
            continue
        for cc in ([cl] if Rr < 0 else [cl, f2c[Rr]]):
            area[cc] += F["area"][f]
            xproj[cc] += abs(F["avec"][f][0])
    Wc = np.repeat(cons(rho, [u, 0, 0], p)[:, None], nc, 1)
    par = oracle.params(cfl=0.5)
    ref = 0.5 * lev["V"] / (c * area + u * xproj)
    np.testing.assert_allclose(H.coarse_dt(par, 1, Wc), ref, rtol=1e-12)
    assert nc < m.n_cells
