"""Pins of the oracle's kinetic core against facts fixed outside it.

Moments are checked against brute-force quadrature, micro-slopes against their
defining moment equations evaluated by quadrature, the BGK interface solution
against closed forms of the Chapman-Enskog limit (Euler flux, Navier-Stokes
shear stress and heat flux), its free-transport limit (KFVS), rotation and
mirror symmetry.  Paper: Sec. 2.1 (BGK, psi, K), Sec. 2.3 (Eqs. co, co-moment,
compatibility2, 2nd-flux, collision times).
"""
import numpy as np
import pytest
from scipy import integrate

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)  # = 2 internal degrees of freedom


def maxw_quad(U, lam, n_pts=40):
    """Gauss-Hermite nodes/weights for the normalised 1-D Maxwellian around U."""
    x, w = np.polynomial.hermite.hermgauss(n_pts)
    return U + x / np.sqrt(lam), w / np.sqrt(np.pi)


def euler_flux(W, gamma=GAMMA):
    rho, m, E = W[0], W[1:4], W[4]
    u = m / rho
    p = (gamma - 1) * (E - 0.5 * rho * u @ u)
    return np.array([m[0], m[0] * u[0] + p, m[0] * u[1], m[0] * u[2], u[0] * (E + p)])


def cons(rho, u, p, gamma=GAMMA):
    u = np.asarray(u, float)
    return np.array([rho, *(rho * u), p / (gamma - 1) + 0.5 * rho * u @ u])


def test_full_moments_vs_gauss_hermite(oracle):
    rng = np.random.default_rng(0)
    for _ in range(5):
        U = rng.normal(size=3)
        lam = rng.uniform(0.3, 3.0)
        xs = [maxw_quad(U[d], lam) for d in range(3)]
        # internal dof: K = 2 -> 2-D Gaussian of variance 1/(2 lam) per dof
        xi, wxi = maxw_quad(0.0, lam)
        for (i, j, k, l) in [(0, 0, 0, 0), (1, 0, 0, 0), (2, 1, 0, 0), (3, 2, 1, 0), (6, 0, 0, 0), (2, 2, 2, 1),
                             (1, 0, 3, 2), (0, 0, 0, 2)]:
            mu = np.sum(xs[0][1] * xs[0][0] ** i)
            mv = np.sum(xs[1][1] * xs[1][0] ** j)
            mw = np.sum(xs[2][1] * xs[2][0] ** k)
            # <xi^(2l)> with xi^2 = xi1^2 + xi2^2
            X1, X2 = np.meshgrid(xi, xi, indexing="ij")
            WW = np.outer(wxi, wxi)
            mx = np.sum(WW * (X1 ** 2 + X2 ** 2) ** l)
            ref = mu * mv * mw * mx
            got = oracle.monomial_moment(U, lam, K, 0, i, j, k, l)
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-13)


def test_half_moments_vs_quadrature(oracle):
    for U, lam in [(0.3, 1.2), (-0.7, 0.5), (2.0, 2.0), (0.0, 1.0)]:
        for half in (+1, -1):
            for n in range(7):
                f = lambda u: u ** n * np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)
                lo, hi = (0, np.inf) if half > 0 else (-np.inf, 0)
                ref, _ = integrate.quad(f, lo, hi, epsabs=1e-15, epsrel=1e-13, limit=200)
                got = oracle.monomial_moment([U, 0.0, 0.0], lam, K, half, n, 0, 0, 0)
                assert got == pytest.approx(ref, rel=1e-11, abs=1e-14)
        # the two half spaces add up to the full space
        for n in range(7):
            s = sum(oracle.monomial_moment([U, 0.1, -0.2], lam, K, h, n, 1, 1, 1) for h in (+1, -1))
            assert s == pytest.approx(oracle.monomial_moment([U, 0.1, -0.2], lam, K, 0, n, 1, 1, 1), rel=1e-13,
                                      abs=1e-15)


def _psi_grid(U, lam, n=12):
    """5-D Gauss-Hermite grid (u, v, w, xi1, xi2) of the normalised Maxwellian."""
    pts = [maxw_quad(U[d], lam, n) for d in range(3)] + [maxw_quad(0.0, lam, n)] * 2
    grids = np.meshgrid(*[p[0] for p in pts], indexing="ij")
    wts = np.ones_like(grids[0])
    for d, p in enumerate(pts):
        shape = [1] * 5
        shape[d] = n
        wts = wts * p[1].reshape(shape)
    u, v, w, x1, x2 = grids
    psi = np.stack([np.ones_like(u), u, v, w, 0.5 * (u * u + v * v + w * w + x1 * x1 + x2 * x2)])
    return psi, wts, (u, v, w)


def test_micro_slopes_satisfy_moment_equations(oracle):
    rng = np.random.default_rng(1)
    rho, U, lam = 1.3, np.array([0.4, -0.2, 0.1]), 0.8
    dW = rng.normal(size=(3, 5))
    a, A = oracle.slopes(rho, U, lam, K, dW)
    psi, wts, vel = _psi_grid(U, lam)
    for j in range(3):
        s = np.tensordot(a[j], psi, axes=1)
        got = rho * np.array([np.sum(wts * psi[al] * s) for al in range(5)])
        np.testing.assert_allclose(got, dW[j], rtol=1e-11, atol=1e-12)
    # compatibility <(A + a.u) psi> = 0
    tot = np.tensordot(A, psi, axes=1) + sum(vel[j] * np.tensordot(a[j], psi, axes=1) for j in range(3))
    res = np.array([np.sum(wts * psi[al] * tot) for al in range(5)])
    np.testing.assert_allclose(res, 0.0, atol=1e-11)


def _euler_flux_dir(W, j, gamma=GAMMA):
    """Euler flux along axis j (works on complex W for complex-step derivatives)."""
    rho, m, E = W[0], W[1:4], W[4]
    u = m / rho
    p = (gamma - 1) * (E - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]))
    e = np.zeros(3)
    e[j] = 1.0
    return np.concatenate([[m[j]], m * u[j] + p * e, [u[j] * (E + p)]])


def test_time_slope_is_euler_time_derivative(oracle):
    """The time slope A of the compatibility condition, Eq. (co), moves the conserved variables at
    the rate the Euler equations give: rho <A psi> = -sum_j (dF_j/dW) dW_j.  The flux Jacobians here
    are complex-step derivatives of the Euler fluxes, so the pin is independent of the moment
    algebra; it fails for a wrong K, a wrong moment of order three or four, or a sign slip."""
    rng = np.random.default_rng(4)
    for _ in range(4):
        rho, lam = rng.uniform(0.5, 2.0), rng.uniform(0.4, 2.5)
        U = rng.normal(scale=0.6, size=3)
        W = cons(rho, U, rho / (2 * lam))
        dW = rng.normal(size=(3, 5))
        a, A = oracle.slopes(rho, U, lam, K, dW)
        ref = np.zeros(5)
        h = 1e-30
        for j in range(3):
            jac = np.stack([_euler_flux_dir(W + 1j * h * e, j).imag / h for e in np.eye(5)], axis=1)
            ref -= jac @ dW[j]
        psi, wts, _ = _psi_grid(U, lam)
        s = np.tensordot(A, psi, axes=1)
        got = rho * np.array([np.sum(wts * psi[al] * s) for al in range(5)])
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("viscous", [False, True])
@pytest.mark.parametrize("dt", [1e-3, 0.05])
def test_uniform_state_gives_euler_flux(oracle, viscous, dt):
    W = cons(1.2, [0.3, -0.4, 0.2], 0.9)
    Z = np.zeros((3, 5))
    par = oracle.params(viscous=viscous, mu=0.01 if viscous else 0.0, prandtl=0.72 if viscous else 1.0)
    out = oracle.gks_point(W, Z, W, Z, dt, par)
    np.testing.assert_allclose(out["F"], euler_flux(W), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(out["Fint"], dt * euler_flux(W), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["Fhalf"], 0.5 * dt * euler_flux(W), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["Wdt"], W, rtol=1e-13)
    np.testing.assert_allclose(out["Wc"], W, rtol=1e-13)


@pytest.mark.parametrize("dt", [1e-4, 0.02, 0.3])
def test_shear_stress_is_navier_stokes(oracle, dt):
    """Continuous data with dV/dx = s at U = 0: momentum flux -mu s exactly (CE limit of Eq. 2nd-flux)."""
    mu, s = 0.02, 0.7
    W = cons(1.0, [0.0, 0.0, 0.0], 1.0)
    dW = np.zeros((3, 5))
    dW[0, 2] = s  # d(rho v)/dx
    par = oracle.params(viscous=True, mu=mu)
    out = oracle.gks_point(W, dW, W, dW, dt, par)
    np.testing.assert_allclose(out["F"], [0.0, 1.0, -mu * s, 0.0, 0.0], atol=1e-14)


@pytest.mark.parametrize("pr", [1.0, 0.72])
def test_heat_flux_is_fourier_with_prandtl_fix(oracle, pr):
    """dp/dx = q at rest, rho uniform: energy flux -> -mu gamma/((gamma-1) Pr) q as dt -> 0."""
    mu, q = 0.01, 0.3
    W = cons(1.0, [0.0, 0.0, 0.0], 1.0)
    dW = np.zeros((3, 5))
    dW[0, 4] = q / (GAMMA - 1)
    par = oracle.params(viscous=True, mu=mu, prandtl=pr)
    out = oracle.gks_point(W, dW, W, dW, 1e-9, par)
    assert out["F"][4] == pytest.approx(-mu * GAMMA / ((GAMMA - 1) * pr) * q, rel=1e-7)
    assert out["F"][1] == pytest.approx(1.0, rel=1e-9)


def test_interface_value_of_smooth_advection(oracle):
    """Density wave advected at U: W(t) = W - t U dW/dx exactly (compatibility, inviscid)."""
    U, r = 0.6, 0.25
    W = cons(1.1, [U, 0.0, 0.0], 1.0)
    dW = np.zeros((3, 5))
    dW[0] = np.array([r, r * U, 0.0, 0.0, 0.5 * U * U * r])
    dt = 0.03
    out = oracle.gks_point(W, dW, W, dW, dt, oracle.params())
    np.testing.assert_allclose(out["Wdt"], W - dt * U * dW[0], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["Whalf"], W - 0.5 * dt * U * dW[0], rtol=1e-13, atol=1e-15)
    # time-averaged flux of linear advection: F(W(t)) averaged over [0, dt]
    Fm = euler_flux(W - 0.5 * dt * U * dW[0])
    np.testing.assert_allclose(out["F"], Fm, rtol=1e-12, atol=1e-14)


def test_free_transport_limit_is_kfvs(oracle):
    """tau_n >> dt (huge C): f -> free transport of the two half Maxwellians."""
    Wl = cons(1.0, [0.2, 0.1, 0.0], 1.0)
    Wr = cons(0.5, [-0.1, 0.0, 0.3], 0.4)
    Z = np.zeros((3, 5))
    out = oracle.gks_point(Wl, Z, Wr, Z, 1e-3, oracle.params(c_tau=1e9))
    np.testing.assert_allclose(out["F"], oracle.kfvs_point(Wl, Wr), rtol=1e-8, atol=1e-10)
    # KFVS with equal states is the Euler flux
    np.testing.assert_allclose(oracle.kfvs_point(Wl, Wl), euler_flux(Wl), rtol=1e-13, atol=1e-15)


def test_kfvs_vs_half_space_quadrature(oracle):
    Wl = cons(1.0, [0.2, 0.1, 0.0], 1.0)
    Wr = cons(0.5, [-0.1, 0.0, 0.3], 0.4)
    ref = np.zeros(5)
    for Wside, half in ((Wl, 1), (Wr, -1)):
        rho = Wside[0]
        u = Wside[1:4] / rho
        p = (GAMMA - 1) * (Wside[4] - 0.5 * rho * u @ u)
        lam = rho / (2 * p)
        g1 = lambda x: np.sqrt(lam / np.pi) * np.exp(-lam * (x - u[0]) ** 2)
        lo, hi = (0, np.inf) if half > 0 else (-np.inf, 0)
        m = [integrate.quad(lambda x, n=n: x ** n * g1(x), lo, hi, epsabs=1e-15, epsrel=1e-13)[0] for n in range(4)]
        ev2, ew2 = u[1] ** 2 + 1 / (2 * lam), u[2] ** 2 + 1 / (2 * lam)
        exi = K / (2 * lam)
        ref += rho * np.array([m[1], m[2], m[1] * u[1], m[1] * u[2], 0.5 * (m[3] + m[1] * (ev2 + ew2 + exi))])
    np.testing.assert_allclose(oracle.kfvs_point(Wl, Wr), ref, rtol=1e-11)


def _rot_tangential(W, dW, th):
    c, s = np.cos(th), np.sin(th)
    R = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    W2 = W.copy()
    W2[1:4] = R @ W[1:4]
    dW2 = np.zeros_like(dW)
    # gradient directions (rows) and momentum components both rotate
    D = R @ dW  # direction rotation
    D[:, 1:4] = D[:, 1:4] @ R.T
    dW2[:] = D
    return W2, dW2, R


def test_rotation_about_normal(oracle):
    rng = np.random.default_rng(5)
    Wl = cons(1.0, [0.2, 0.3, -0.1], 1.0)
    Wr = cons(0.9, [0.1, -0.2, 0.2], 0.8)
    dWl, dWr = rng.normal(size=(3, 5)) * 0.1, rng.normal(size=(3, 5)) * 0.1
    par = oracle.params(viscous=True, mu=0.01, prandtl=0.72)
    a = oracle.gks_point(Wl, dWl, Wr, dWr, 0.02, par)
    th = 0.7
    Wl2, dWl2, R = _rot_tangential(Wl, dWl, th)
    Wr2, dWr2, _ = _rot_tangential(Wr, dWr, th)
    b = oracle.gks_point(Wl2, dWl2, Wr2, dWr2, 0.02, par)
    for key in ("F", "Wdt", "Wc"):
        exp = a[key].copy()
        exp[1:4] = R @ a[key][1:4]
        np.testing.assert_allclose(b[key], exp, rtol=1e-11, atol=1e-13)


def test_mirror_symmetry(oracle):
    """Swap sides and reverse the normal: the flux changes sign (mirror x -> -x)."""
    rng = np.random.default_rng(6)
    Wl = cons(1.0, [0.2, 0.3, -0.1], 1.0)
    Wr = cons(0.7, [-0.1, -0.2, 0.2], 0.6)
    dWl, dWr = rng.normal(size=(3, 5)) * 0.1, rng.normal(size=(3, 5)) * 0.1
    par = oracle.params()

    def mirror(W, dW):
        W2 = W.copy()
        W2[1] = -W[1]
        dW2 = dW.copy()
        dW2[0] = -dW[0]      # d/dx flips
        dW2[:, 1] = -dW2[:, 1]  # x-momentum flips
        return W2, dW2

    a = oracle.gks_point(Wl, dWl, Wr, dWr, 0.02, par)
    Wl2, dWl2 = mirror(Wr, dWr)
    Wr2, dWr2 = mirror(Wl, dWl)
    b = oracle.gks_point(Wl2, dWl2, Wr2, dWr2, 0.02, par)
    exp = a["F"].copy()
    exp[[0, 2, 3, 4]] *= -1.0   # mass, tangential momentum, energy flux reverse; normal momentum flux keeps sign
    np.testing.assert_allclose(b["F"], exp, rtol=1e-11, atol=1e-13)


def test_ghost_states(oracle):
    n = np.array([0.6, 0.8, 0.0])
    W = cons(1.1, [0.3, 0.2, 0.1], 0.9)
    G = np.arange(15, dtype=float) * 0.01
    Wg, Gg = oracle.bc_ghost(oracle.BC_SLIP, n, W, G)
    assert Wg[0] == W[0] and Wg[4] == W[4]
    assert (W[1:4] + Wg[1:4]) @ n == pytest.approx(0.0, abs=1e-15)
    Wg, _ = oracle.bc_ghost(oracle.BC_NOSLIP, n, W, G)
    np.testing.assert_allclose(Wg[1:4], -W[1:4])
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1 / 1.4])
    Wf = cons(1.0, [0.5, 0.0, 0.0], 1 / 1.4)
    for nn in (np.array([1.0, 0, 0]), np.array([-1.0, 0, 0]), n):
        Wg, Gg = oracle.bc_ghost(oracle.BC_FARFIELD, nn, Wf, G, prim=prim)
        np.testing.assert_allclose(Wg, Wf, rtol=1e-13, atol=1e-15)
        assert np.all(Gg == 0)
