"""Oracle pins of the implicit coarse smoother (paper Sec. 4.3).

The smoother solves D_i dU_i + sum_p [F-(U_p + dU_p) - F-(U_p)] S_p = rhs_i by point
relaxation, with D_i = |Omega_i|/dt_i + 1/2 sum_p lambda_p S_p.  For a small right-hand
side the nonlinear flux difference equals the Jacobian product A-_p dU_p to second order,
so after enough relaxation sweeps the increment must match the solution of the linear
system assembled here from the textbook flux Jacobian of the Euler equations (written out
in this file, independent of the oracle) and solved densely.  A periodic mesh has no
boundary faces, so every term of the system is a pair term.
"""
import numpy as np
import pytest

from paper_2402_02075_amd import meshgen as mg

GAMMA = 1.4


def euler_flux(U, n, g=GAMMA):
    rho, m, E = U[0], U[1:4], U[4]
    u = m / rho
    p = (g - 1.0) * (E - 0.5 * rho * u @ u)
    un = u @ n
    return np.concatenate([[rho * un], m * un + p * n, [(E + p) * un]])


def euler_jacobian(U, n, g=GAMMA):
    """dF_n/dU of the 3-D Euler equations in conservative variables (standard closed form)."""
    rho, E = U[0], U[4]
    u = U[1:4] / rho
    q2 = u @ u
    p = (g - 1.0) * (E - 0.5 * rho * q2)
    H = (E + p) / rho
    phi2 = 0.5 * (g - 1.0) * q2
    V = u @ n
    A = np.zeros((5, 5))
    A[0, 1:4] = n
    for i in range(3):
        A[1 + i, 0] = phi2 * n[i] - u[i] * V
        for j in range(3):
            A[1 + i, 1 + j] = u[i] * n[j] - (g - 1.0) * u[j] * n[i] + (V if i == j else 0.0)
        A[1 + i, 4] = (g - 1.0) * n[i]
    A[4, 0] = V * (phi2 - H)
    A[4, 1:4] = H * n - (g - 1.0) * u * V
    A[4, 4] = g * V
    return A


def radius(U, n, g=GAMMA):
    rho = U[0]
    u = U[1:4] / rho
    p = (g - 1.0) * (U[4] - 0.5 * rho * u @ u)
    return abs(u @ n) + np.sqrt(g * p / rho)


def test_textbook_jacobian_self_check():
    """The Euler flux is homogeneous of degree one: A(U) U = F_n(U); and A matches differences."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        U = np.array([1.2, 0.3, -0.2, 0.1, 2.5]) + 0.05 * rng.standard_normal(5)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        A = euler_jacobian(U, n)
        np.testing.assert_allclose(A @ U, euler_flux(U, n), rtol=1e-13, atol=1e-13)
        h = 1e-6
        fd = np.stack([(euler_flux(U + h * e, n) - euler_flux(U - h * e, n)) / (2 * h) for e in np.eye(5)], axis=1)
        np.testing.assert_allclose(A, fd, rtol=1e-7, atol=1e-8)


@pytest.fixture(scope="module")
def periodic(oracle):
    m = mg.periodic_mixed_box(6, jitter=0.1, seed=3)
    M = oracle.Mesh(m)
    H = oracle.Hierarchy(M, levels=2, passes=2, seed=1)
    return m, M, H


def _assemble(oracle, H, par, l, W):
    """Dense matrix of the linearised implicit system on level l (periodic: pair terms only)."""
    L = H.level(l)
    n = L["n"]
    # the implicit step's local dt is the coarse local step at the implicit CFL number
    dt = H.coarse_dt(oracle.params(cfl=par.cfl_implicit), l, W)
    M = np.zeros((5 * n, 5 * n))
    diag = L["V"] / dt
    for j in range(L["m"]):
        A = L["A"][j]
        S = np.linalg.norm(A)
        if S == 0:
            continue
        nn = A / S
        a, b = L["a"][j], L["b"][j]
        lam = max(radius(W[:, a], nn), radius(W[:, b], nn))
        diag[a] += 0.5 * lam * S
        diag[b] += 0.5 * lam * S
        # row a, column b: outward normal +n; row b, column a: outward normal -n
        M[5 * a:5 * a + 5, 5 * b:5 * b + 5] += 0.5 * S * (euler_jacobian(W[:, b], nn) - lam * np.eye(5))
        M[5 * b:5 * b + 5, 5 * a:5 * a + 5] += 0.5 * S * (euler_jacobian(W[:, a], -nn) - lam * np.eye(5))
    for i in range(n):
        M[5 * i:5 * i + 5, 5 * i:5 * i + 5] += diag[i] * np.eye(5)
    return M, diag


@pytest.mark.parametrize("sweeps", [0, 80])
def test_implicit_increment_solves_linearised_system(oracle, periodic, sweeps):
    m, M, H = periodic
    l = 1
    n = H.size(l)[0]
    x = mg.cell_node_mean(m)
    W = mg.random_smooth_state(x, seed=11, amp=0.1)
    Wc, _ = H.restrict(l, W, np.zeros_like(W))
    rng = np.random.default_rng(5)
    rhs = 1e-7 * rng.standard_normal((5, n)) * np.abs(Wc).max(axis=1, keepdims=True)
    par = oracle.params(coarse_smoother=1, relax_sweeps=sweeps, cfl_implicit=1.0)
    dU = H.coarse_implicit(par, l, Wc, rhs)
    Mat, diag = _assemble(oracle, H, par, l, Wc)
    if sweeps == 0:
        # diagonal only: dU = rhs / (|Omega|/dt + 1/2 sum lambda S)
        np.testing.assert_allclose(dU, rhs / diag[None, :], rtol=1e-12, atol=0)
        return
    ref = np.linalg.solve(Mat, rhs.T.reshape(-1)).reshape(n, 5).T
    err = np.abs(dU - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert err.max() < 1e-5, err


def test_implicit_boundary_terms(oracle):
    """Channel with far-field and slip boundaries: each boundary face adds lambda S / 2 to its
    owner's diagonal, lambda the larger radius of owner and ghost state; no off-diagonal term."""
    m = mg.bump_channel(12, 6, 4, n_prism=2, n_pyr=2, jitter=0.05, seed=2, amp=0.05)
    M = oracle.Mesh(m)
    prim = np.array([1.0, 0.5, 0.0, 0.0, 1 / 1.4])
    kinds = {}
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        M.set_bc(tag, oracle.BC_FARFIELD, prim)
        kinds[tag] = (oracle.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        M.set_bc(tag, oracle.BC_SLIP)
        kinds[tag] = (oracle.BC_SLIP, None)
    H = oracle.Hierarchy(M, levels=2, passes=2, seed=1)
    l = 1
    n = H.size(l)[0]
    W = mg.random_smooth_state(mg.cell_node_mean(m), seed=12, amp=0.1)
    Wc, _ = H.restrict(l, W, np.zeros_like(W))
    rhs = 1e-7 * np.random.default_rng(6).standard_normal((5, n)) * np.abs(Wc).max(axis=1, keepdims=True)
    par = oracle.params(coarse_smoother=1, relax_sweeps=80, cfl_implicit=1.0)
    dU = H.coarse_implicit(par, l, Wc, rhs)
    Mat, diag = _assemble(oracle, H, par, l, Wc)
    bown, btag, bA = H.level_boundary(l)
    assert len(bown) > 0
    for o, tag, A in zip(bown, btag, bA):
        S = np.linalg.norm(A)
        nn = A / S
        kind, pr = kinds[int(tag) & 63]
        Wg, _ = oracle.bc_ghost(kind, nn, Wc[:, o], prim=pr)
        lam = max(radius(Wc[:, o], nn), radius(Wg, nn))
        Mat[5 * o:5 * o + 5, 5 * o:5 * o + 5] += 0.5 * lam * S * np.eye(5)
    ref = np.linalg.solve(Mat, rhs.T.reshape(-1)).reshape(n, 5).T
    err = np.abs(dU - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert err.max() < 1e-5, err
