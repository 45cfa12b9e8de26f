"""Discrete adjoint on top of the library's vector-Jacobian products.

* ``ResidualFunction``: the fine CGKS operator E(W, G, alpha) = (R, G_new,
  alpha_new) as a ``torch.autograd.Function``; forward is ``cgks_residual``,
  backward linearises at the forward state and applies ``cgks_vjp_residual``.
* ``gradients``: sensitivities of the wall force with respect to the inflow
  Mach number and the bump amplitude at a converged state, from the adjoint
  fixed point (``cgks_adjoint_solve``) plus the explicit dependence of the
  operator and of the objective on the parameter at the fixed state.

The explicit parameter partials are central differences of the operator and of
the objective evaluated at the *fixed* converged state (one residual evaluation
per side); the state sensitivity, which carries the converged solution's
response, comes entirely from the adjoint.  The bump parameter displaces the
mesh by linear blending in y: y' = y_0 + A exp(-25 (x - 1.5)^2) (1 - y_0) with
y_0 the unbumped node height, so meshes at A +- h share their topology.
"""
from __future__ import annotations

import numpy as np

from . import cgks as cg
from . import meshgen as mg


def _torch():
    import torch
    return torch


class ResidualFunction(_torch().autograd.Function):
    """(R, G_new, alpha_new) = E(W, G, alpha); gradients by the library's exact VJP."""

    @staticmethod
    def forward(ctx, W, G, alpha, solver):
        R, Gn, an = solver.residual(W, G, alpha, grad=True)
        ctx.solver = solver
        ctx.save_for_backward(W, G, alpha)
        return R, Gn, an

    @staticmethod
    def backward(ctx, bR, bG, bA):
        W, G, alpha = ctx.saved_tensors
        S = ctx.solver
        torch = _torch()
        S.linearize(W, G, alpha)
        N = S.n_cells
        bR = bR.contiguous() if bR is not None else torch.zeros(5, N, dtype=torch.float64, device=W.device)
        bG = bG.contiguous() if bG is not None else None
        bA = bA.contiguous() if bA is not None else None
        gW, gG, gA = S.vjp_residual(bR, bG, bA)
        return gW, gG, gA, None


def residual(solver, W, G, alpha):
    return ResidualFunction.apply(W, G, alpha, solver)


def _operator(S, W, G, al):
    R, Gn, an = S.residual(W, G, al, grad=True)
    return R, Gn, an


def _dot(cots, outs):
    return float(sum((c * o).sum() for c, o in zip(cots, outs)))


def explicit_partials(S_plus, S_minus, W, G, al, cots, tag, e, h):
    """Central differences at the fixed state of J and of cots . E with respect to one parameter."""
    torch = _torch()
    Jp = float(torch.dot(S_plus.wall_force(W, G, al, tag), torch.tensor(e, dtype=torch.float64, device=W.device)))
    Jm = float(torch.dot(S_minus.wall_force(W, G, al, tag), torch.tensor(e, dtype=torch.float64, device=W.device)))
    Ep = _operator(S_plus, W, G, al)
    Em = _operator(S_minus, W, G, al)
    dJ = (Jp - Jm) / (2 * h)
    dE = (_dot(cots, Ep) - _dot(cots, Em)) / (2 * h)
    return dJ, dE


def channel_solver(m, mach, gamma=1.4, agglomerate=True, **par):
    """Library solver on a bump-channel mesh with far field of Mach `mach` and slip walls."""
    S = cg.Solver(**par)
    S.set_mesh(m)
    # free stream rho = 1, p = 1/gamma: sound speed 1, so u = Mach
    prim = np.array([1.0, mach, 0.0, 0.0, 1.0 / gamma])
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        S.set_bc(tag, cg.BC_FARFIELD, prim)
    for tag in (mg.TAG_WALL_BOTTOM, mg.TAG_WALL_TOP, mg.TAG_WALL_SIDE):
        S.set_bc(tag, cg.BC_SLIP)
    if agglomerate:
        S.agglomerate()
    return S


def gradients(mesh_fn, amp, mach, W, G, al, tag=mg.TAG_WALL_BOTTOM, e=(1.0, 0.0, 0.0), h=1e-5, max_iter=40000,
              tol=1e-11, **par):
    """dJ/dMach and dJ/dA at the converged state (W, G, al) of mesh_fn(amp) at `mach`.

    mesh_fn(a) builds the mesh at bump amplitude a (same topology for every a).
    Returns a dict with the two gradients, the adjoint iteration count and history.
    """
    S = channel_solver(mesh_fn(amp), mach, **par)
    S.linearize(W, G, al)
    adj = S.adjoint_solve(tag, e, max_iter=max_iter, tol=tol)
    cots = (adj["cR"], adj["cG"], adj["cA"])
    out = {"adjoint_iterations": adj["iterations"], "adjoint_final_change": float(adj["hist"][-1])}
    # Mach: far-field state at M +- h on unagglomerated solvers (the coarse levels do not enter)
    Sp = channel_solver(mesh_fn(amp), mach + h, agglomerate=False, **par)
    Sm = channel_solver(mesh_fn(amp), mach - h, agglomerate=False, **par)
    dJ, dE = explicit_partials(Sp, Sm, W, G, al, cots, tag, e, h)
    out["dJ_dMach"] = dJ + dE
    out["dJ_dMach_explicit"] = dJ
    # bump amplitude: meshes at A +- h
    Sp = channel_solver(mesh_fn(amp + h), mach, agglomerate=False, **par)
    Sm = channel_solver(mesh_fn(amp - h), mach, agglomerate=False, **par)
    dJ, dE = explicit_partials(Sp, Sm, W, G, al, cots, tag, e, h)
    out["dJ_dA"] = dJ + dE
    out["dJ_dA_explicit"] = dJ
    out["hist"] = adj["hist"]
    return out


def converge(S, m, W=None, G=None, al=None, cycles=40000, tol=1e-13):
    """V-cycles from (W, G, al) (free stream when None) to a residual drop of tol."""
    torch = _torch()
    if W is None:
        W0, G0 = mg.uniform_state(m.n_cells)
        W = torch.from_numpy(W0).cuda()
        G = torch.from_numpy(G0).cuda()
        al = torch.ones(m.n_cells, dtype=torch.float64, device="cuda")
    hist, ok = S.vcycle(W, G, al, cycles, tol)
    return W, G, al, hist, ok
