"""Discrete adjoint on top of the library's vector-Jacobian products.

* ``ResidualFunction``: the fine CGKS operator E(W, G, alpha) = (R, G_new,
  alpha_new) as a ``torch.autograd.Function``; forward is ``cgks_residual``,
  backward linearises at the forward state and applies ``cgks_vjp_residual``.
* ``gradients``: sensitivities of the wall force with respect to the inflow
  Mach number and the bump amplitude at a converged state, from the library's
  adjoint solve (``cgks_adjoint_solve`` with the parameter directions of
  ``cgks_set_param_directions``); this module only describes the two
  parameters: the far-field velocity of the inlet and outlet tags (Mach), and
  the node displacement of the bump blending y' = y_0 + A exp(-25 (x - 1.5)^2)
  (1 - y_0), y_0 the unbumped node height.
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


def bump_direction(mesh_fn, amp, delta=0.01):
    """Node displacement per unit bump amplitude: the generator places every node affinely in the
    amplitude (grid nodes by the blending y' = y0 + A b(x) (1 - y0), pyramid centres as means of
    blended corners), so the difference of its meshes at amp +- delta is exact up to rounding."""
    return (mesh_fn(amp + delta).xyz - mesh_fn(amp - delta).xyz) / (2.0 * delta)


def mach_direction(gamma=1.4):
    """Far-field primitive change per unit Mach number (rho = 1 and p = 1/gamma fixed, so the sound
    speed is 1 and u = Mach) on the inlet and outlet tags."""
    d = np.zeros((64, 5))
    for tag in (mg.TAG_INLET, mg.TAG_OUTLET):
        d[tag, 1] = 1.0
    return d


def gradients(S, mesh_fn, amp, mach, W, G, al, tag=mg.TAG_WALL_BOTTOM, e=(1.0, 0.0, 0.0), max_iter=40000,
              tol=1e-11, step=1e-6):
    """dJ/dMach and dJ/dA at the converged state (W, G, al) of the bump channel mesh_fn(amp)
    at `mach`, from the library's adjoint solve with two parameter directions: the far-field
    velocity of the inlet and outlet tags, and the bump blending of the mesh nodes.
    Returns a dict with the two gradients, the adjoint iteration count and history."""
    dprim = np.stack([mach_direction(), np.zeros((64, 5))])
    d = bump_direction(mesh_fn, amp)
    dxyz = np.stack([np.zeros_like(d), d])
    S.set_param_directions(dprim, dxyz, step)
    S.linearize(W, G, al)
    adj = S.adjoint_solve(tag, e, max_iter=max_iter, tol=tol)
    return {"dJ_dMach": float(adj["dJ_dparams"][0]), "dJ_dA": float(adj["dJ_dparams"][1]),
            "adjoint_iterations": adj["iterations"], "adjoint_final_change": float(adj["hist"][-1]),
            "hist": adj["hist"]}


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
