"""ctypes wrapper of the CPU oracle (plain C, FP64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module; the GPU library never imports it and
shares no code with it.  Every array crossing this wrapper is numpy float64 /
int64 in the oracle's own layouts: cell fields component-major, W[c, i]
(5 x N) and G[3c+d, i] (15 x N).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

BC_SLIP, BC_NOSLIP, BC_FARFIELD = 1, 2, 3


class OmParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double), ("cfl", C.c_double),
                ("eps_tau", C.c_double), ("c_tau", C.c_double), ("weno_eps", C.c_double),
                ("gamma_lin", C.c_double), ("viscous", C.c_int), ("coarse_smoother", C.c_int),
                ("relax_sweeps", C.c_int), ("cfl_implicit", C.c_double), ("cycle_gamma", C.c_int)]


def params(gamma=1.4, mu=0.0, prandtl=1.0, cfl=0.5, eps_tau=0.01, c_tau=1.0, weno_eps=1e-5, gamma_lin=0.5,
           viscous=False, coarse_smoother=0, relax_sweeps=2, cfl_implicit=0.25, cycle_gamma=1) -> OmParams:
    """coarse_smoother 0: forward Euler on the coarse levels; 1: the implicit smoother of Sec. 4.3.
    cycle_gamma 1: V-cycle; 2: W-cycle (each coarser level visited twice per parent visit)."""
    return OmParams(gamma, mu, prandtl, cfl, eps_tau, c_tau, weno_eps, gamma_lin, int(bool(viscous)),
                    int(coarse_smoother), int(relax_sweeps), float(cfl_implicit), int(cycle_gamma))


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        P, I64, D = C.c_void_p, C.c_int64, C.c_double
        L.om_mesh_build.restype = C.c_void_p
        L.om_mesh_build.argtypes = [I64, P, I64, P, P, P, I64, P, P, P, P, C.c_char_p]
        L.om_mesh_free.argtypes = [P]
        L.om_mesh_sizes.argtypes = [P, P]
        L.om_mesh_cells.argtypes = [P, P, P, P]
        L.om_mesh_faces.argtypes = [P] + [P] * 11
        L.om_mesh_set_bc.argtypes = [P, C.c_int32, C.c_int, P]
        L.om_residual.argtypes = [P, P, P, P, P, P, P, P, P, P, I64, P]
        L.om_wall_force.argtypes = [P, P, P, P, P, C.c_int32, P, P]
        L.om_residual_norm.restype = D
        L.om_residual_norm.argtypes = [P, P]
        L.om_local_dt.argtypes = [P, P, P, P]
        L.om_step_fe.argtypes = [P, P, P, P, P, P, P]
        L.om_step_s2o4.argtypes = [P, P, D, P, P, P, P]
        L.om_reconstruct_all.argtypes = [P, P, P, P, P, P]
        L.om_gks_point_flat.argtypes = [P, P, P, P, D, P, P]
        L.om_kfvs_point.argtypes = [P, P, D, P]
        L.om_cf_point.restype = D
        L.om_cf_point.argtypes = [P, P, D]
        L.om_slopes_flat.argtypes = [D, P, D, D, P, P, P]
        L.om_monomial_moment.restype = D
        L.om_monomial_moment.argtypes = [P, D, D, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.om_bc_ghost_flat.argtypes = [C.c_int, P, P, P, P, D, P, P]
        L.om_skew_accept.argtypes = [D, D, P, P, D, P, P, D, D]
        L.om_face_hash.restype = C.c_uint64
        L.om_face_hash.argtypes = [C.c_uint64] * 4
        L.om_agglomerate_graph.restype = I64
        L.om_agglomerate_graph.argtypes = [I64, P, P, I64, P, P, P, P, P, C.c_uint64, C.c_int, D, D, P, P, P, P,
                                           P, P, P, P, P, P]
        L.om_hier_build.restype = C.c_void_p
        L.om_hier_build.argtypes = [P, C.c_int, C.c_int, C.c_uint64, D, D]
        L.om_hier_free.argtypes = [P]
        L.om_hier_level_size.restype = I64
        L.om_hier_level_size.argtypes = [P, C.c_int, P, P]
        L.om_hier_level_get.argtypes = [P, C.c_int, P, P, P, P, P, P, P]
        L.om_kfvs_residual.argtypes = [P, C.c_int, P, P, P]
        L.om_coarse_dt.argtypes = [P, C.c_int, P, P, P]
        L.om_coarse_implicit.argtypes = [P, C.c_int, P, P, P, P]
        L.om_hier_level_boundary.argtypes = [P, C.c_int, P, P, P]
        L.om_restrict.argtypes = [P, C.c_int, P, P, P, P]
        L.om_prolong.argtypes = [P, C.c_int, P, P]
        L.om_vcycle.argtypes = [P, P, P, P, P, P, P, P, P]
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


class OracleError(RuntimeError):
    pass


class Mesh:
    """Oracle mesh: connectivity and geometry computed by the oracle itself."""

    def __init__(self, m):
        L = lib()
        self._keep = [_f64(m.xyz), np.ascontiguousarray(m.ctype, np.uint8), _i64(m.cnode_ptr), _i64(m.cnode),
                      _i64(m.bnode_ptr), _i64(m.bnode), np.ascontiguousarray(m.btag, np.int32),
                      None if m.node_canon is None else _i64(m.node_canon)]
        xyz, ct, cp, cn, bp, bn, bt, canon = self._keep
        err = C.create_string_buffer(256)
        self.h = L.om_mesh_build(m.n_nodes, _p(xyz), m.n_cells, _p(ct), _p(cp), _p(cn), m.n_bfaces, _p(bp), _p(bn),
                                 _p(bt), _p(canon), err)
        if not self.h:
            raise OracleError(err.value.decode())
        s = np.zeros(4, np.int64)
        L.om_mesh_sizes(self.h, _p(s))
        self.n_cells, self.n_faces, self.n_int, self.n_nodes = (int(x) for x in s)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.om_mesh_free(self.h)
            self.h = None

    def cells(self):
        N = self.n_cells
        vol, cen, m2 = np.zeros(N), np.zeros((N, 3)), np.zeros((N, 6))
        lib().om_mesh_cells(self.h, _p(vol), _p(cen), _p(m2))
        return vol, cen, m2

    def faces(self):
        F = self.n_faces
        out = dict(fl=np.zeros(F, np.int64), fr=np.zeros(F, np.int64), tag=np.zeros(F, np.int32),
                   area=np.zeros(F), avec=np.zeros((F, 3)), fmom=np.zeros((F, 3)), shift=np.zeros((F, 3)),
                   ngp=np.zeros(F, np.int32), gpx=np.zeros((F, 4, 3)), gpw=np.zeros((F, 4)), gpn=np.zeros((F, 4, 3)))
        lib().om_mesh_faces(self.h, *[_p(out[k]) for k in ("fl", "fr", "tag", "area", "avec", "fmom", "shift", "ngp",
                                                           "gpx", "gpw", "gpn")])
        return out

    def set_bc(self, tag, kind, prim=None):
        pr = None if prim is None else _f64(prim)
        if lib().om_mesh_set_bc(self.h, int(tag), int(kind), _p(pr)):
            raise OracleError("bad tag")

    def local_dt(self, par, W):
        W = _f64(W)
        dt = np.zeros(self.n_cells)
        if lib().om_local_dt(self.h, C.byref(par), _p(W), _p(dt)):
            raise OracleError("non-positive time step")
        return dt

    def residual(self, par, W, G, alpha=None, sub=None):
        N = self.n_cells
        W, G = _f64(W), _f64(G)
        al = None if alpha is None else _f64(alpha)
        R, Gn, an, dt = np.zeros((5, N)), np.zeros((15, N)), np.zeros(N), np.zeros(N)
        bad = C.c_int64(-1)
        sb = None if sub is None else _i64(sub)
        e = lib().om_residual(self.h, C.byref(par), _p(W), _p(G), _p(al), _p(R), _p(Gn), _p(an), _p(dt), _p(sb),
                              0 if sb is None else sb.shape[0], C.byref(bad))
        if e:
            raise OracleError(f"residual failed ({e}) at cell {bad.value}")
        return R, Gn, an, dt

    def residual_norm(self, R):
        return lib().om_residual_norm(self.h, _p(_f64(R)))

    def wall_force(self, par, W, G, alpha, tag):
        """Force of the gas on the boundary faces with `tag` (3 components)."""
        out = np.zeros(3)
        bad = C.c_int64(-1)
        al = None if alpha is None else _f64(alpha)
        e = lib().om_wall_force(self.h, C.byref(par), _p(_f64(W)), _p(_f64(G)), _p(al), int(tag), _p(out),
                                C.byref(bad))
        if e:
            raise OracleError(f"wall force failed ({e}) at cell {bad.value}")
        return out

    def step_fe(self, par, W, G, alpha):
        bad = C.c_int64(-1)
        rn = C.c_double(0)
        e = lib().om_step_fe(self.h, C.byref(par), _p(W), _p(G), _p(alpha), C.byref(rn), C.byref(bad))
        if e:
            raise OracleError(f"step failed ({e}) at cell {bad.value}")
        return rn.value

    def step_s2o4(self, par, dt, W, G, alpha):
        bad = C.c_int64(-1)
        e = lib().om_step_s2o4(self.h, C.byref(par), float(dt), _p(W), _p(G), _p(alpha), C.byref(bad))
        if e:
            raise OracleError(f"step failed ({e}) at cell {bad.value}")

    def reconstruct(self, par, W, G, alpha=None):
        coef = np.zeros((self.n_cells, 5, 10))
        al = None if alpha is None else _f64(alpha)
        e = lib().om_reconstruct_all(self.h, C.byref(par), _p(_f64(W)), _p(_f64(G)), _p(al), _p(coef))
        if e:
            raise OracleError(f"reconstruction failed at cell {e - 1}")
        return coef


# ---------------------------------------------------------------- point kernels
def gks_point(Wl, dWl, Wr, dWr, dt, par):
    """BGK interface solution at one Gauss point, local frame (normal = x).
    dWl, dWr: (3, 5) gradients of the local-frame conservative variables."""
    out = np.zeros(30)
    e = lib().om_gks_point_flat(_p(_f64(Wl)), _p(_f64(dWl)), _p(_f64(Wr)), _p(_f64(dWr)), float(dt), C.byref(par),
                                _p(out))
    if e:
        raise OracleError(f"gks_point failed ({e})")
    return dict(F=out[0:5], Fint=out[5:10], Fhalf=out[10:15], Wdt=out[15:20], Whalf=out[20:25], Wc=out[25:30])


def kfvs_point(Wl, Wr, gamma=1.4):
    F = np.zeros(5)
    lib().om_kfvs_point(_p(_f64(Wl)), _p(_f64(Wr)), float(gamma), _p(F))
    return F


def cf_point(Wl, Wr, gamma=1.4):
    """Compression factor of one Gauss point from the two states in the face frame (normal = x)."""
    return lib().om_cf_point(_p(_f64(Wl)), _p(_f64(Wr)), float(gamma))


def slopes(rho, U, lam, K, dW):
    a, A = np.zeros((3, 5)), np.zeros(5)
    if lib().om_slopes_flat(float(rho), _p(_f64(U)), float(lam), float(K), _p(_f64(dW)), _p(a), _p(A)):
        raise OracleError("singular moment matrix")
    return a, A


def monomial_moment(U, lam, K, half, i, j, k, l):
    return lib().om_monomial_moment(_p(_f64(U)), float(lam), float(K), int(half), i, j, k, l)


def bc_ghost(kind, n, Wi, Gi=None, prim=None, gamma=1.4):
    Wg = np.zeros(5)
    Gg = None if Gi is None else np.zeros(15)
    lib().om_bc_ghost_flat(int(kind), _p(None if prim is None else _f64(prim)), _p(_f64(n)), _p(_f64(Wi)),
                           _p(None if Gi is None else _f64(Gi)), float(gamma), _p(Wg), _p(Gg))
    return Wg, Gg


def face_hash(a, b, nf, seed=1):
    return int(lib().om_face_hash(a, b, nf, seed))


def skew_accept(Va, Vb, Pa, Pb, S, M, A, delta, smin):
    return bool(lib().om_skew_accept(float(Va), float(Vb), _p(_f64(Pa)), _p(_f64(Pb)), float(S), _p(_f64(M)),
                                     _p(_f64(A)), float(delta), float(smin)))


# ---------------------------------------------------------------- agglomeration / multigrid
@dataclass
class Graph:
    V: np.ndarray      # (n,)
    P: np.ndarray      # (n, 3) first moments
    a: np.ndarray      # (m,) int64, a < b, lexicographic
    b: np.ndarray
    S: np.ndarray      # (m,)
    M: np.ndarray      # (m, 3)
    A: np.ndarray      # (m, 3)


def agglomerate_graph(g: Graph, seed=1, passes=3, delta=0.25, smin=np.sin(np.deg2rad(10.0))):
    n, m = g.V.shape[0], g.a.shape[0]
    f2c = np.zeros(n, np.int64)
    Vo, Po = np.zeros(n), np.zeros((n, 3))
    ao, bo = np.zeros(max(m, 1), np.int64), np.zeros(max(m, 1), np.int64)
    So, Mo, Ao = np.zeros(max(m, 1)), np.zeros((max(m, 1), 3)), np.zeros((max(m, 1), 3))
    mo = C.c_int64(0)
    stats = np.zeros((max(passes, 1), 4), np.int64)
    keep = [_f64(g.V), _f64(g.P), _i64(g.a), _i64(g.b), _f64(g.S), _f64(g.M), _f64(g.A)]
    nc = lib().om_agglomerate_graph(n, *[_p(k) for k in keep[:2]], m, *[_p(k) for k in keep[2:]], int(seed),
                                    int(passes), float(delta), float(smin), _p(f2c), _p(Vo), _p(Po), C.byref(mo),
                                    _p(ao), _p(bo), _p(So), _p(Mo), _p(Ao), _p(stats))
    mo = mo.value
    return f2c, Graph(Vo[:nc], Po[:nc], ao[:mo], bo[:mo], So[:mo], Mo[:mo], Ao[:mo]), stats


class Hierarchy:
    def __init__(self, mesh: Mesh, levels=3, passes=3, seed=1, delta=0.25, smin=np.sin(np.deg2rad(10.0))):
        self.mesh = mesh
        self.levels = levels
        self.h = lib().om_hier_build(mesh.h, int(levels), int(passes), int(seed), float(delta), float(smin))

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.om_hier_free(self.h)
            self.h = None

    def size(self, l):
        m, nb = C.c_int64(0), C.c_int64(0)
        n = lib().om_hier_level_size(self.h, int(l), C.byref(m), C.byref(nb))
        return int(n), m.value, nb.value

    def level(self, l):
        n, m, nb = self.size(l)
        nf = self.size(l - 1)[0] if l > 0 else 0
        f2c = np.zeros(nf, np.int64) if l > 0 else None
        V, P = np.zeros(n), np.zeros((n, 3))
        a, b, A = np.zeros(m, np.int64), np.zeros(m, np.int64), np.zeros((m, 3))
        stats = np.zeros((16, 4), np.int64)
        lib().om_hier_level_get(self.h, int(l), _p(f2c), _p(V), _p(P), _p(a), _p(b), _p(A), _p(stats))
        return dict(n=n, m=m, nb=nb, f2c=f2c, V=V, P=P, a=a, b=b, A=A, stats=stats)

    def level_boundary(self, l):
        """Boundary faces of level l: owner cell, boundary tag, outward area vector."""
        n, m, nb = self.size(l)
        bown, btag, bA = np.zeros(nb, np.int64), np.zeros(nb, np.int32), np.zeros((nb, 3))
        lib().om_hier_level_boundary(self.h, int(l), _p(bown), _p(btag), _p(bA))
        return bown, btag, bA

    def kfvs_residual(self, par, l, W):
        n = self.size(l)[0]
        R = np.zeros((5, n))
        lib().om_kfvs_residual(self.h, int(l), C.byref(par), _p(_f64(W)), _p(R))
        return R

    def coarse_dt(self, par, l, W):
        n = self.size(l)[0]
        dt = np.zeros(n)
        lib().om_coarse_dt(self.h, int(l), C.byref(par), _p(_f64(W)), _p(dt))
        return dt

    def coarse_implicit(self, par, l, W, rhs):
        """Increment dU of the implicit coarse smoother (Sec. 4.3) at state W for right-hand side rhs."""
        n = self.size(l)[0]
        dU = np.zeros((5, n))
        lib().om_coarse_implicit(self.h, int(l), C.byref(par), _p(_f64(W)), _p(_f64(rhs)), _p(dU))
        return dU

    def restrict(self, l, Wf, Rf):
        n = self.size(l)[0]
        Wc, Rc = np.zeros((5, n)), np.zeros((5, n))
        lib().om_restrict(self.h, int(l), _p(_f64(Wf)), _p(_f64(Rf)), _p(Wc), _p(Rc))
        return Wc, Rc

    def prolong(self, l, dWc, Wf):
        Wf = _f64(Wf).copy()
        lib().om_prolong(self.h, int(l), _p(_f64(dWc)), _p(Wf))
        return Wf

    def vcycle(self, par, W, G, alpha, nu_pre=None, nu_post=None):
        pre = None if nu_pre is None else np.ascontiguousarray(nu_pre, np.int32)
        post = None if nu_post is None else np.ascontiguousarray(nu_post, np.int32)
        rn = C.c_double(0)
        bad = C.c_int64(-1)
        e = lib().om_vcycle(self.h, C.byref(par), _p(pre), _p(post), _p(W), _p(G), _p(alpha), C.byref(rn),
                            C.byref(bad))
        if e:
            raise OracleError(f"vcycle failed ({e}) at cell {bad.value}")
        return rn.value
