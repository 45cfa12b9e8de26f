"""Thin Python binding of libcgks (the C ABI in include/cgks.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libcgks.so.  PyTorch supplies device memory and the current HIP stream.  If the
shared library is missing the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CGKS_LIBRARY") or os.path.join(HERE, "libcgks.so")

OK, E_ARG, E_MESH, E_DEVICE, E_NONFINITE, E_PHYS, E_NOCONV, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
BC_SLIP, BC_NOSLIP_ADIABATIC, BC_FARFIELD = 1, 2, 3

# symbols the header declares (checked by the CPU test suite)
EXPORTS = ["cgks_default_params", "cgks_create", "cgks_destroy", "cgks_last_error", "cgks_set_params",
           "cgks_set_stream", "cgks_set_mesh", "cgks_set_bc", "cgks_mesh_info", "cgks_geometry", "cgks_local_dt",
           "cgks_reconstruct", "cgks_residual", "cgks_step", "cgks_check", "cgks_residual_norm",
           "cgks_agglomerate_graph", "cgks_agglomerate", "cgks_level_map", "cgks_kfvs_residual", "cgks_restrict",
           "cgks_prolong", "cgks_vcycle", "cgks_timing", "cgks_wall_force", "cgks_linearize", "cgks_vjp_residual",
           "cgks_vjp_wall_force", "cgks_vjp_kfvs", "cgks_adjoint_solve", "cgks_coarse_implicit", "cgks_cell_order",
           "cgks_residual_noalloc", "cgks_set_param_directions", "cgks_jvp_residual",
           "cgks_residual_host", "cgks_vcycle_host"]


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double), ("cfl", C.c_double),
                ("eps_tau", C.c_double), ("c_tau", C.c_double), ("weno_eps", C.c_double), ("gamma_lin", C.c_double),
                ("skew_delta", C.c_double), ("skew_sin", C.c_double), ("viscous", C.c_int32), ("levels", C.c_int32),
                ("passes", C.c_int32), ("precision", C.c_int32), ("nu_pre", C.c_int32 * 8),
                ("nu_post", C.c_int32 * 8), ("mixed_switch", C.c_double), ("seed", C.c_uint64),
                ("coarse_smoother", C.c_int32), ("relax_sweeps", C.c_int32), ("cfl_implicit", C.c_double),
                ("cycle_gamma", C.c_int32), ("cell_order", C.c_int32), ("mixed_stall", C.c_int32),
                ("adjoint_tape", C.c_int32)]


class CgksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cgks error {code}: {msg}")
        self.code = code


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_2402_02075_amd.build (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "cgks_default_params": [P], "cgks_create": [P, P], "cgks_set_params": [P, P], "cgks_set_stream": [P, P],
            "cgks_set_mesh": [P, I64, P, I64, P, P, P, I64, P, P, P, P], "cgks_set_bc": [P, I32, I32, P],
            "cgks_mesh_info": [P, P], "cgks_geometry": [P, P, P, P], "cgks_local_dt": [P, P, P],
            "cgks_reconstruct": [P, P, P, P, P], "cgks_residual": [P, P, P, P, P, P, P],
            "cgks_step": [P, P, P, P, D, P], "cgks_check": [P], "cgks_residual_norm": [P, P, P],
            "cgks_agglomerate_graph": [P, I64, P, P, I64, P, P, P, P, P, I32, P, P, P, P, P, P],
            "cgks_agglomerate": [P], "cgks_level_map": [P, I32, P], "cgks_kfvs_residual": [P, I32, P, P],
            "cgks_restrict": [P, I32, P, P, P, P], "cgks_prolong": [P, I32, P, P],
            "cgks_vcycle": [P, P, P, P, I32, D, P, P], "cgks_timing": [P, I32, P, P],
            "cgks_wall_force": [P, P, P, P, I32, P], "cgks_linearize": [P, P, P, P],
            "cgks_vjp_residual": [P, P, P, P, P, P, P], "cgks_vjp_wall_force": [P, I32, P, P, P, P],
            "cgks_vjp_kfvs": [P, I32, P, P, P], "cgks_adjoint_solve": [P, I32, P, I32, D, P, P, P, P, P, P, P, P, P],
            "cgks_set_param_directions": [P, I32, P, P, D], "cgks_jvp_residual": [P, P, P, P, P, P, P, P, P, P],
            "cgks_residual_host": [P, P, P, P, P, P, P], "cgks_vcycle_host": [P, P, P, P, I32, D, P, P],
            "cgks_coarse_implicit": [P, I32, P, P, P], "cgks_cell_order": [P, P],
            "cgks_residual_noalloc": [P, P, P, P, P, P, P],
        }
        for name, args in sig.items():
            if not hasattr(L, name):
                continue
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.cgks_destroy.argtypes = [P]
        L.cgks_destroy.restype = None
        L.cgks_last_error.argtypes = [P]
        L.cgks_last_error.restype = C.c_char_p
        _LIB = L
    return _LIB


def default_params(**kw) -> Params:
    p = Params()
    lib().cgks_default_params(C.byref(p))
    for k, v in kw.items():
        if k in ("nu_pre", "nu_post"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = int(x)
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors crossing the C ABI must be contiguous")
    return C.c_void_p(t.data_ptr())


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Solver:
    """One libcgks context bound to the current device and torch stream."""

    def __init__(self, params: Params | None = None, **kw):
        import torch
        self.torch = torch
        self.params = params if params is not None else default_params(**kw)
        h = C.c_void_p()
        self._check(lib().cgks_create(C.byref(self.params), C.byref(h)), None)
        self.h = h
        self.sync_stream()

    def _check(self, code, h="self"):
        if code != OK:
            msg = lib().cgks_last_error(self.h if h == "self" else None)
            raise CgksError(code, msg.decode() if msg else "")

    def sync_stream(self):
        s = self.torch.cuda.current_stream().cuda_stream
        self._check(lib().cgks_set_stream(self.h, C.c_void_p(s)))

    def set_params(self, **kw):
        """Change parameters; on an error from the library the previous parameters stay in force."""
        p = Params.from_buffer_copy(self.params)
        for k, v in kw.items():
            if k in ("nu_pre", "nu_post"):
                arr = getattr(p, k)
                for i, x in enumerate(v):
                    arr[i] = int(x)
            else:
                setattr(p, k, v)
        self._check(lib().cgks_set_params(self.h, C.byref(p)))
        self.params = p

    def close(self):
        if getattr(self, "h", None):
            lib().cgks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- mesh
    def set_mesh(self, m):
        self._n_params = 0
        keep = [_np(m.xyz, np.float64), _np(m.ctype, np.uint8), _np(m.cnode_ptr, np.int64), _np(m.cnode, np.int64),
                _np(m.bnode_ptr, np.int64), _np(m.bnode, np.int64), _np(m.btag, np.int32),
                None if m.node_canon is None else _np(m.node_canon, np.int64)]
        p = [None if a is None else a.ctypes.data_as(C.c_void_p) for a in keep]
        self._check(lib().cgks_set_mesh(self.h, m.n_nodes, p[0], m.n_cells, p[1], p[2], p[3], m.n_bfaces, p[4], p[5],
                                        p[6], p[7]))
        self.info()

    def cell_order(self):
        """perm[i] = caller id of the i-th cell in the library's internal (locality) order."""
        perm = np.zeros(self.n_cells, np.int32)
        self._check(lib().cgks_cell_order(self.h, perm.ctypes.data_as(C.c_void_p)))
        return perm

    def set_bc(self, tag, kind, prim=None):
        pr = None if prim is None else _np(prim, np.float64)
        self._check(lib().cgks_set_bc(self.h, int(tag), int(kind),
                                      None if pr is None else pr.ctypes.data_as(C.c_void_p)))

    def info(self):
        out = np.zeros(16, np.int64)
        self._check(lib().cgks_mesh_info(self.h, out.ctypes.data_as(C.c_void_p)))
        self.n_cells, self.n_faces, self.n_int, self.n_bfaces, self.n_gp = (int(x) for x in out[:5])
        self.level_sizes = [int(x) for x in out[6:6 + int(out[5])]]
        return out

    # ---------------------------------------------------------------- tensors
    def empty(self, *shape, dtype=None):
        t = self.torch
        return t.empty(*shape, dtype=dtype or t.float64, device="cuda")

    def geometry(self):
        N = self.n_cells
        vol, cen, m2 = self.empty(N), self.empty(3, N), self.empty(6, N)
        self._check(lib().cgks_geometry(self.h, _ptr(vol), _ptr(cen), _ptr(m2)))
        return vol, cen, m2

    def local_dt(self, W):
        dt = self.empty(self.n_cells)
        self._check(lib().cgks_local_dt(self.h, _ptr(W), _ptr(dt)))
        return dt

    def reconstruct(self, W, G, alpha=None):
        coef = self.empty(50, self.n_cells)
        self._check(lib().cgks_reconstruct(self.h, _ptr(W), _ptr(G), _ptr(alpha), _ptr(coef)))
        return coef

    def residual(self, W, G, alpha=None, grad=True):
        N = self.n_cells
        R = self.empty(5, N)
        Gn = self.empty(15, N) if grad else None
        an = self.empty(N) if grad else None
        self._check(lib().cgks_residual(self.h, _ptr(W), _ptr(G), _ptr(alpha), _ptr(R), _ptr(Gn), _ptr(an)))
        return R, Gn, an

    def residual_noalloc(self, W, G, alpha=None, R=None, Gn=None, an=None):
        """cgks_residual with the library's fixed work array (no device allocation in the library);
        the outputs are the caller's tensors when given."""
        N = self.n_cells
        R = self.empty(5, N) if R is None else R
        self._check(lib().cgks_residual_noalloc(self.h, _ptr(W), _ptr(G), _ptr(alpha), _ptr(R), _ptr(Gn), _ptr(an)))
        return R, Gn, an

    def residual_host(self, W, G, alpha=None):
        """cgks_residual on host (numpy) arrays in the caller's order -> numpy (R, G_new, alpha_new)."""
        N = self.n_cells
        W, G = _np(W, np.float64), _np(G, np.float64)
        al = None if alpha is None else _np(alpha, np.float64)
        R, Gn, an = np.zeros((5, N)), np.zeros((15, N)), np.zeros(N)
        p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        self._check(lib().cgks_residual_host(self.h, p(W), p(G), p(al), p(R), p(Gn), p(an)))
        return R, Gn, an

    def vcycle_host(self, W, G, alpha, max_cycles, tol_drop=1e-10):
        """cgks_vcycle on host (numpy, contiguous float64, updated in place) arrays."""
        for a in (W, G, alpha):
            if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
                raise ValueError("vcycle_host needs contiguous float64 numpy arrays (updated in place)")
        hist = np.zeros(max(max_cycles, 1))
        done = C.c_int32(0)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        code = lib().cgks_vcycle_host(self.h, p(W), p(G), p(alpha), int(max_cycles), float(tol_drop), p(hist),
                                      C.byref(done))
        if code not in (OK, E_NOCONV):
            self._check(code)
        return hist[:done.value], code == OK

    def step(self, W, G, alpha, dt_global=-1.0, resnorm=None):
        self._check(lib().cgks_step(self.h, _ptr(W), _ptr(G), _ptr(alpha), float(dt_global), _ptr(resnorm)))

    def check(self):
        self._check(lib().cgks_check(self.h))

    def residual_norm(self, R):
        out = self.empty(1)
        self._check(lib().cgks_residual_norm(self.h, _ptr(R), _ptr(out)))
        return out

    def wall_force(self, W, G, alpha, tag):
        """Force of the gas on the boundary faces with `tag`: device tensor of 3 doubles."""
        out = self.empty(3)
        self._check(lib().cgks_wall_force(self.h, _ptr(W), _ptr(G), _ptr(alpha), C.c_int32(int(tag)), _ptr(out)))
        return out

    # ---------------------------------------------------------------- discrete adjoint
    def linearize(self, W, G, alpha=None):
        """Record the exact local Jacobians of the fine operator at (W, G, alpha)."""
        self._check(lib().cgks_linearize(self.h, _ptr(W), _ptr(G), _ptr(alpha)))

    def vjp_residual(self, barR, barGnew=None, barAnew=None):
        """(dE/dU)^T (barR, barGnew, barAnew) at the linearised state -> (barW, barG, barAlpha)."""
        N = self.n_cells
        bW, bG, bA = self.empty(5, N), self.empty(15, N), self.empty(N)
        self._check(lib().cgks_vjp_residual(self.h, _ptr(barR), _ptr(barGnew), _ptr(barAnew), _ptr(bW), _ptr(bG),
                                            _ptr(bA)))
        return bW, bG, bA

    def jvp_residual(self, W, G, alpha, vW, vG, vA=None):
        """dE/dU . (vW, vG, vA) at (W, G, alpha) by forward-mode dual numbers -> (dR, dG, dA)."""
        N = self.n_cells
        dR, dG, dA = self.empty(5, N), self.empty(15, N), self.empty(N)
        self._check(lib().cgks_jvp_residual(self.h, _ptr(W), _ptr(G), _ptr(alpha), _ptr(vW), _ptr(vG), _ptr(vA),
                                            _ptr(dR), _ptr(dG), _ptr(dA)))
        return dR, dG, dA

    def vjp_wall_force(self, tag, e=(1.0, 0.0, 0.0)):
        """Gradient of e . F_wall(tag) with respect to (W, G, alpha) at the linearised state."""
        N = self.n_cells
        bW, bG, bA = self.empty(5, N), self.empty(15, N), self.empty(N)
        ev = (C.c_double * 3)(*[float(x) for x in e])
        self._check(lib().cgks_vjp_wall_force(self.h, C.c_int32(int(tag)), ev, _ptr(bW), _ptr(bG), _ptr(bA)))
        return bW, bG, bA

    def vjp_kfvs(self, level, Wc, barRc):
        out = self.empty(*tuple(Wc.shape))
        self._check(lib().cgks_vjp_kfvs(self.h, C.c_int32(int(level)), _ptr(Wc), _ptr(barRc), _ptr(out)))
        return out

    def set_param_directions(self, dprim=None, dxyz=None, step=1e-6):
        """Parameter directions of the adjoint gradients: dprim (n, 64, 5) far-field primitive
        derivatives per tag, dxyz (n, n_nodes, 3) node displacements per unit parameter."""
        n = None
        for a in (dprim, dxyz):
            if a is not None:
                n = a.shape[0] if n is None else n
                if a.shape[0] != n:
                    raise ValueError("dprim and dxyz must describe the same number of parameters")
        n = n or 0
        dp = None if dprim is None else _np(dprim, np.float64).reshape(n, 64, 5)
        dx = None if dxyz is None else _np(dxyz, np.float64).reshape(n, -1, 3)
        self._n_params = n
        self._check(lib().cgks_set_param_directions(self.h, C.c_int32(n),
                                                    None if dp is None else dp.ctypes.data_as(C.c_void_p),
                                                    None if dx is None else dx.ctypes.data_as(C.c_void_p),
                                                    float(step)))

    def adjoint_solve(self, tag, e=(1.0, 0.0, 0.0), max_iter=20000, tol=1e-10):
        """Adjoint fixed point through the transposed V-cycle at the linearised (converged) state.

        Returns dict with lamW, lamG, lamA, cR, cG, cA (device tensors), hist (numpy), iterations
        and dJ_dparams (numpy, one per direction of set_param_directions)."""
        N = self.n_cells
        out = {k: self.empty(*s) for k, s in (("lamW", (5, N)), ("lamG", (15, N)), ("lamA", (N,)), ("cR", (5, N)),
                                                ("cG", (15, N)), ("cA", (N,)))}
        hist = np.zeros(int(max_iter))
        nd = C.c_int32(0)
        ev = (C.c_double * 3)(*[float(x) for x in e])
        dj = np.zeros(max(getattr(self, "_n_params", 0), 1))
        self._check(lib().cgks_adjoint_solve(self.h, C.c_int32(int(tag)), ev, C.c_int32(int(max_iter)), float(tol),
                                             _ptr(out["lamW"]), _ptr(out["lamG"]), _ptr(out["lamA"]), _ptr(out["cR"]),
                                             _ptr(out["cG"]), _ptr(out["cA"]), hist.ctypes.data_as(C.c_void_p),
                                             C.byref(nd), dj.ctypes.data_as(C.c_void_p)))
        out["hist"] = hist[:nd.value]
        out["iterations"] = nd.value
        out["dJ_dparams"] = dj[:getattr(self, "_n_params", 0)]
        return out

    # ---------------------------------------------------------------- multigrid
    def agglomerate_graph(self, V, P, a, b, S, M, A, passes):
        """Raw-graph agglomeration; device tensors; returns (f2c, Vc, Pc, n_coarse, m_coarse, stats)."""
        n, m = int(V.shape[0]), int(a.shape[0])
        f2c = self.empty(n, dtype=self.torch.int32)
        Vc, Pc = self.empty(n), self.empty(n, 3)
        nc, mc = C.c_int64(0), C.c_int64(0)
        stats = np.zeros((max(passes, 1), 4), np.int64)
        self._check(lib().cgks_agglomerate_graph(self.h, n, _ptr(V), _ptr(P), m, _ptr(a), _ptr(b), _ptr(S), _ptr(M),
                                                 _ptr(A), int(passes), _ptr(f2c), _ptr(Vc), _ptr(Pc), C.byref(nc),
                                                 C.byref(mc), stats.ctypes.data_as(C.c_void_p)))
        return f2c, Vc[:nc.value], Pc[:nc.value], nc.value, mc.value, stats

    def agglomerate(self):
        self._check(lib().cgks_agglomerate(self.h))
        self.info()
        return self.level_sizes

    def level_map(self, level):
        f2c = self.empty(self.level_sizes[level - 1], dtype=self.torch.int32)
        self._check(lib().cgks_level_map(self.h, int(level), _ptr(f2c)))
        return f2c

    def kfvs_residual(self, level, W):
        R = self.empty(5, self.level_sizes[level])
        self._check(lib().cgks_kfvs_residual(self.h, int(level), _ptr(W), _ptr(R)))
        return R

    def coarse_implicit(self, level, W, rhs):
        """Increment of the implicit coarse smoother (Sec. 4.3) on `level` at state W for rhs."""
        n = self.level_sizes[level] if 0 <= level < len(self.level_sizes) else 1  # the library rejects bad levels
        dU = self.empty(5, n)
        self._check(lib().cgks_coarse_implicit(self.h, int(level), _ptr(W), _ptr(rhs), _ptr(dU)))
        return dU

    def restrict(self, level, Wf, Rf):
        n = self.level_sizes[level]
        Wc, Rc = self.empty(5, n), self.empty(5, n)
        self._check(lib().cgks_restrict(self.h, int(level), _ptr(Wf), _ptr(Rf), _ptr(Wc), _ptr(Rc)))
        return Wc, Rc

    def prolong(self, level, dWc, Wf):
        self._check(lib().cgks_prolong(self.h, int(level), _ptr(dWc), _ptr(Wf)))

    def timing_start(self):
        self._check(lib().cgks_timing(self.h, 1, None, None))

    def timing_stop(self):
        """Accumulated face-kernel milliseconds and launch count since timing_start()."""
        ms, n = C.c_double(0), C.c_int64(0)
        self._check(lib().cgks_timing(self.h, 0, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def vcycle(self, W, G, alpha, max_cycles, tol_drop=1e-10):
        hist = np.zeros(max(max_cycles, 1))
        done = C.c_int32(0)
        code = lib().cgks_vcycle(self.h, _ptr(W), _ptr(G), _ptr(alpha), int(max_cycles), float(tol_drop),
                                 hist.ctypes.data_as(C.c_void_p), C.byref(done))
        if code not in (OK, E_NOCONV):
            self._check(code)
        return hist[:done.value], code == OK
