/*
 * cgks.h -- C ABI of the MI355X multigrid compact gas-kinetic scheme library.
 *
 * Method: multigrid compact gas-kinetic scheme (CGKS) for steady flow on 3-D
 * hybrid tet/pyramid/prism/hex meshes, arXiv 2402.02075 (Liu, Ji, Mao, Ding,
 * Xu).  Fine level: third-order CGKS (HWENO reconstruction, BGK interface
 * solution at face Gauss points, Gauss-Green update of cell-averaged
 * gradients); coarse levels: first-order KFVS with forward Euler (or the
 * implicit smoother of Sec. 4.3), on meshes built by two-step random-hash
 * agglomeration; three-level V-cycle (levels, sweeps and W-cycles configurable).
 *
 * Conventions for every call:
 *  - Return value: CGKS_OK (0) or a negative cgks_status; cgks_last_error()
 *    gives a message.  No C++ exception crosses this boundary.
 *  - "device" pointers are HIP device allocations (e.g. torch CUDA tensors on
 *    ROCm), used stream-ordered on the stream given to cgks_set_stream (the
 *    null stream by default).  The library never frees caller memory.
 *    "host" pointers are read or written before the call returns.
 *  - Cell fields are FP64, component-major, in the caller's cell order (or in the library's
 *    internal order with params.cell_order = 2, see cgks_cell_order):
 *      W[c*N + i]        c = rho, rho u, rho v, rho w, rho E      (5 x N)
 *      G[(3c+d)*N + i]   cell average of dW_c/dx_d, d = x, y, z    (15 x N)
 *      alpha[i]          gradient compression factor               (N)
 *  - No call synchronises the device except where stated (mesh set-up,
 *    agglomeration, and the once-per-cycle residual read of cgks_vcycle).
 *  - One context per host thread; contexts are independent.
 *  - Calls that evaluate boundary faces (reconstruction, residual, step, wall force, the
 *    adjoint calls, coarse KFVS and implicit smoother, V-cycle) return CGKS_E_STATE while a
 *    boundary tag used by the mesh has no condition from cgks_set_bc.
 */
#ifndef CGKS_H
#define CGKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgks_ctx cgks_ctx;

typedef enum {
    CGKS_OK = 0,
    CGKS_E_ARG = -1,       /* invalid argument; nothing written */
    CGKS_E_MESH = -2,      /* invalid or non-conforming mesh; nothing written */
    CGKS_E_DEVICE = -3,    /* HIP runtime error */
    CGKS_E_NONFINITE = -4, /* NaN or Inf in a state */
    CGKS_E_PHYS = -5,      /* non-positive density or pressure; message names the first cell */
    CGKS_E_NOCONV = -6,    /* cgks_vcycle: max_cycles reached before the requested drop */
    CGKS_E_STATE = -7      /* call out of order (e.g. no mesh, no hierarchy) */
} cgks_status;

/* element types: the node count, VTK node order */
enum { CGKS_TET = 4, CGKS_PYR = 5, CGKS_PRISM = 6, CGKS_HEX = 8 };
/* boundary kinds */
enum { CGKS_BC_SLIP = 1, CGKS_BC_NOSLIP_ADIABATIC = 2, CGKS_BC_FARFIELD = 3 };

typedef struct {
    double gamma;        /* ratio of specific heats (1.4) */
    double mu;           /* dynamic viscosity, constant (0 for inviscid) */
    double prandtl;      /* Prandtl number (1 = BGK value, no correction) */
    double cfl;          /* CFL number of the local time step (fine and coarse) */
    double eps_tau;      /* inviscid collision time tau_n = eps dt + ...  (0.01) */
    double c_tau;        /* pressure-jump coefficient C of tau_n (1) */
    double weno_eps;     /* epsilon of the nonlinear weights (1e-5) */
    double gamma_lin;    /* linear weight gamma_2 of the large stencil (0.5) */
    double skew_delta;   /* agglomeration: accept if the virtual centre is within delta V^(1/3) (0.25) */
    double skew_sin;     /* agglomeration: or if the angle to the face plane has sine >= this (sin 10 deg) */
    int32_t viscous;     /* 0 inviscid, 1 Navier-Stokes */
    int32_t levels;      /* multigrid levels including the fine one (3) */
    int32_t passes;      /* agglomeration passes per coarse level (3) */
    int32_t precision;   /* 0 FP64 everywhere, 1 mixed (FP32 coarse levels, transfers and flux evaluation;
                            the first selection with a mesh set allocates FP32 copies of the
                            reconstruction operator and the lane geometry, about 0.9 KB per cell) */
    int32_t nu_pre[8];   /* pre-smoothing sweeps per level (1) */
    int32_t nu_post[8];  /* post-smoothing sweeps per level (0) */
    double mixed_switch; /* mixed precision: FP64 flux once the residual drop is below this (1e-6) */
    uint64_t seed;       /* hash seed multiplier s (1 reproduces the paper's hash) */
    int32_t coarse_smoother; /* coarse levels: 0 forward Euler (default), 1 implicit backward Euler
                                with point relaxation (paper Sec. 4.3) */
    int32_t relax_sweeps;    /* relaxation sweeps of the implicit coarse smoother (2) */
    double cfl_implicit;     /* CFL number of the implicit coarse smoother's local step (0.25) */
    int32_t cycle_gamma;     /* visits of each coarser level per visit of its parent, each continuing
                                with the same forcing: 1 V-cycle (default), 2 W-cycle (1..3) */
    int32_t cell_order;      /* internal order of the cells, fixed by cgks_set_mesh:
                                0  the caller's order;
                                1  (default) a locality order (by element type, then along the
                                   Hilbert curve through the cell centroids; faces sorted by their
                                   cells in that order); every cell array at
                                   this ABI stays in the caller's order and is gathered / scattered
                                   at the call (one extra pass over the array);
                                2  the same locality order, and cell arrays at this ABI are exchanged
                                   in it (no gather or scatter; cgks_cell_order gives the order).
                                Switching between 0 and 1/2 needs a new cgks_set_mesh. */
    int32_t mixed_stall;     /* mixed precision: FP64 flux also once the residual norm has not
                                reached a new minimum for this many cycles (300; >= 1) */
    int32_t adjoint_tape;    /* storage of the Jacobians cgks_linearize records: 0 FP64 (default),
                                1 FP32 (half the memory; every product still accumulates in FP64,
                                so only the stored entries are rounded, to 2^-24 relative) */
} cgks_params;

/* Fill *p with the defaults above. */
cgks_status cgks_default_params(cgks_params *p);

/* Create a context on the current HIP device. */
cgks_status cgks_create(const cgks_params *p, cgks_ctx **out);
void cgks_destroy(cgks_ctx *ctx);
const char *cgks_last_error(const cgks_ctx *ctx);

/* Replace the parameters (mesh and hierarchy are kept; levels/passes/seed take effect at the next agglomerate). */
cgks_status cgks_set_params(cgks_ctx *ctx, const cgks_params *p);

/* Stream for all later work (a hipStream_t; NULL = null stream). */
cgks_status cgks_set_stream(cgks_ctx *ctx, void *hip_stream);

/*
 * Mesh (paper Sec. 2.2: hybrid cells, linear iso-parametric faces; 3 Gauss
 * points on a triangle, 4 on a quadrilateral).  All host arrays, copied:
 *   xyz[3*n_nodes] interleaved coordinates;
 *   ctype[n_cells] node count of each cell, cnode_ptr[n_cells+1] / cnode[] its nodes;
 *   bnode_ptr[n_bfaces+1] / bnode[] / btag[n_bfaces] boundary faces (3 or 4 nodes, tag 1..63);
 *   node_canon[n_nodes] or NULL: nodes with equal canonical id are periodic images
 *   (faces whose canonical node sets match are joined across the period).
 * Every cell face must be shared by two cells or listed once as a boundary face
 * (else CGKS_E_MESH).  Computes geometry and reconstruction operators on the device.
 * Synchronises.
 */
cgks_status cgks_set_mesh(cgks_ctx *ctx, int64_t n_nodes, const double *xyz, int64_t n_cells, const uint8_t *ctype,
                          const int64_t *cnode_ptr, const int64_t *cnode, int64_t n_bfaces, const int64_t *bnode_ptr,
                          const int64_t *bnode, const int32_t *btag, const int64_t *node_canon);

/*
 * Internal cell order (the data layout in HBM): perm[i] (host out, int32[N]) is the caller's id of
 * the i-th cell as the library stores it.  The identity with params.cell_order = 0.  With
 * cell_order = 2 every cell array at this ABI is indexed in this order.  The agglomeration
 * (cgks_agglomerate) always hashes and orders by the caller's ids (paper Sec. 4.1), so the
 * hierarchy does not depend on the internal order.  CGKS_E_STATE without a mesh.
 */
cgks_status cgks_cell_order(const cgks_ctx *ctx, int32_t *perm);

/* Boundary condition of a tag (1..63).  prim = far-field rho, u, v, w, p (host, used by CGKS_BC_FARFIELD). */
cgks_status cgks_set_bc(cgks_ctx *ctx, int32_t tag, int32_t kind, const double *prim);

/*
 * Sizes (host out[16]): [0] cells, [1] faces, [2] interior faces, [3] boundary faces,
 * [4] Gauss points, [5] hierarchy levels built, [6..13] cells per level.
 */
cgks_status cgks_mesh_info(const cgks_ctx *ctx, int64_t *out);

/* Geometry (device out, caller order, each nullable): vol[N], cen[3N] (component-major), mom2[6N]
 * second moments about the centroid, order xx yy zz xy yz xz, component-major. */
cgks_status cgks_geometry(cgks_ctx *ctx, double *vol, double *cen, double *mom2);

/*
 * Local time step (paper Secs. 1, 4.3: local time stepping on every level):
 * dt[i] = CFL |Omega_i| / sum_p lambda_p S_p, lambda_p = |U.n_p| + c + 2 mu S_p/(rho |Omega_i|).
 * W: device 5N in, dt: device N out.
 */
cgks_status cgks_local_dt(cgks_ctx *ctx, const double *W, double *dt);

/*
 * HWENO reconstruction (paper Sec. 3): per cell and component the 10 monomial
 * coefficients of R(x) about the cell centroid, order 1, dx, dy, dz, dx^2, dy^2,
 * dz^2, dxdy, dydz, dxdz.  coef: device [50 N], coef[(10 c + k) N + i].
 */
cgks_status cgks_reconstruct(cgks_ctx *ctx, const double *W, const double *G, const double *alpha, double *coef);

/*
 * Fine CGKS residual (paper Eqs. semidiscrete, 2nd-flux, gauss-formula; Sec. 3.3):
 *   R[5N]         = - sum_p S_p sum_k w_k F(x_pk).n_p, F time-averaged over the face step
 *                   dt_f = min(dt_L, dt_R) of the local steps;
 *   G_new[15N]    = alpha_new / |Omega| * sum_p sum_k w_k W_pk(dt_f) n_pk S_p;
 *   alpha_new[N]  = product over interior-face Gauss points of 1/(1 + A^2).
 * Inputs W, G, alpha (alpha of the previous update, scales the Green-Gauss p^1).
 * G_new and alpha_new may be NULL (residual only).  All device.  With precision 1 the
 * flux is evaluated in FP32: FP32 reconstruction coefficients (FP64 arithmetic), FP32 polynomial
 * evaluation, frame rotations, BGK solution and compression factor; face sums, gathers and
 * outputs stay FP64.
 */
cgks_status cgks_residual(cgks_ctx *ctx, const double *W, const double *G, const double *alpha, double *R,
                          double *G_new, double *alpha_new);

/*
 * One explicit step in place on device W, G, alpha.
 *   dt_global <= 0: fine smoother W += dt_i/|Omega_i| R with local steps (paper Eq. smo);
 *   dt_global  > 0: two-stage fourth-order step with this global step.
 * resnorm (device, nullable) receives sqrt(mean_i (R_rho,i/|Omega_i|)^2) of the step (smoother only).
 */
cgks_status cgks_step(cgks_ctx *ctx, double *W, double *G, double *alpha, double dt_global, double *resnorm);

/*
 * Synchronise and report kernel-detected state errors: CGKS_E_PHYS (with the
 * first offending cell in the message) if any Gauss-point state had
 * non-positive density or pressure since the previous check, else CGKS_OK.
 */
cgks_status cgks_check(cgks_ctx *ctx);

/*
 * cgks_residual without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc).  Same arguments, outputs and
 * kernels as cgks_residual; its work memory (local steps, polynomial coefficients, boundary ghost
 * states, face records, and with params.cell_order = 1 the reordered inputs and outputs) comes from
 * one fixed device array of 32 Mi doubles (256 MiB) per GPU, kept until the process ends, instead
 * of the context's buffers.  It needs N + 50 N + 5 Fb + 21 F doubles (5 F without G_new), plus
 * 42 N with cell_order 1, each rounded up to 32; a mesh that needs more returns CGKS_E_ARG before
 * any work (about 230k mixed cells with cell_order 1, 330k with 0 or 2).  With precision 1 the
 * FP32 coefficients take the coefficient piece (the FP32 operator and lane-geometry copies are
 * the context's, made when precision 1 was selected).  Nothing in the array
 * needs clearing: every call writes all it reads.  All calls on one GPU share the array, from every
 * context: calls that overlap on one GPU (other streams, other host threads) race and must be
 * ordered by the caller.  The context's device must be the current device (CGKS_E_DEVICE).
 */
cgks_status cgks_residual_noalloc(cgks_ctx *ctx, const double *W, const double *G, const double *alpha, double *R,
                                  double *G_new, double *alpha_new);

/*
 * Force of the gas on the boundary faces carrying `tag` (the integrated surface force behind the
 * drag coefficients of paper Sec. 5): F[d] = sum over those faces of S_p sum_k w_k F_mom,d(x_pk),
 * the momentum part of the same time-averaged face flux as cgks_residual, normal pointing out of
 * the gas.  W, G, alpha (nullable) device in; F: device double[3] out.  Faces are summed in a fixed
 * order by one work-group: deterministic.  CGKS_E_ARG for a tag outside 1..63.
 */
cgks_status cgks_wall_force(cgks_ctx *ctx, const double *W, const double *G, const double *alpha, int32_t tag,
                            double *F);

/*
 * Discrete adjoint (vector-Jacobian products of the operators above).
 *
 * The fine operator is E(W, G, alpha) = (R, G_new, alpha_new) of cgks_residual.
 * cgks_linearize records its exact local Jacobians at one state (device W, G,
 * alpha nullable = ones): per Gauss point the derivatives of the time-averaged
 * flux, interface value and compression factor (paper Eq. 2nd-flux, Sec. 2.4,
 * Sec. 3.3) with respect to the two reconstructed states, their gradients and
 * the face step; per cell and component those of the HWENO coefficients (Sec. 3)
 * with respect to the stencil data; per cell that of the local time step.
 * Device memory kept: the Jacobians, 452 NGP + 1500 N values (NGP = Gauss points of all
 * faces, cgks_mesh_info[4], rounded up to a multiple of 64; 451 values per Gauss point padded to
 * 452; FP64, or FP32 with params.adjoint_tape = 1), and about
 * 300 N + 150 F doubles of state and work buffers (some 100 N more once cgks_adjoint_solve
 * has run), released with the context.  Its dual-number kernels also need about 2.3 KB of
 * scratch memory per GPU lane in flight (up to a few GB), which the HIP runtime allocates at launch:
 * leave that much device memory free beyond the tape (the runtime aborts the queue, rather
 * than return an error, when it cannot get it).  If the tape itself does not fit, CGKS_E_DEVICE
 * says how much it needs.  CGKS_E_PHYS if a Gauss-point state is non-physical.  Any later
 * cgks_set_mesh, cgks_set_bc, cgks_set_params or cgks_agglomerate invalidates it.
 */
cgks_status cgks_linearize(cgks_ctx *ctx, const double *W, const double *G, const double *alpha);

/*
 * barW[5N], barG[15N], barAlpha[N] (device out, barAlpha nullable) =
 *   (dE/d(W, G, alpha))^T (barR[5N], barGnew[15N], barAnew[N]) at the linearised state.
 * barGnew and barAnew may be NULL (zero cotangents).  CGKS_E_STATE without cgks_linearize.
 */
cgks_status cgks_vjp_residual(cgks_ctx *ctx, const double *barR, const double *barGnew, const double *barAnew,
                              double *barW, double *barG, double *barAlpha);

/*
 * Directional derivative of the fine operator: (dR, dG, dA) = dE/d(W, G, alpha) . (vW, vG, vA) at
 * (W, G, alpha) (device; alpha and vA nullable = ones / zero; dG, dA nullable), by one pass of
 * forward-mode dual numbers through the reconstruction (Sec. 3), the local steps, the Gauss-point
 * BGK solution in its moment-matrix form (Eq. 2nd-flux, Sec. 2.4, Sec. 3.3) and the cell sums.
 * It needs no cgks_linearize and shares no recorded Jacobian with the vector-Jacobian products,
 * so <u, J v> against <J^T u, v> checks them.  Same one-sided conventions at kinks as the
 * linearisation.  Allocates its work memory per call; synchronises.
 */
cgks_status cgks_jvp_residual(cgks_ctx *ctx, const double *W, const double *G, const double *alpha, const double *vW,
                              const double *vG, const double *vA, double *dR, double *dG, double *dA);

/*
 * Gradient of J = e . F_wall(tag) (cgks_wall_force) at the linearised state with
 * respect to (W, G, alpha): device barW[5N], barG[15N], barAlpha[N] (nullable); e host double[3].
 */
cgks_status cgks_vjp_wall_force(cgks_ctx *ctx, int32_t tag, const double *e, double *barW, double *barG,
                                double *barAlpha);

/*
 * Coarse KFVS operator of cgks_kfvs_residual on `level` (>= 1, paper Sec. 4.2):
 * barWc[5n] = (dR_c/dW_c)^T barRc[5n] at the coarse state Wc (all device, FP64).
 * Exact face Jacobians, recomputed per call; deterministic gathers.
 */
cgks_status cgks_vjp_kfvs(cgks_ctx *ctx, int32_t level, const double *Wc, const double *barRc, double *barWc);

/*
 * Parameter directions for the gradients of cgks_adjoint_solve (for instance the inflow Mach number
 * and the bump amplitude of the bump channel's drag sensitivities, or any other scalar parameters).  Parameter k
 * moves, per unit, the far-field primitives (rho, u, v, w, p) of boundary tag t by
 * dprim[(k * 64 + t) * 5 + q] (host, nullable = no change) and node j of the mesh (caller's node
 * numbering) by dxyz[k * 3 n_nodes + 3 j + d] (host, nullable = no node moves); n_params <= 8.
 * step: the parameter step h of the differences of the explicit dependence (see
 * cgks_adjoint_solve; 1e-6 suits parameters of order one: the operator has kinks (|p_l - p_r| of
 * the collision time, min of the smoothness indicators) that a larger step may straddle).  Copied; cleared by cgks_set_mesh.  CGKS_E_STATE without a mesh.
 */
cgks_status cgks_set_param_directions(cgks_ctx *ctx, int32_t n_params, const double *dprim, const double *dxyz,
                                      double step);

/*
 * Adjoint fixed point of the V-cycle (cgks_vcycle, FP64, one pre-sweep per level,
 * no post-sweeps) at the linearised state, which must be converged:
 *   lam = (dPhi/dU)^T lam + dJ/dU,  J = e . F_wall(tag),  U = (W, G, alpha),
 * iterated until |lam_k+1 - lam_k| <= tol |lam_k+1| or max_iter.  Device outputs
 * (each nullable): lamW[5N], lamG[15N], lamA[N]; and the cotangents cR[5N], cG[15N],
 * cA[N] on the fine operator's outputs (R, G_new, alpha_new) with which a parameter
 * p enters: dJ/dp = dJ/dp|_U + cR . dR/dp + cG . dG_new/dp + cA . dalpha_new/dp.
 * dJ_dparams (host, nullable, one per direction of cgks_set_param_directions) receives that
 * gradient for every parameter: the library rebuilds the geometry, reconstruction operators and
 * boundary states at p = +-h, +-2h (same cells and faces), evaluates J and E at the fixed state,
 * and forms dJ/dp|_U and c . dE/dp|_U by the fourth-order central difference
 * (8 (f(h) - f(-h)) - (f(2h) - f(-2h))) / 12h (truncation O(h^4), rounding O(eps/h)).
 * hist (host, nullable, max_iter doubles) receives the relative change per iteration;
 * n_done (host) the iterations run.  Synchronises once per iteration.
 */
cgks_status cgks_adjoint_solve(cgks_ctx *ctx, int32_t tag, const double *e, int32_t max_iter, double tol,
                               double *lamW, double *lamG, double *lamA, double *cR, double *cG, double *cA,
                               double *hist, int32_t *n_done, double *dJ_dparams);

/* RMS of R_rho/|Omega| (device R in, device scalar out). */
cgks_status cgks_residual_norm(cgks_ctx *ctx, const double *R, double *out);

/*
 * Agglomeration on a raw graph (paper Sec. 4.1, Algorithm 1), P passes.
 * Device inputs: V[n], P[3n] first moments (V*centroid, interleaved xyz),
 * pair_a[m] < pair_b[m] (int32, lexicographically sorted, no duplicates),
 * S[m] face areas, M[3m] first area moments (interleaved), A[3m] area vectors a->b.
 * Device outputs: f2c[n] (int32, coarse ids numbered by smallest member),
 * Vc[n], Pc[3n] (first *n_coarse valid).  Host out: n_coarse, m_coarse, stats[4*passes]
 * (selected, skew-accepted, merged, new pair count per pass; nullable).
 * Deterministic: identical inputs give identical outputs; synchronises.
 */
cgks_status cgks_agglomerate_graph(cgks_ctx *ctx, int64_t n, const double *V, const double *P, int64_t m,
                                   const int32_t *pair_a, const int32_t *pair_b, const double *S, const double *M,
                                   const double *A, int32_t passes, int32_t *f2c, double *Vc, double *Pc,
                                   int64_t *n_coarse, int64_t *m_coarse, int64_t *stats);

/* Build the multigrid hierarchy on the context's mesh (params.levels, .passes, .seed). Synchronises. */
cgks_status cgks_agglomerate(cgks_ctx *ctx);

/* Level map: f2c[n_{level-1}] (device int32) from level-1 cells to level cells; level >= 1. */
cgks_status cgks_level_map(cgks_ctx *ctx, int32_t level, int32_t *f2c);

/* Coarse KFVS residual on level >= 1 (paper Secs. 1, 4.2): R = - sum S n.F_kfvs. Device W, R (5 N_l),
 * FP64; with precision 1 the operator is evaluated in FP32 (as on the coarse levels of the mixed cycle). */
cgks_status cgks_kfvs_residual(cgks_ctx *ctx, int32_t level, const double *W, double *R);

/* Increment of the implicit coarse smoother on level >= 1 (paper Sec. 4.3): backward Euler
 * linearised with the Lax-Friedrichs flux Jacobian A+- = (A +- lambda I)/2, solved without a
 * matrix by params.relax_sweeps point-relaxation (Jacobi) sweeps after dU = rhs/D:
 *   (|Omega_i|/dt_i + 1/2 sum_p lambda_p S_p) dU_i + sum_p [F-(U_p + dU_p) - F-(U_p)] S_p = rhs_i,
 *   F- = (F_n - lambda U)/2, lambda = max of the two cells' |U.n| + c + 2 mu S/(rho |Omega|),
 * dt_i the coarse local step at params.cfl_implicit, S the coarse face's |A|; a boundary face adds
 * lambda S/2 (owner vs ghost state) to the diagonal and no neighbour term.
 * W, rhs, dU: device [5][N_l] FP64, dU overwritten; with precision 1 evaluated in FP32.
 * The V-cycle uses it on every coarse sweep when params.coarse_smoother = 1, with rhs =
 * Res_2h(W) + F (the FAS right-hand side) and W += dU. */
cgks_status cgks_coarse_implicit(cgks_ctx *ctx, int32_t level, const double *W, const double *rhs, double *dU);

/* Restriction to level >= 1 (paper Sec. 4.2): Wc = sum V W / Vc, Rc = sum R (either pair nullable). */
cgks_status cgks_restrict(cgks_ctx *ctx, int32_t level, const double *Wf, const double *Rf, double *Wc, double *Rc);

/* Prolongation (paper Sec. 4.2 correction): Wf[i] += dWc[f2c[i]] from level to level-1. */
cgks_status cgks_prolong(cgks_ctx *ctx, int32_t level, const double *dWc, double *Wf);

/*
 * V-cycles (paper Sec. 4.2, Fig. Procedure): fine smoothing (nu_pre[0]), fine residual at the
 * smoothed state restricted with the volume-weighted state, forcing term, coarse
 * KFVS sweeps (or the implicit smoother, params.coarse_smoother), recursion with
 * params.cycle_gamma visits per coarser level (2: W-cycle), correction; repeated until the residual drops by tol_drop
 * relative to the first cycle or max_cycles.  In place on device W, G, alpha.
 * hist (host, nullable, max_cycles) receives the residual norm of each cycle;
 * *n_done the cycles run.  Cycles are queued in batches (16; all cycles, up to 2^22, when
 * tol_drop <= 0 in FP64) with their norms kept on the device and read once per batch; the state at
 * a batch's start is kept (21 N doubles of device memory), so that a stop, a precision switch or a
 * non-physical state before the batch's end is reproduced by re-running from it: the results are
 * those of a loop that checks after every cycle (the kernels are deterministic).
 * With params.precision 1 every call starts with the FP32 flux and FP32 coarse levels and
 * switches to FP64 for the rest of the call once the drop reaches params.mixed_switch or the norm
 * has gone params.mixed_stall cycles without a new minimum.
 * Returns CGKS_E_NOCONV if the drop was not reached (state and history valid).
 */
cgks_status cgks_vcycle(cgks_ctx *ctx, double *W, double *G, double *alpha, int32_t max_cycles, double tol_drop,
                        double *hist, int32_t *n_done);

/*
 * Host-pointer twins of cgks_residual and cgks_vcycle: the same arguments and results with every
 * cell array in host memory (caller's cell order); the library copies them to and from device
 * memory it allocates for the call and synchronises before returning.  cgks_vcycle_host writes the
 * state back also when it returns CGKS_E_NOCONV, CGKS_E_PHYS or CGKS_E_NONFINITE (the state the
 * device call leaves).
 */
cgks_status cgks_residual_host(cgks_ctx *ctx, const double *W, const double *G, const double *alpha, double *R,
                               double *G_new, double *alpha_new);
cgks_status cgks_vcycle_host(cgks_ctx *ctx, double *W, double *G, double *alpha, int32_t max_cycles, double tol_drop,
                             double *hist, int32_t *n_done);

/*
 * Kernel timing for profiling: with enable = 1 the library brackets every
 * launch of the fine face-flux kernel in its steady mode with gradient update
 * (the BGK interface solution at the Gauss points, flux and interface values)
 * with HIP events on its stream.  A call with enable = 0 synchronises,
 * writes the accumulated kernel time (host *face_ms) and launch count (host
 * *face_launches, nullable), and stops timing.  Timing adds two event records
 * per launch and no synchronisation until it is read.
 */
cgks_status cgks_timing(cgks_ctx *ctx, int32_t enable, double *face_ms, int64_t *face_launches);

#ifdef __cplusplus
}
#endif
#endif
