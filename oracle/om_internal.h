/*
 * CGKS CPU oracle -- internal declarations.
 *
 * TEST INFRASTRUCTURE ONLY.  This tree is a plain, slow FP64 re-statement of
 * the multigrid compact gas-kinetic scheme (arXiv 2402.02075) used to check
 * the GPU library.  It shares no code, header or table with the library; only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  Nothing here is tuned for speed.
 */
#ifndef OM_INTERNAL_H
#define OM_INTERNAL_H

#include <stdint.h>
#include <stddef.h>

#define OM_MAXGP 4
#define OM_MAXNF 6

enum { OM_TET = 4, OM_PYR = 5, OM_PRISM = 6, OM_HEX = 8 };
enum { OM_BC_SLIP = 1, OM_BC_NOSLIP = 2, OM_BC_FARFIELD = 3 };

typedef struct {
    double gamma, mu, prandtl, cfl;
    double eps_tau, c_tau, weno_eps, gamma_lin;
    int viscous;
    /* coarse-level smoother: 0 forward Euler, 1 implicit backward Euler (Sec. 4.3) */
    int coarse_smoother;
    int relax_sweeps;    /* point-relaxation sweeps of the implicit smoother */
    double cfl_implicit; /* CFL number of the implicit smoother's local time step */
    int cycle_gamma;     /* visits of each coarser level per visit of its parent: 1 V-cycle, 2 W-cycle */
} om_params;

typedef struct {
    int kind;
    double prim[5]; /* rho, u, v, w, p of the far field */
} om_bc;

typedef struct om_mesh {
    int64_t n_nodes, n_cells;
    double *xyz;
    /* cells */
    double *vol;     /* |Omega| */
    double *cen;     /* 3 per cell, centroid */
    double *mom2;    /* 6 per cell: xx yy zz xy yz xz second moments about centroid */
    int *nface;      /* faces per cell */
    /* faces: interior first, then boundary */
    int64_t n_faces, n_int;
    int64_t *fl, *fr;        /* fr = -1 on boundary */
    int32_t *ftag;
    double *shift;           /* 3 per face: (face seen from L) - (face seen from R) */
    int *ngp;
    double *gpx, *gpw, *gpn; /* per face OM_MAXGP points: xyz, normalised weight, unit normal (L->R) */
    double *area;            /* S */
    double *avec;            /* integral of n dS (3) */
    double *fmom;            /* integral of x dS (3) */
    /* cell -> face */
    int64_t *cf_ptr, *cf_face;
    int *cf_sign;            /* +1 if the cell is L of that face */
    /* boundary conditions by tag */
    om_bc bc[64];
} om_mesh;

/* kinetic.c */
void om_moments_1d(double U, double lam, int half, int nmax, double *m);
double om_xi_moment(int l, double lam, double K);
void om_prim_from_cons(const double *W, double gamma, double *rho, double *U, double *lam);
int om_micro_slope(double rho, const double *U, double lam, double K, const double *dW, double *a);
int om_time_slope(const double *U, double lam, double K, const double a[3][5], double *A);
typedef struct {
    double F[5];      /* time-averaged flux over [0,dt] (local frame) */
    double Fint[5];   /* time-integrated flux over [0,dt] */
    double Fhalf[5];  /* time-integrated flux over [0,dt/2] */
    double Wdt[5];    /* interface value at t = dt */
    double Whalf[5];  /* interface value at t = dt/2 */
    double Wc[5];     /* interface equilibrium state */
} om_gks_out;
int om_gks_point(const double *Wl, const double *dWl /*[3][5] local-frame gradients*/,
                 const double *Wr, const double *dWr, double dt, const om_params *p, om_gks_out *out);
void om_kfvs_point(const double *Wl, const double *Wr, double gamma, double *F);

/* geometry helpers */
void om_frame(const double *n, double *t1, double *t2);
void om_rotate_state(const double *W, const double *n, const double *t1, const double *t2, double *Wl);
void om_rotate_back(const double *Wl, const double *n, const double *t1, const double *t2, double *W);
void om_rotate_grad(const double *G, const double *n, const double *t1, const double *t2, double *Gl);

double om_cf_point(const double *wl, const double *wr, double gamma);

/* bc.c */
void om_bc_ghost_state(const om_bc *bc, const double *n, const double *Wi, double gamma, double *Wg);
void om_bc_ghost_grad(const om_bc *bc, const double *n, const double *Gi, double *Gg);

/* recon.c */
int om_reconstruct_cell(const om_mesh *m, const om_params *p, const double *W, const double *G,
                        const double *alpha, int64_t c, double *coef /*[5][10]*/);
void om_eval_poly(const double *coef10, const double *dx, double *val, double *grad);

/* linear algebra */
int om_lu_solve(int n, double *A, double *b, int nrhs);

#endif
