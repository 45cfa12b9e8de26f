/*
 * CGKS CPU oracle -- fine-level residual, gradient update and time stepping.
 * TEST INFRASTRUCTURE ONLY (see om_internal.h).
 *
 * Paper passages:
 *  - semi-discrete finite volume update with face Gauss quadrature, fluxes in
 *    the local face frame: Sec. 2.2, Eq. (semidiscrete);
 *  - interface values W_{p,k}(t^{n+1}) and the Gauss-Green update of the
 *    cell-averaged gradients: Sec. 2.4, Eq. (gauss-formula);
 *  - gradient compression factor alpha_i = prod alpha_{p,k}, applied to the
 *    updated gradients and to the next Green-Gauss p^1: Sec. 3.3;
 *  - fine smoother W^{n+1} = W^n + dt_i/|Omega_i| Res(W^n): Sec. 4.2, Eq. (smo);
 *  - local time stepping on every level: Secs. 1, 4.3, 6.
 * Readings: local step dt_i = CFL |Omega_i| / sum_p lambda_p S_p with
 * lambda_p = |U.n_p| + c + 2 mu S_p / (rho |Omega_i|); face step = min of the
 * two cells; the CF product runs over interior faces (k from 1); the residual
 * norm is the RMS of rho-residual per unit volume.  The two-stage fourth-order
 * marching (cited by the paper for unsteady flow) uses flux integrals over dt
 * and dt/2; gradients at the intermediate stage come from W(dt/2), the final
 * ones from W^c,n + (W*(dt) - W^c,*).
 */
#include "om_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

static void prim_speed(const double *W, double gamma, double *U, double *c, double *rho)
{
    *rho = W[0];
    double q2 = 0;
    for (int d = 0; d < 3; ++d) {
        U[d] = W[1 + d] / W[0];
        q2 += U[d] * U[d];
    }
    double p = (gamma - 1.0) * (W[4] - 0.5 * W[0] * q2);
    *c = sqrt(gamma * p / W[0]);
}

int om_local_dt(const om_mesh *m, const om_params *p, const double *W, double *dt)
{
    const int64_t N = m->n_cells;
    int bad = -1;
    for (int64_t c = 0; c < N; ++c) {
        double Wc[5];
        for (int k = 0; k < 5; ++k) Wc[k] = W[k * N + c];
        double U[3], cs, rho;
        prim_speed(Wc, p->gamma, U, &cs, &rho);
        double sum = 0;
        for (int64_t q = m->cf_ptr[c]; q < m->cf_ptr[c + 1]; ++q) {
            int64_t f = m->cf_face[q];
            const double *A = &m->avec[3 * f];
            double na = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
            double un = fabs(U[0] * A[0] + U[1] * A[1] + U[2] * A[2]) / na;
            double S = m->area[f];
            double lam = un + cs + (p->viscous ? 2.0 * p->mu * S / (rho * m->vol[c]) : 0.0);
            sum += lam * S;
        }
        dt[c] = p->cfl * m->vol[c] / sum;
        if (!(dt[c] > 0) && bad < 0) bad = (int)c;
    }
    return bad < 0 ? 0 : -1;
}

/* Gradient compression factor of one Gauss point (Sec. 3.3) from the two reconstructed states in
 * the face frame (first momentum component along the normal): 1/(1 + A^2) with A the pressure
 * jump relative to each side's pressure plus the squared jumps of the normal and tangential Mach
 * numbers (tangential speed over sound speed). */
double om_cf_point(const double *wl, const double *wr, double gamma)
{
    double pr[2], man[2], mat[2];
    const double *S2[2] = {wl, wr};
    for (int s = 0; s < 2; ++s) {
        const double *ws = S2[s];
        double u = ws[1] / ws[0], v = ws[2] / ws[0], ww = ws[3] / ws[0];
        pr[s] = (gamma - 1.0) * (ws[4] - 0.5 * ws[0] * (u * u + v * v + ww * ww));
        double cs = sqrt(gamma * pr[s] / ws[0]);
        man[s] = u / cs;
        mat[s] = sqrt(v * v + ww * ww) / cs;
    }
    double dp = fabs(pr[0] - pr[1]);
    double A = dp / pr[0] + dp / pr[1] + (man[0] - man[1]) * (man[0] - man[1]) + (mat[0] - mat[1]) * (mat[0] - mat[1]);
    return 1.0 / (1.0 + A * A);
}

typedef struct {
    double F[5];      /* sum_k w_k S F_avg (along n, L -> R) */
    double Fh[5];     /* sum_k w_k S F_int(dt/2) */
    double Wdt[15];   /* sum_k w_k S W(dt) n_k */
    double Wh[15];    /* sum_k w_k S W(dt/2) n_k */
    double Wc[15];    /* sum_k w_k S W^c n_k */
    double alpha;
} facesum;

static int face_eval(const om_mesh *m, const om_params *p, const double *coef, int64_t f, double dtf, facesum *o)
{
    memset(o, 0, sizeof(*o));
    o->alpha = 1.0;
    const int64_t l = m->fl[f], r = m->fr[f];
    for (int k = 0; k < m->ngp[f]; ++k) {
        const double *x = &m->gpx[3 * (OM_MAXGP * f + k)];
        const double *n = &m->gpn[3 * (OM_MAXGP * f + k)];
        const double w = m->gpw[OM_MAXGP * f + k] * m->area[f];
        double WL[5], GL[15], WR[5], GR[15];
        double dxl[3] = {x[0] - m->cen[3 * l], x[1] - m->cen[3 * l + 1], x[2] - m->cen[3 * l + 2]};
        for (int q = 0; q < 5; ++q) om_eval_poly(&coef[50 * l + 10 * q], dxl, &WL[q], &GL[3 * q]);
        if (r >= 0) {
            double dxr[3];
            for (int d = 0; d < 3; ++d) dxr[d] = x[d] - m->shift[3 * f + d] - m->cen[3 * r + d];
            for (int q = 0; q < 5; ++q) om_eval_poly(&coef[50 * r + 10 * q], dxr, &WR[q], &GR[3 * q]);
        } else {
            const om_bc *bc = &m->bc[m->ftag[f] & 63];
            om_bc_ghost_state(bc, n, WL, p->gamma, WR);
            om_bc_ghost_grad(bc, n, GL, GR);
        }
        double t1[3], t2[3];
        om_frame(n, t1, t2);
        double wl[5], wr[5], gl[15], gr[15];
        om_rotate_state(WL, n, t1, t2, wl);
        om_rotate_state(WR, n, t1, t2, wr);
        om_rotate_grad(GL, n, t1, t2, gl);
        om_rotate_grad(GR, n, t1, t2, gr);
        om_gks_out g;
        int e = om_gks_point(wl, gl, wr, gr, dtf, p, &g);
        if (e) return e;
        double F[5], Fh[5], Wd[5], Whf[5], Wcc[5];
        om_rotate_back(g.F, n, t1, t2, F);
        om_rotate_back(g.Fhalf, n, t1, t2, Fh);
        om_rotate_back(g.Wdt, n, t1, t2, Wd);
        om_rotate_back(g.Whalf, n, t1, t2, Whf);
        om_rotate_back(g.Wc, n, t1, t2, Wcc);
        for (int q = 0; q < 5; ++q) {
            o->F[q] += w * F[q];
            o->Fh[q] += w * Fh[q];
            for (int d = 0; d < 3; ++d) {
                o->Wdt[3 * q + d] += w * Wd[q] * n[d];
                o->Wh[3 * q + d] += w * Whf[q] * n[d];
                o->Wc[3 * q + d] += w * Wcc[q] * n[d];
            }
        }
        if (r >= 0) o->alpha *= om_cf_point(wl, wr, p->gamma);
    }
    return 0;
}

/* per-cell sums over its faces in CSR order */
typedef struct {
    double *R;     /* 5N  -sum s S w F_avg */
    double *Rh;    /* 5N  -sum s S w F_int(dt/2) */
    double *Sdt;   /* 15N sum outward W(dt) n S w */
    double *Sh;    /* 15N */
    double *Sc;    /* 15N */
    double *alpha; /* N */
} cellsums;

/* Evaluate all faces touching the cells marked in `need_out` (all when NULL). */
static int residual_core(const om_mesh *m, const om_params *p, const double *W, const double *G, const double *alpha,
                         const double *dtc, double dt_global, const int64_t *sub, int64_t nsub, cellsums *cs,
                         int64_t *bad_cell)
{
    const int64_t N = m->n_cells, NF = m->n_faces;
    char *need_out = (char *)calloc(N, 1), *need_rec = (char *)calloc(N, 1), *need_face = (char *)calloc(NF, 1);
    if (sub) {
        for (int64_t i = 0; i < nsub; ++i) need_out[sub[i]] = 1;
    } else
        memset(need_out, 1, N);
    for (int64_t c = 0; c < N; ++c)
        if (need_out[c])
            for (int64_t q = m->cf_ptr[c]; q < m->cf_ptr[c + 1]; ++q) {
                int64_t f = m->cf_face[q];
                need_face[f] = 1;
                need_rec[m->fl[f]] = 1;
                if (m->fr[f] >= 0) need_rec[m->fr[f]] = 1;
            }
    double *coef = (double *)calloc(50 * N, sizeof(double));
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < N; ++c) {
        if (!need_rec[c]) continue;
        int e = om_reconstruct_cell(m, p, W, G, alpha, c, &coef[50 * c]);
        if (e) {
#pragma omp critical
            {
                if (!err || c < *bad_cell) *bad_cell = c;
                err = e;
            }
        }
    }
    facesum *fs = NULL;
    if (!err) {
        fs = (facesum *)calloc(NF, sizeof(facesum));
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t f = 0; f < NF; ++f) {
            if (!need_face[f]) continue;
            double dtf = dt_global;
            if (dtf <= 0) {
                dtf = dtc[m->fl[f]];
                if (m->fr[f] >= 0 && dtc[m->fr[f]] < dtf) dtf = dtc[m->fr[f]];
            }
            int e = face_eval(m, p, coef, f, dtf, &fs[f]);
            if (e) {
#pragma omp critical
                {
                    if (!err || m->fl[f] < *bad_cell) *bad_cell = m->fl[f];
                    err = e;
                }
            }
        }
    }
    if (!err) {
        for (int64_t c = 0; c < N; ++c) {
            if (!need_out[c]) continue;
            double R[5] = {0}, Rh[5] = {0}, Sd[15] = {0}, Sh[15] = {0}, Sc[15] = {0}, al = 1.0;
            for (int64_t q = m->cf_ptr[c]; q < m->cf_ptr[c + 1]; ++q) {
                const facesum *o = &fs[m->cf_face[q]];
                double s = m->cf_sign[q];
                for (int k = 0; k < 5; ++k) {
                    R[k] -= s * o->F[k];
                    Rh[k] -= s * o->Fh[k];
                }
                for (int k = 0; k < 15; ++k) {
                    Sd[k] += s * o->Wdt[k];
                    Sh[k] += s * o->Wh[k];
                    Sc[k] += s * o->Wc[k];
                }
                al *= o->alpha;
            }
            for (int k = 0; k < 5; ++k) {
                if (cs->R) cs->R[k * N + c] = R[k];
                if (cs->Rh) cs->Rh[k * N + c] = Rh[k];
            }
            for (int k = 0; k < 15; ++k) {
                if (cs->Sdt) cs->Sdt[k * N + c] = Sd[k];
                if (cs->Sh) cs->Sh[k * N + c] = Sh[k];
                if (cs->Sc) cs->Sc[k * N + c] = Sc[k];
            }
            if (cs->alpha) cs->alpha[c] = al;
        }
    }
    free(fs);
    free(coef);
    free(need_out);
    free(need_rec);
    free(need_face);
    return err;
}

/*
 * Steady residual with local time stepping:
 *   R[5N]      = -sum_p S_p sum_k w_k F_avg(x_pk) . n (time average over the face step)
 *   Gnew[15N]  = alpha_new / |Omega| * sum_p sum_k w_k W_pk(dt_f) n_pk S_p
 *   alpha_new  = prod over interior faces and Gauss points of alpha_pk
 *   dt[N]      = local time steps (computed from W)
 * With `sub` only the listed cells are written.
 */
int om_residual(const om_mesh *m, const om_params *p, const double *W, const double *G, const double *alpha,
                double *R, double *Gnew, double *alpha_new, double *dt, const int64_t *sub, int64_t nsub,
                int64_t *bad_cell)
{
    const int64_t N = m->n_cells;
    double *dtc = (double *)malloc(sizeof(double) * N);
    *bad_cell = -1;
    if (om_local_dt(m, p, W, dtc)) {
        free(dtc);
        return -5;
    }
    double *Sdt = Gnew ? (double *)calloc(15 * N, sizeof(double)) : NULL;
    double *al = (double *)calloc(N, sizeof(double));
    cellsums cs = {R, NULL, Sdt, NULL, NULL, al};
    int e = residual_core(m, p, W, G, alpha, dtc, -1.0, sub, nsub, &cs, bad_cell);
    if (!e) {
        for (int64_t c = 0; c < N; ++c) {
            if (sub) continue;
            if (Gnew)
                for (int k = 0; k < 15; ++k) Gnew[k * N + c] = al[c] * Sdt[k * N + c] / m->vol[c];
            if (alpha_new) alpha_new[c] = al[c];
        }
        if (sub)
            for (int64_t i = 0; i < nsub; ++i) {
                int64_t c = sub[i];
                if (Gnew)
                    for (int k = 0; k < 15; ++k) Gnew[k * N + c] = al[c] * Sdt[k * N + c] / m->vol[c];
                if (alpha_new) alpha_new[c] = al[c];
            }
        if (dt) memcpy(dt, dtc, sizeof(double) * N);
    }
    free(Sdt);
    free(al);
    free(dtc);
    return e;
}

double om_residual_norm(const om_mesh *m, const double *R)
{
    double s = 0;
    for (int64_t c = 0; c < m->n_cells; ++c) {
        double v = R[c] / m->vol[c];
        s += v * v;
    }
    return sqrt(s / (double)m->n_cells);
}

/* one explicit fine smoothing step (forward Euler, local time step); returns residual norm */
int om_step_fe(const om_mesh *m, const om_params *p, double *W, double *G, double *alpha, double *resnorm,
               int64_t *bad_cell)
{
    const int64_t N = m->n_cells;
    double *R = (double *)malloc(sizeof(double) * 5 * N), *Gn = (double *)malloc(sizeof(double) * 15 * N);
    double *an = (double *)malloc(sizeof(double) * N), *dt = (double *)malloc(sizeof(double) * N);
    int e = om_residual(m, p, W, G, alpha, R, Gn, an, dt, NULL, 0, bad_cell);
    if (!e) {
        for (int64_t c = 0; c < N; ++c)
            for (int k = 0; k < 5; ++k) W[k * N + c] += dt[c] / m->vol[c] * R[k * N + c];
        memcpy(G, Gn, sizeof(double) * 15 * N);
        memcpy(alpha, an, sizeof(double) * N);
        if (resnorm) *resnorm = om_residual_norm(m, R);
    }
    free(R);
    free(Gn);
    free(an);
    free(dt);
    return e;
}

/* one two-stage fourth-order step with a global time step dt */
int om_step_s2o4(const om_mesh *m, const om_params *p, double dt, double *W, double *G, double *alpha,
                 int64_t *bad_cell)
{
    const int64_t N = m->n_cells;
    double *R1 = malloc(sizeof(double) * 5 * N), *Rh1 = malloc(sizeof(double) * 5 * N);
    double *Sh1 = malloc(sizeof(double) * 15 * N), *Sc1 = malloc(sizeof(double) * 15 * N);
    double *a1 = malloc(sizeof(double) * N);
    double *R2 = malloc(sizeof(double) * 5 * N), *Rh2 = malloc(sizeof(double) * 5 * N);
    double *Sd2 = malloc(sizeof(double) * 15 * N), *Sc2 = malloc(sizeof(double) * 15 * N);
    double *a2 = malloc(sizeof(double) * N);
    double *Ws = malloc(sizeof(double) * 5 * N), *Gs = malloc(sizeof(double) * 15 * N);
    *bad_cell = -1;
    cellsums c1 = {R1, Rh1, NULL, Sh1, Sc1, a1};
    int e = residual_core(m, p, W, G, alpha, NULL, dt, NULL, 0, &c1, bad_cell);
    if (!e) {
        for (int64_t c = 0; c < N; ++c) {
            double V = m->vol[c];
            for (int k = 0; k < 5; ++k) {
                double I = R1[k * N + c] * dt, Ih = Rh1[k * N + c];
                double L = (4.0 * Ih - I) / (dt * V);
                double Lt = 4.0 * (I - 2.0 * Ih) / (dt * dt * V);
                Ws[k * N + c] = W[k * N + c] + 0.5 * dt * L + 0.125 * dt * dt * Lt;
            }
            for (int k = 0; k < 15; ++k) Gs[k * N + c] = a1[c] * Sh1[k * N + c] / V;
        }
        cellsums c2 = {R2, Rh2, Sd2, NULL, Sc2, a2};
        e = residual_core(m, p, Ws, Gs, a1, NULL, dt, NULL, 0, &c2, bad_cell);
    }
    if (!e) {
        for (int64_t c = 0; c < N; ++c) {
            double V = m->vol[c];
            for (int k = 0; k < 5; ++k) {
                double I1 = R1[k * N + c] * dt, Ih1 = Rh1[k * N + c];
                double I2 = R2[k * N + c] * dt, Ih2 = Rh2[k * N + c];
                double L1 = (4.0 * Ih1 - I1) / (dt * V);
                double Lt1 = 4.0 * (I1 - 2.0 * Ih1) / (dt * dt * V);
                double Lt2 = 4.0 * (I2 - 2.0 * Ih2) / (dt * dt * V);
                W[k * N + c] += dt * L1 + dt * dt / 6.0 * (Lt1 + 2.0 * Lt2);
            }
            for (int k = 0; k < 15; ++k)
                G[k * N + c] = a2[c] * (Sc1[k * N + c] + Sd2[k * N + c] - Sc2[k * N + c]) / V;
            alpha[c] = a2[c];
        }
    }
    free(R1);
    free(Rh1);
    free(Sh1);
    free(Sc1);
    free(a1);
    free(R2);
    free(Rh2);
    free(Sd2);
    free(Sc2);
    free(a2);
    free(Ws);
    free(Gs);
    return e;
}

/* reconstruction coefficients of all cells ([N][5][10]) for pins */
int om_reconstruct_all(const om_mesh *m, const om_params *p, const double *W, const double *G, const double *alpha,
                       double *coef)
{
    for (int64_t c = 0; c < m->n_cells; ++c)
        if (om_reconstruct_cell(m, p, W, G, alpha, c, &coef[50 * c])) return (int)c + 1;
    return 0;
}

/*
 * Force of the gas on the boundary faces carrying `tag` (the drag/lift integrand of the
 * sphere and bump results, Sec. 5): the momentum components of the face flux,
 *   F = sum_{faces with tag} S_p sum_k w_k F_mom(x_pk),
 * with the same reconstruction, local face step and time-averaged BGK flux as the residual
 * (Sec. 2.2, Eq. 2nd-flux, Eq. gauss-formula), the normal pointing out of the gas.  Faces are
 * summed in ascending face order.
 */
int om_wall_force(const om_mesh *m, const om_params *p, const double *W, const double *G, const double *alpha,
                  int32_t tag, double Fout[3], int64_t *bad_cell)
{
    const int64_t N = m->n_cells, NF = m->n_faces;
    *bad_cell = -1;
    Fout[0] = Fout[1] = Fout[2] = 0.0;
    double *dtc = (double *)malloc(sizeof(double) * N);
    if (om_local_dt(m, p, W, dtc)) {
        free(dtc);
        return -5;
    }
    double *coef = (double *)calloc(50 * N, sizeof(double));
    int err = 0;
    for (int64_t f = 0; f < NF && !err; ++f) {
        if (m->fr[f] >= 0 || m->ftag[f] != tag) continue;
        const int64_t l = m->fl[f];
        err = om_reconstruct_cell(m, p, W, G, alpha, l, &coef[50 * l]);
        if (err) {
            *bad_cell = l;
            break;
        }
        facesum s;
        err = face_eval(m, p, coef, f, dtc[l], &s);
        if (err) {
            *bad_cell = l;
            break;
        }
        for (int d = 0; d < 3; ++d) Fout[d] += s.F[1 + d];
    }
    free(coef);
    free(dtc);
    return err;
}
