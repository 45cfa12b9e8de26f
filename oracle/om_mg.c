/*
 * CGKS CPU oracle -- geometric multigrid: coarse levels, KFVS coarse operator,
 * restriction, forcing term, coarse sweeps, correction and the V-cycle.
 * TEST INFRASTRUCTURE ONLY (see om_internal.h).
 *
 * Paper Sec. 4.2 (geometric multigrid and p-multigrid for the third-order CGKS):
 *  - fine smoother = one explicit CGKS step, Eq. (smo);
 *  - state restriction W_2h^0 = sum V_i W_i / V_2h;
 *  - residual restriction Res*_2h = sum Res_i^{n+1} (the fine residual at the
 *    smoothed state);
 *  - forcing F = Res*_2h - Res_2h(W_2h^0);
 *  - coarse update W^{k+1} = W^k + dt/V (Res_2h(W^k) + F) with first-order KFVS
 *    and local time steps (Secs. 1, 4.2, 6);
 *  - correction W_h* = W_h^{n+1} + (W_2h^{k+1} - W_2h^0), averages only;
 *  - three-level V-cycle, one pre-smoothing and no post-smoothing by default;
 *  - optionally the implicit coarse smoother of Sec. 4.3 (om_coarse_implicit);
 *  - optionally gamma > 1 visits of each coarser level per visit of its parent
 *    (gamma = 2: W-cycle), each continuing from the level's state with its forcing.
 * Readings: coarse faces carry the summed fine area vectors (n = A/|A|,
 * S = |A|); coarse boundary faces are the fine boundary faces with the coarse
 * owner's ghost state; the coarse operator is inviscid KFVS, its local time
 * step uses the fine formula on coarse geometry with |U.A| for the convective
 * part and the summed fine face area S for the acoustic and viscous parts (an
 * agglomerate enclosed by another has a closed interface with A = 0); a level
 * below the second
 * restricts the level's state and (Res_2h(W_2h) + F) as its Res*.
 */
#include "om_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

int64_t om_agglomerate_graph(int64_t n, const double *V, const double *P, int64_t m, const int64_t *pa,
                             const int64_t *pb, const double *S, const double *M, const double *A, uint64_t seed,
                             int passes, double delta, double smin, int64_t *f2c, double *Vo, double *Po,
                             int64_t *m_out, int64_t *pao, int64_t *pbo, double *So, double *Mo, double *Ao,
                             int64_t *stats);
int om_residual(const om_mesh *m, const om_params *p, const double *W, const double *G, const double *alpha,
                double *R, double *Gnew, double *alpha_new, double *dt, const int64_t *sub, int64_t nsub,
                int64_t *bad_cell);
double om_residual_norm(const om_mesh *m, const double *R);

typedef struct {
    int64_t n, m, nb;
    double *V, *P;
    int64_t *a, *b;
    double *S, *M, *A; /* pair geometry: summed fine areas, first moments, area vectors */
    char *per;         /* pair crosses a periodic boundary */
    int64_t *bown;
    int32_t *btag;
    double *bA;        /* fine boundary faces */
    int64_t *f2c;      /* map from the next finer level */
} om_level;

typedef struct {
    const om_mesh *mesh;
    int nlev;
    om_level lev[8];   /* lev[0] = fine graph */
    int64_t stats[8][4 * 16];
} om_hier;

static void level_free(om_level *L)
{
    free(L->V);
    free(L->P);
    free(L->a);
    free(L->b);
    free(L->S);
    free(L->M);
    free(L->A);
    free(L->per);
    free(L->bown);
    free(L->btag);
    free(L->bA);
    free(L->f2c);
}

void om_hier_free(om_hier *h)
{
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) level_free(&h->lev[l]);
    free(h);
}

/* fine graph: non-periodic interior faces as pairs, boundary faces kept */
static void fine_level(const om_mesh *m, om_level *L)
{
    memset(L, 0, sizeof(*L));
    int64_t N = m->n_cells;
    L->n = N;
    L->V = malloc(sizeof(double) * N);
    L->P = malloc(sizeof(double) * 3 * N);
    for (int64_t c = 0; c < N; ++c) {
        L->V[c] = m->vol[c];
        for (int d = 0; d < 3; ++d) L->P[3 * c + d] = m->vol[c] * m->cen[3 * c + d];
    }
    int64_t cnt = 0, nb = 0;
    for (int64_t f = 0; f < m->n_faces; ++f) {
        if (m->fr[f] < 0) {
            ++nb;
            continue;
        }
        ++cnt;
    }
    L->a = malloc(sizeof(int64_t) * (cnt + 1));
    L->b = malloc(sizeof(int64_t) * (cnt + 1));
    L->S = malloc(sizeof(double) * (cnt + 1));
    L->M = malloc(sizeof(double) * 3 * (cnt + 1));
    L->A = malloc(sizeof(double) * 3 * (cnt + 1));
    L->per = calloc(cnt + 1, 1);
    L->bown = malloc(sizeof(int64_t) * (nb + 1));
    L->btag = malloc(sizeof(int32_t) * (nb + 1));
    L->bA = malloc(sizeof(double) * 3 * (nb + 1));
    int64_t j = 0, k = 0;
    for (int64_t f = 0; f < m->n_faces; ++f) {
        if (m->fr[f] < 0) {
            L->bown[k] = m->fl[f];
            L->btag[k] = m->ftag[f];
            for (int d = 0; d < 3; ++d) L->bA[3 * k + d] = m->avec[3 * f + d];
            ++k;
            continue;
        }
        /* pairs sorted by (l, r) already; duplicates between the same cells merged */
        int periodic = m->shift[3 * f] != 0 || m->shift[3 * f + 1] != 0 || m->shift[3 * f + 2] != 0;
        if (j > 0 && L->a[j - 1] == m->fl[f] && L->b[j - 1] == m->fr[f] && !periodic && !L->per[j - 1]) {
            L->S[j - 1] += m->area[f];
            for (int d = 0; d < 3; ++d) {
                L->M[3 * (j - 1) + d] += m->fmom[3 * f + d];
                L->A[3 * (j - 1) + d] += m->avec[3 * f + d];
            }
            continue;
        }
        L->a[j] = m->fl[f];
        L->b[j] = m->fr[f];
        L->S[j] = m->area[f];
        L->per[j] = (char)periodic;
        for (int d = 0; d < 3; ++d) {
            L->M[3 * j + d] = m->fmom[3 * f + d];
            L->A[3 * j + d] = m->avec[3 * f + d];
        }
        ++j;
    }
    L->m = j;
    L->nb = k;
}

/*
 * Build `levels` levels with `passes` agglomeration passes each.  Periodic pairs are
 * never candidates; they stay as coarse interior pairs.
 */
om_hier *om_hier_build(const om_mesh *m, int levels, int passes, uint64_t seed, double delta, double smin)
{
    om_hier *h = calloc(1, sizeof(om_hier));
    h->mesh = m;
    h->nlev = levels;
    fine_level(m, &h->lev[0]);
    for (int l = 1; l < levels; ++l) {
        om_level *F = &h->lev[l - 1], *C = &h->lev[l];
        memset(C, 0, sizeof(*C));
        /* candidate graph excludes periodic pairs */
        int64_t mc = 0;
        for (int64_t j = 0; j < F->m; ++j) mc += !F->per[j];
        int64_t *ga = malloc(sizeof(int64_t) * (mc + 1)), *gb = malloc(sizeof(int64_t) * (mc + 1));
        double *gS = malloc(sizeof(double) * (mc + 1)), *gM = malloc(sizeof(double) * 3 * (mc + 1)),
               *gA = malloc(sizeof(double) * 3 * (mc + 1));
        int64_t q = 0;
        for (int64_t j = 0; j < F->m; ++j) {
            if (F->per[j]) continue;
            ga[q] = F->a[j];
            gb[q] = F->b[j];
            gS[q] = F->S[j];
            for (int d = 0; d < 3; ++d) {
                gM[3 * q + d] = F->M[3 * j + d];
                gA[3 * q + d] = F->A[3 * j + d];
            }
            ++q;
        }
        C->f2c = malloc(sizeof(int64_t) * F->n);
        C->V = malloc(sizeof(double) * F->n);
        C->P = malloc(sizeof(double) * 3 * F->n);
        int64_t *pa = malloc(sizeof(int64_t) * (mc + 1)), *pb = malloc(sizeof(int64_t) * (mc + 1));
        double *pS = malloc(sizeof(double) * (mc + 1)), *pM = malloc(sizeof(double) * 3 * (mc + 1)),
               *pA = malloc(sizeof(double) * 3 * (mc + 1));
        int64_t mo = 0;
        C->n = om_agglomerate_graph(F->n, F->V, F->P, mc, ga, gb, gS, gM, gA, seed, passes, delta, smin, C->f2c, C->V,
                                    C->P, &mo, pa, pb, pS, pM, pA, h->stats[l]);
        /* periodic pairs of the finer level become coarse pairs (not merged with others) */
        int64_t nper = F->m - mc;
        C->a = malloc(sizeof(int64_t) * (mo + nper + 1));
        C->b = malloc(sizeof(int64_t) * (mo + nper + 1));
        C->S = malloc(sizeof(double) * (mo + nper + 1));
        C->M = malloc(sizeof(double) * 3 * (mo + nper + 1));
        C->A = malloc(sizeof(double) * 3 * (mo + nper + 1));
        C->per = calloc(mo + nper + 1, 1);
        memcpy(C->a, pa, sizeof(int64_t) * mo);
        memcpy(C->b, pb, sizeof(int64_t) * mo);
        memcpy(C->S, pS, sizeof(double) * mo);
        memcpy(C->M, pM, sizeof(double) * 3 * mo);
        memcpy(C->A, pA, sizeof(double) * 3 * mo);
        int64_t r = mo;
        for (int64_t j = 0; j < F->m; ++j) {
            if (!F->per[j]) continue;
            int64_t a = C->f2c[F->a[j]], b = C->f2c[F->b[j]];
            C->a[r] = a;
            C->b[r] = b;
            C->S[r] = F->S[j];
            C->per[r] = 1;
            for (int d = 0; d < 3; ++d) {
                C->M[3 * r + d] = 0;
                C->A[3 * r + d] = F->A[3 * j + d];
            }
            ++r;
        }
        C->m = r;
        C->nb = F->nb;
        C->bown = malloc(sizeof(int64_t) * (F->nb + 1));
        C->btag = malloc(sizeof(int32_t) * (F->nb + 1));
        C->bA = malloc(sizeof(double) * 3 * (F->nb + 1));
        for (int64_t k = 0; k < F->nb; ++k) {
            C->bown[k] = C->f2c[F->bown[k]];
            C->btag[k] = F->btag[k];
            for (int d = 0; d < 3; ++d) C->bA[3 * k + d] = F->bA[3 * k + d];
        }
        free(ga);
        free(gb);
        free(gS);
        free(gM);
        free(gA);
        free(pa);
        free(pb);
        free(pS);
        free(pM);
        free(pA);
    }
    return h;
}

int64_t om_hier_level_size(const om_hier *h, int l, int64_t *m, int64_t *nb)
{
    if (m) *m = h->lev[l].m;
    if (nb) *nb = h->lev[l].nb;
    return h->lev[l].n;
}

void om_hier_level_get(const om_hier *h, int l, int64_t *f2c, double *V, double *P, int64_t *a, int64_t *b, double *A,
                       int64_t *stats)
{
    const om_level *L = &h->lev[l];
    if (f2c && L->f2c) memcpy(f2c, L->f2c, sizeof(int64_t) * h->lev[l - 1].n);
    if (V) memcpy(V, L->V, sizeof(double) * L->n);
    if (P) memcpy(P, L->P, sizeof(double) * 3 * L->n);
    if (a) memcpy(a, L->a, sizeof(int64_t) * L->m);
    if (b) memcpy(b, L->b, sizeof(int64_t) * L->m);
    if (A) memcpy(A, L->A, sizeof(double) * 3 * L->m);
    if (stats) memcpy(stats, h->stats[l], sizeof(h->stats[l]));
}

/* boundary faces of level l: owner, tag and outward area vector (3 per face) */
void om_hier_level_boundary(const om_hier *h, int l, int64_t *bown, int32_t *btag, double *bA)
{
    const om_level *L = &h->lev[l];
    if (bown) memcpy(bown, L->bown, sizeof(int64_t) * L->nb);
    if (btag) memcpy(btag, L->btag, sizeof(int32_t) * L->nb);
    if (bA) memcpy(bA, L->bA, sizeof(double) * 3 * L->nb);
}

/* KFVS residual on level l (l >= 1): R = - sum S n . F over coarse faces */
int om_kfvs_residual(const om_hier *h, int l, const om_params *p, const double *W, double *R)
{
    const om_level *L = &h->lev[l];
    const int64_t N = L->n;
    for (int64_t i = 0; i < 5 * N; ++i) R[i] = 0;
    for (int64_t j = 0; j < L->m; ++j) {
        const double *A = &L->A[3 * j];
        double S = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        if (S == 0) continue;
        double n[3] = {A[0] / S, A[1] / S, A[2] / S}, t1[3], t2[3];
        om_frame(n, t1, t2);
        double Wa[5], Wb[5], wa[5], wb[5], Fl[5], F[5];
        for (int k = 0; k < 5; ++k) {
            Wa[k] = W[k * N + L->a[j]];
            Wb[k] = W[k * N + L->b[j]];
        }
        om_rotate_state(Wa, n, t1, t2, wa);
        om_rotate_state(Wb, n, t1, t2, wb);
        om_kfvs_point(wa, wb, p->gamma, Fl);
        om_rotate_back(Fl, n, t1, t2, F);
        for (int k = 0; k < 5; ++k) {
            R[k * N + L->a[j]] -= S * F[k];
            R[k * N + L->b[j]] += S * F[k];
        }
    }
    for (int64_t k2 = 0; k2 < L->nb; ++k2) {
        const double *A = &L->bA[3 * k2];
        double S = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        double n[3] = {A[0] / S, A[1] / S, A[2] / S}, t1[3], t2[3];
        om_frame(n, t1, t2);
        int64_t o = L->bown[k2];
        double Wa[5], Wg[5], wa[5], wg[5], Fl[5], F[5];
        for (int k = 0; k < 5; ++k) Wa[k] = W[k * N + o];
        om_bc_ghost_state(&h->mesh->bc[L->btag[k2] & 63], n, Wa, p->gamma, Wg);
        om_rotate_state(Wa, n, t1, t2, wa);
        om_rotate_state(Wg, n, t1, t2, wg);
        om_kfvs_point(wa, wg, p->gamma, Fl);
        om_rotate_back(Fl, n, t1, t2, F);
        for (int k = 0; k < 5; ++k) R[k * N + o] -= S * F[k];
    }
    return 0;
}

/* local time step on level l >= 1 */
void om_coarse_dt(const om_hier *h, int l, const om_params *p, const double *W, double *dt)
{
    const om_level *L = &h->lev[l];
    const int64_t N = L->n;
    double *sum = calloc(N, sizeof(double));
    double *U = malloc(sizeof(double) * 3 * N), *cs = malloc(sizeof(double) * N);
    for (int64_t c = 0; c < N; ++c) {
        double q2 = 0;
        for (int d = 0; d < 3; ++d) {
            U[3 * c + d] = W[(1 + d) * N + c] / W[c];
            q2 += U[3 * c + d] * U[3 * c + d];
        }
        double pr = (p->gamma - 1.0) * (W[4 * N + c] - 0.5 * W[c] * q2);
        cs[c] = sqrt(p->gamma * pr / W[c]);
    }
    for (int64_t j = 0; j < L->m; ++j) {
        /* |U . A| + (c + 2 mu S / (rho V)) S with S the summed fine area of the coarse face */
        const double *A = &L->A[3 * j];
        double S = L->S[j];
        int64_t ab[2] = {L->a[j], L->b[j]};
        for (int s = 0; s < 2; ++s) {
            int64_t c = ab[s];
            double uA = fabs(U[3 * c] * A[0] + U[3 * c + 1] * A[1] + U[3 * c + 2] * A[2]);
            double lam = cs[c] + (p->viscous ? 2.0 * p->mu * S / (W[c] * L->V[c]) : 0.0);
            sum[c] += uA + lam * S;
        }
    }
    for (int64_t k = 0; k < L->nb; ++k) {
        const double *A = &L->bA[3 * k];
        double S = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        int64_t c = L->bown[k];
        double un = fabs(U[3 * c] * A[0] + U[3 * c + 1] * A[1] + U[3 * c + 2] * A[2]) / S;
        double lam = un + cs[c] + (p->viscous ? 2.0 * p->mu * S / (W[c] * L->V[c]) : 0.0);
        sum[c] += lam * S;
    }
    for (int64_t c = 0; c < N; ++c) dt[c] = p->cfl * L->V[c] / sum[c];
    free(sum);
    free(U);
    free(cs);
}

/* restriction from level l-1 to l: Wc = sum V W / Vc, Rc = sum R */
void om_restrict(const om_hier *h, int l, const double *Wf, const double *Rf, double *Wc, double *Rc)
{
    const om_level *F = &h->lev[l - 1], *C = &h->lev[l];
    const int64_t Nf = F->n, Nc = C->n;
    for (int64_t i = 0; i < 5 * Nc; ++i) {
        if (Wc) Wc[i] = 0;
        if (Rc) Rc[i] = 0;
    }
    /* ascending fine id within each coarse cell */
    for (int64_t i = 0; i < Nf; ++i) {
        int64_t c = C->f2c[i];
        for (int k = 0; k < 5; ++k) {
            if (Wc) Wc[k * Nc + c] += F->V[i] * Wf[k * Nf + i];
            if (Rc) Rc[k * Nc + c] += Rf[k * Nf + i];
        }
    }
    if (Wc)
        for (int64_t c = 0; c < Nc; ++c)
            for (int k = 0; k < 5; ++k) Wc[k * Nc + c] /= C->V[c];
}

/* prolongation (injection of the correction): Wf += dWc[f2c] */
void om_prolong(const om_hier *h, int l, const double *dWc, double *Wf)
{
    const om_level *F = &h->lev[l - 1], *C = &h->lev[l];
    const int64_t Nf = F->n, Nc = C->n;
    for (int64_t i = 0; i < Nf; ++i)
        for (int k = 0; k < 5; ++k) Wf[k * Nf + i] += dWc[k * Nc + C->f2c[i]];
}

/*
 * Implicit coarse smoother, paper Sec. 4.3.  Backward Euler on the coarse
 * level, linearised with the Jacobian of a first-order Lax-Friedrichs flux:
 * A+- = (A +- lambda I)/2 with lambda the larger of the two cells' spectral
 * radii |U.n| + c + 2 mu S/(rho |Omega|) (the viscous term carries 1/rho so
 * that it is a rate).  Because the outward area vectors of a closed cell sum
 * to zero, the A part of A+ drops out of the diagonal, which is
 * |Omega_i|/dt_i + (1/2) sum_p lambda_p S_p.  The off-diagonal product is
 * taken without a matrix: A-_p dU_p ~ F-(U_p + dU_p) - F-(U_p) with
 * F-(U) = (F_n(U) - lambda U)/2 and F_n the Euler flux along the outward
 * normal of cell i.  The system
 *     D_i dU_i + sum_p [F-(U_p + dU_p) - F-(U_p)] S_p = rhs_i
 * is solved by point relaxation: dU^0 = rhs/D, then each sweep recomputes
 * every cell from the previous sweep's neighbour increments.
 * Readings: S is the coarse face's |A| (the factor of its KFVS flux);
 * boundary faces add lambda S/2 to the diagonal with lambda the larger of the
 * owner's and the ghost state's radius, and their ghost increment is zero;
 * dt_i is the coarse local step with the implicit CFL number.
 */
static void euler_flux_n(const double *U, const double *n, double gamma, double *F)
{
    const double rho = U[0];
    const double u[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
    const double pr = (gamma - 1.0) * (U[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
    const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    F[0] = rho * un;
    for (int d = 0; d < 3; ++d) F[1 + d] = U[1 + d] * un + pr * n[d];
    F[4] = (U[4] + pr) * un;
}

static double spectral_radius(const double *U, const double *n, double S, double V, const om_params *p)
{
    const double rho = U[0];
    const double u[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
    const double pr = (p->gamma - 1.0) * (U[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
    const double c = sqrt(p->gamma * pr / rho);
    const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    return fabs(un) + c + (p->viscous ? 2.0 * p->mu * S / (rho * V) : 0.0);
}

void om_coarse_implicit(const om_hier *h, int l, const om_params *p, const double *W, const double *rhs, double *dU)
{
    const om_level *L = &h->lev[l];
    const int64_t N = L->n;
    double *dt = malloc(sizeof(double) * N), *diag = malloc(sizeof(double) * N);
    double *lam = calloc(L->m > 0 ? L->m : 1, sizeof(double));
    double *prev = malloc(sizeof(double) * 5 * N), *acc = malloc(sizeof(double) * 5 * N);
    om_params pi = *p;
    pi.cfl = p->cfl_implicit;
    om_coarse_dt(h, l, &pi, W, dt);
    for (int64_t c = 0; c < N; ++c) diag[c] = L->V[c] / dt[c];
    for (int64_t j = 0; j < L->m; ++j) {
        const double *A = &L->A[3 * j];
        const double S = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        if (S == 0) continue;
        const double n[3] = {A[0] / S, A[1] / S, A[2] / S};
        double Ua[5], Ub[5];
        for (int k = 0; k < 5; ++k) {
            Ua[k] = W[k * N + L->a[j]];
            Ub[k] = W[k * N + L->b[j]];
        }
        const double la = spectral_radius(Ua, n, S, L->V[L->a[j]], p);
        const double lb = spectral_radius(Ub, n, S, L->V[L->b[j]], p);
        lam[j] = la > lb ? la : lb;
        diag[L->a[j]] += 0.5 * lam[j] * S;
        diag[L->b[j]] += 0.5 * lam[j] * S;
    }
    for (int64_t q = 0; q < L->nb; ++q) {
        const double *A = &L->bA[3 * q];
        const double S = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        const double n[3] = {A[0] / S, A[1] / S, A[2] / S};
        const int64_t o = L->bown[q];
        double Uo[5], Ug[5];
        for (int k = 0; k < 5; ++k) Uo[k] = W[k * N + o];
        om_bc_ghost_state(&h->mesh->bc[L->btag[q] & 63], n, Uo, p->gamma, Ug);
        const double lo = spectral_radius(Uo, n, S, L->V[o], p);
        const double lg = spectral_radius(Ug, n, S, L->V[o], p);
        diag[o] += 0.5 * (lo > lg ? lo : lg) * S;
    }
    for (int64_t c = 0; c < N; ++c)
        for (int k = 0; k < 5; ++k) dU[k * N + c] = rhs[k * N + c] / diag[c];
    for (int sweep = 0; sweep < p->relax_sweeps; ++sweep) {
        memcpy(prev, dU, sizeof(double) * 5 * N);
        memcpy(acc, rhs, sizeof(double) * 5 * N);
        for (int64_t j = 0; j < L->m; ++j) {
            const double *A = &L->A[3 * j];
            const double S = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
            if (S == 0) continue;
            const int64_t ab[2] = {L->a[j], L->b[j]};
            for (int side = 0; side < 2; ++side) {
                /* cell i = ab[side] with outward normal +-A/S, neighbour p = ab[1 - side] */
                const int64_t i = ab[side], nb = ab[1 - side];
                const double sg = side == 0 ? 1.0 : -1.0;
                const double n[3] = {sg * A[0] / S, sg * A[1] / S, sg * A[2] / S};
                double Up[5], Un[5], F1[5], F0[5];
                for (int k = 0; k < 5; ++k) {
                    Up[k] = W[k * N + nb];
                    Un[k] = Up[k] + prev[k * N + nb];
                }
                euler_flux_n(Un, n, p->gamma, F1);
                euler_flux_n(Up, n, p->gamma, F0);
                for (int k = 0; k < 5; ++k)
                    acc[k * N + i] -= 0.5 * ((F1[k] - F0[k]) - lam[j] * prev[k * N + nb]) * S;
            }
        }
        for (int64_t c = 0; c < N; ++c)
            for (int k = 0; k < 5; ++k) dU[k * N + c] = acc[k * N + c] / diag[c];
    }
    free(dt);
    free(diag);
    free(lam);
    free(prev);
    free(acc);
}

/* one coarse sweep: W += dt/V (R + F) (forward Euler) or W += dU of the implicit smoother */
static void coarse_sweep(const om_hier *h, int l, const om_params *p, const double *F, double *W)
{
    const int64_t N = h->lev[l].n;
    double *R = malloc(sizeof(double) * 5 * N), *dt = malloc(sizeof(double) * N);
    om_kfvs_residual(h, l, p, W, R);
    if (p->coarse_smoother == 1) {
        double *dU = malloc(sizeof(double) * 5 * N);
        for (int64_t i = 0; i < 5 * N; ++i) R[i] += F[i];
        om_coarse_implicit(h, l, p, W, R, dU);
        for (int64_t i = 0; i < 5 * N; ++i) W[i] += dU[i];
        free(dU);
    } else {
        om_coarse_dt(h, l, p, W, dt);
        for (int64_t c = 0; c < N; ++c)
            for (int k = 0; k < 5; ++k) W[k * N + c] += dt[c] / h->lev[l].V[c] * (R[k * N + c] + F[k * N + c]);
    }
    free(R);
    free(dt);
}

typedef struct {
    int nu_pre[8], nu_post[8];
} om_cycle;

static void coarse_visit(const om_hier *h, int l, const om_params *p, const om_cycle *cy, const double *W0,
                         const double *Rs, double *W);

/*
 * FAS cycle on level l >= 1 with forcing F, state W in place: pre-sweeps, then (below the
 * coarsest level) the next level's forcing from the restricted state and residual, gamma visits
 * of the next level that continue from its state with that forcing, the correction, post-sweeps.
 */
static void fas_level(const om_hier *h, int l, const om_params *p, const om_cycle *cy, const double *F, double *W)
{
    const int64_t N = h->lev[l].n;
    for (int s = 0; s < cy->nu_pre[l]; ++s) coarse_sweep(h, l, p, F, W);
    if (l + 1 < h->nlev) {
        const int64_t Nc = h->lev[l + 1].n;
        double *R = malloc(sizeof(double) * 5 * N);
        om_kfvs_residual(h, l, p, W, R);
        for (int64_t i = 0; i < 5 * N; ++i) R[i] += F[i];
        double *Wc0 = malloc(sizeof(double) * 5 * Nc), *Rc = malloc(sizeof(double) * 5 * Nc),
               *Wc = malloc(sizeof(double) * 5 * Nc);
        om_restrict(h, l + 1, W, R, Wc0, Rc);
        coarse_visit(h, l + 1, p, cy, Wc0, Rc, Wc);
        for (int64_t i = 0; i < 5 * Nc; ++i) Wc[i] -= Wc0[i];
        om_prolong(h, l + 1, Wc, W);
        free(R);
        free(Wc0);
        free(Rc);
        free(Wc);
    }
    for (int s = 0; s < cy->nu_post[l]; ++s) coarse_sweep(h, l, p, F, W);
}

/* visit of level l from its parent: forcing F = Res* - Res_2h(W0), W = W0, gamma FAS cycles */
static void coarse_visit(const om_hier *h, int l, const om_params *p, const om_cycle *cy, const double *W0,
                         const double *Rs, double *W)
{
    const int64_t N = h->lev[l].n;
    double *R0 = malloc(sizeof(double) * 5 * N), *F = malloc(sizeof(double) * 5 * N);
    om_kfvs_residual(h, l, p, W0, R0);
    for (int64_t i = 0; i < 5 * N; ++i) F[i] = Rs[i] - R0[i];
    memcpy(W, W0, sizeof(double) * 5 * N);
    const int gamma = p->cycle_gamma > 1 ? p->cycle_gamma : 1;
    for (int k = 0; k < gamma; ++k) fas_level(h, l, p, cy, F, W);
    free(R0);
    free(F);
}

/*
 * One V-cycle on the fine state (W, G, alpha), in place.  resnorm receives the
 * RMS density residual per volume of the smoothing step.
 */
int om_vcycle(const om_hier *h, const om_params *p, const int *nu_pre, const int *nu_post, double *W, double *G,
              double *alpha, double *resnorm, int64_t *bad_cell)
{
    const om_mesh *m = h->mesh;
    const int64_t N = m->n_cells;
    om_cycle cy;
    for (int l = 0; l < 8; ++l) {
        cy.nu_pre[l] = nu_pre ? nu_pre[l] : 1;
        cy.nu_post[l] = nu_post ? nu_post[l] : 0;
    }
    double *R = malloc(sizeof(double) * 5 * N), *Gn = malloc(sizeof(double) * 15 * N);
    double *an = malloc(sizeof(double) * N), *dt = malloc(sizeof(double) * N);
    int e = 0;
    for (int s = 0; s < cy.nu_pre[0] && !e; ++s) {
        e = om_residual(m, p, W, G, alpha, R, Gn, an, dt, NULL, 0, bad_cell);
        if (e) break;
        if (s == 0 && resnorm) *resnorm = om_residual_norm(m, R);
        for (int64_t c = 0; c < N; ++c)
            for (int k = 0; k < 5; ++k) W[k * N + c] += dt[c] / m->vol[c] * R[k * N + c];
        memcpy(G, Gn, sizeof(double) * 15 * N);
        memcpy(alpha, an, sizeof(double) * N);
    }
    if (!e && h->nlev > 1) {
        e = om_residual(m, p, W, G, alpha, R, NULL, NULL, NULL, NULL, 0, bad_cell);
        if (!e) {
            const int64_t Nc = h->lev[1].n;
            double *Wc0 = malloc(sizeof(double) * 5 * Nc), *Rc = malloc(sizeof(double) * 5 * Nc),
                   *Wc = malloc(sizeof(double) * 5 * Nc);
            om_restrict(h, 1, W, R, Wc0, Rc);
            coarse_visit(h, 1, p, &cy, Wc0, Rc, Wc);
            for (int64_t i = 0; i < 5 * Nc; ++i) Wc[i] -= Wc0[i];
            om_prolong(h, 1, Wc, W);
            free(Wc0);
            free(Rc);
            free(Wc);
        }
    }
    for (int s = 0; s < cy.nu_post[0] && !e; ++s) {
        e = om_residual(m, p, W, G, alpha, R, Gn, an, dt, NULL, 0, bad_cell);
        if (e) break;
        for (int64_t c = 0; c < N; ++c)
            for (int k = 0; k < 5; ++k) W[k * N + c] += dt[c] / m->vol[c] * R[k * N + c];
        memcpy(G, Gn, sizeof(double) * 15 * N);
        memcpy(alpha, an, sizeof(double) * N);
    }
    free(R);
    free(Gn);
    free(an);
    free(dt);
    return e;
}
