/*
 * CGKS CPU oracle -- Maxwellian moments, micro-slopes and the BGK interface
 * solution at one Gauss point.  TEST INFRASTRUCTURE ONLY (see om_internal.h).
 *
 * Every moment is taken the slow, generic way: the integrand is expanded into
 * monomials u^i v^j w^k xi^(2l) by a small polynomial algebra, and each
 * monomial moment is the product of one-dimensional Maxwellian moments.  Every
 * small linear system is solved by LU with partial pivoting.
 *
 * Paper passages followed:
 *  - BGK model, Maxwellian g, psi = (1, u, (u^2+xi^2)/2), K = (5-3 gamma)/(gamma-1):
 *    Sec. 2.1, Eq. (bgk).
 *  - micro-slopes a_{x_i} and A from <a> = dW/dx_i and <A + a.u> = 0: Sec. 2.3, Eqs. (co), (co-moment).
 *  - interface equilibrium W^c from the two half-space moments: Eq. (compatibility2).
 *  - collision times tau = mu/p, tau_n with the pressure jump (C = 1, eps = 0.01).
 *  - time-dependent distribution at the interface: Eq. (2nd-flux).
 *  - interface conservative value W(t) = int psi f: Sec. 2.4.
 * Readings where the paper is silent (also listed in the design notes):
 *  - slopes of g^c are the kinetic-weighted half-space moments of the two side slopes;
 *  - inviscid flow: tau = 0 outside the exponentials, tau_n inside;
 *  - tau_n uses the Gauss-point pressures of the two sides;
 *  - the flux of a single step is the time average of F(t) over [0, dt];
 *  - Prandtl-number fix: the energy flux gains (1/Pr - 1) q with q the
 *    time-averaged heat flux of f relative to the velocity of g^c.
 * One-dimensional moment recursions: the standard Maxwellian moments,
 * <u^0> = 1, <u> = U, <u^{n+2}> = U <u^{n+1}> + (n+1)/(2 lambda) <u^n>;
 * half spaces start from erfc and exp(-lambda U^2).
 */
#include "om_internal.h"
#include <math.h>
#include <string.h>

#define NMAXU 12
#define MAXT 512

typedef struct {
    int n;
    double c[MAXT];
    unsigned char e[MAXT][4];
} poly;

static void p_zero(poly *p) { p->n = 0; }

static void p_term(poly *p, double c, int i, int j, int k, int l)
{
    for (int t = 0; t < p->n; ++t)
        if (p->e[t][0] == i && p->e[t][1] == j && p->e[t][2] == k && p->e[t][3] == l) {
            p->c[t] += c;
            return;
        }
    p->c[p->n] = c;
    p->e[p->n][0] = (unsigned char)i;
    p->e[p->n][1] = (unsigned char)j;
    p->e[p->n][2] = (unsigned char)k;
    p->e[p->n][3] = (unsigned char)l;
    p->n++;
}

static void p_mul(const poly *a, const poly *b, poly *out)
{
    p_zero(out);
    for (int s = 0; s < a->n; ++s)
        for (int t = 0; t < b->n; ++t)
            p_term(out, a->c[s] * b->c[t], a->e[s][0] + b->e[t][0], a->e[s][1] + b->e[t][1],
                   a->e[s][2] + b->e[t][2], a->e[s][3] + b->e[t][3]);
}

static void p_axpy(poly *y, double a, const poly *x)
{
    for (int t = 0; t < x->n; ++t) p_term(y, a * x->c[t], x->e[t][0], x->e[t][1], x->e[t][2], x->e[t][3]);
}

/* psi_alpha, alpha = 0..4 */
static void p_psi(int alpha, poly *p)
{
    p_zero(p);
    switch (alpha) {
    case 0: p_term(p, 1.0, 0, 0, 0, 0); break;
    case 1: p_term(p, 1.0, 1, 0, 0, 0); break;
    case 2: p_term(p, 1.0, 0, 1, 0, 0); break;
    case 3: p_term(p, 1.0, 0, 0, 1, 0); break;
    default:
        p_term(p, 0.5, 2, 0, 0, 0);
        p_term(p, 0.5, 0, 2, 0, 0);
        p_term(p, 0.5, 0, 0, 2, 0);
        p_term(p, 0.5, 0, 0, 0, 1);
    }
}

/* particle velocity component u_j as a polynomial */
static void p_vel(int j, poly *p)
{
    p_zero(p);
    p_term(p, 1.0, j == 0, j == 1, j == 2, 0);
}

/* s = sum_beta a_beta psi_beta */
static void p_slope(const double *a, poly *p)
{
    poly q;
    p_zero(p);
    for (int b = 0; b < 5; ++b) {
        p_psi(b, &q);
        p_axpy(p, a[b], &q);
    }
}

/* one-dimensional Maxwellian moments <u^n>, n = 0..nmax, of exp(-lam (u-U)^2) sqrt(lam/pi)
 * over all u (half = 0), u > 0 (half = +1) or u < 0 (half = -1). */
void om_moments_1d(double U, double lam, int half, int nmax, double *m)
{
    if (half == 0) {
        m[0] = 1.0;
        m[1] = U;
    } else {
        double s = (double)half;
        m[0] = 0.5 * erfc(-s * sqrt(lam) * U);
        m[1] = U * m[0] + s * 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
    }
    for (int n = 0; n + 2 <= nmax; ++n) m[n + 2] = U * m[n + 1] + (n + 1) / (2.0 * lam) * m[n];
}

/* <xi^(2l)> over K internal degrees of freedom */
double om_xi_moment(int l, double lam, double K)
{
    double r = 1.0;
    for (int i = 0; i < l; ++i) r *= (K + 2.0 * i) / (2.0 * lam);
    return r;
}

typedef struct {
    double mu[NMAXU + 1], mv[NMAXU + 1], mw[NMAXU + 1], mx[6];
} mtab;

static void mtab_build(mtab *t, const double *U, double lam, double K, int half)
{
    om_moments_1d(U[0], lam, half, NMAXU, t->mu);
    om_moments_1d(U[1], lam, 0, NMAXU, t->mv);
    om_moments_1d(U[2], lam, 0, NMAXU, t->mw);
    for (int l = 0; l < 6; ++l) t->mx[l] = om_xi_moment(l, lam, K);
}

static double p_moment(const poly *p, const mtab *t)
{
    double s = 0.0;
    for (int k = 0; k < p->n; ++k)
        s += p->c[k] * t->mu[p->e[k][0]] * t->mv[p->e[k][1]] * t->mw[p->e[k][2]] * t->mx[p->e[k][3]];
    return s;
}

/* W -> rho, U[3], lambda = rho / (2 p) */
void om_prim_from_cons(const double *W, double gamma, double *rho, double *U, double *lam)
{
    *rho = W[0];
    for (int d = 0; d < 3; ++d) U[d] = W[1 + d] / W[0];
    double p = (gamma - 1.0) * (W[4] - 0.5 * W[0] * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    *lam = W[0] / (2.0 * p);
}

int om_lu_solve(int n, double *A, double *b, int nrhs)
{
    int piv[32];
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
        if (A[p * n + k] == 0.0) return -1;
        piv[k] = p;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
            for (int r = 0; r < nrhs; ++r) {
                double t = b[r * n + k];
                b[r * n + k] = b[r * n + p];
                b[r * n + p] = t;
            }
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            A[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int r = 0; r < nrhs; ++r) b[r * n + i] -= f * b[r * n + k];
        }
    }
    for (int r = 0; r < nrhs; ++r)
        for (int i = n - 1; i >= 0; --i) {
            double s = b[r * n + i];
            for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[r * n + j];
            b[r * n + i] = s / A[i * n + i];
        }
    (void)piv;
    return 0;
}

/* moment matrix M_ab = <psi_a psi_b> of the normalised Maxwellian */
static void moment_matrix(const mtab *t, double *M)
{
    poly pa, pb, pab;
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            p_psi(a, &pa);
            p_psi(b, &pb);
            p_mul(&pa, &pb, &pab);
            M[a * 5 + b] = p_moment(&pab, t);
        }
}

/* rho M a = dW  ->  a (5 coefficients of a = sum a_b psi_b) */
int om_micro_slope(double rho, const double *U, double lam, double K, const double *dW, double *a)
{
    mtab t;
    mtab_build(&t, U, lam, K, 0);
    double M[25];
    moment_matrix(&t, M);
    for (int b = 0; b < 5; ++b) a[b] = dW[b] / rho;
    return om_lu_solve(5, M, a, 1);
}

/* <(A + sum_j u_j a_j) psi> = 0  ->  A */
int om_time_slope(const double *U, double lam, double K, const double a[3][5], double *A)
{
    mtab t;
    mtab_build(&t, U, lam, K, 0);
    double M[25];
    moment_matrix(&t, M);
    poly s, uj, ps, tmp, tmp2;
    for (int al = 0; al < 5; ++al) {
        double b = 0.0;
        p_psi(al, &ps);
        for (int j = 0; j < 3; ++j) {
            p_slope(a[j], &s);
            p_vel(j, &uj);
            p_mul(&uj, &s, &tmp);
            p_mul(&tmp, &ps, &tmp2);
            b -= p_moment(&tmp2, &t);
        }
        A[al] = b;
    }
    return om_lu_solve(5, M, A, 1);
}

/* sum_j u_j s_j as a polynomial */
static void p_transport(const double a[3][5], poly *out)
{
    poly s, uj, tmp;
    p_zero(out);
    for (int j = 0; j < 3; ++j) {
        p_slope(a[j], &s);
        p_vel(j, &uj);
        p_mul(&uj, &s, &tmp);
        p_axpy(out, 1.0, &tmp);
    }
}

/* acc[al] += rho * < weight * psi_al * extra > over table t */
static void acc_moments(double *acc, double rho, const poly *weight, const poly *extra, const mtab *t)
{
    poly ps, a1, a2;
    for (int al = 0; al < 5; ++al) {
        p_psi(al, &ps);
        p_mul(weight, &ps, &a1);
        p_mul(&a1, extra, &a2);
        acc[al] += rho * p_moment(&a2, t);
    }
}

static double acc_scalar(const poly *h, const poly *extra, double rho, const mtab *t)
{
    poly a;
    p_mul(h, extra, &a);
    return rho * p_moment(&a, t);
}

int om_gks_point(const double *Wl, const double *dWl, const double *Wr, const double *dWr, double dt,
                 const om_params *p, om_gks_out *out)
{
    const double g = p->gamma, K = (5.0 - 3.0 * g) / (g - 1.0);
    double rl, rr, Ul[3], Ur[3], ll, lr;
    om_prim_from_cons(Wl, g, &rl, Ul, &ll);
    om_prim_from_cons(Wr, g, &rr, Ur, &lr);
    if (!(rl > 0 && rr > 0 && ll > 0 && lr > 0)) return -1;
    double al[3][5], ar[3][5], Al[5], Ar[5];
    for (int j = 0; j < 3; ++j) {
        if (om_micro_slope(rl, Ul, ll, K, &dWl[5 * j], al[j])) return -2;
        if (om_micro_slope(rr, Ur, lr, K, &dWr[5 * j], ar[j])) return -2;
    }
    if (om_time_slope(Ul, ll, K, al, Al) || om_time_slope(Ur, lr, K, ar, Ar)) return -2;
    mtab tl, tr;
    mtab_build(&tl, Ul, ll, K, +1);
    mtab_build(&tr, Ur, lr, K, -1);
    poly one, u1, sl, sr, trl, trr, Apl, Apr;
    p_zero(&one);
    p_term(&one, 1.0, 0, 0, 0, 0);
    p_vel(0, &u1);
    /* interface equilibrium state and its slopes (kinetic-weighted) */
    double Wc[5] = {0, 0, 0, 0, 0}, dWc[3][5];
    acc_moments(Wc, rl, &one, &one, &tl);
    acc_moments(Wc, rr, &one, &one, &tr);
    for (int j = 0; j < 3; ++j) {
        for (int c = 0; c < 5; ++c) dWc[j][c] = 0;
        p_slope(al[j], &sl);
        p_slope(ar[j], &sr);
        acc_moments(dWc[j], rl, &one, &sl, &tl);
        acc_moments(dWc[j], rr, &one, &sr, &tr);
    }
    double rc, Uc[3], lc;
    om_prim_from_cons(Wc, g, &rc, Uc, &lc);
    if (!(rc > 0 && lc > 0)) return -1;
    double ac[3][5], Ac[5];
    for (int j = 0; j < 3; ++j)
        if (om_micro_slope(rc, Uc, lc, K, dWc[j], ac[j])) return -2;
    if (om_time_slope(Uc, lc, K, ac, Ac)) return -2;
    mtab tc;
    mtab_build(&tc, Uc, lc, K, 0);
    /* collision times */
    double pl = rl / (2.0 * ll), pr = rr / (2.0 * lr), pc = rc / (2.0 * lc);
    double jump = fabs((pl - pr) / (pl + pr));
    double tau = p->viscous ? p->mu / pc : 0.0;
    double taun = (p->viscous ? tau : p->eps_tau * dt) + p->c_tau * jump * dt;
    /* moment vectors: flux (weight u) and value (weight 1) */
    double Mc[3][5], Mk[3][5], Vc[3][5], Vk[3][5];
    memset(Mc, 0, sizeof(Mc));
    memset(Mk, 0, sizeof(Mk));
    memset(Vc, 0, sizeof(Vc));
    memset(Vk, 0, sizeof(Vk));
    poly trc, Apc;
    p_transport(ac, &trc);
    p_slope(Ac, &Apc);
    p_transport(al, &trl);
    p_transport(ar, &trr);
    p_slope(Al, &Apl);
    p_slope(Ar, &Apr);
    acc_moments(Mc[0], rc, &u1, &one, &tc);
    acc_moments(Mc[1], rc, &u1, &trc, &tc);
    acc_moments(Mc[2], rc, &u1, &Apc, &tc);
    acc_moments(Vc[0], rc, &one, &one, &tc);
    acc_moments(Vc[1], rc, &one, &trc, &tc);
    acc_moments(Vc[2], rc, &one, &Apc, &tc);
    acc_moments(Mk[0], rl, &u1, &one, &tl);
    acc_moments(Mk[0], rr, &u1, &one, &tr);
    acc_moments(Mk[1], rl, &u1, &trl, &tl);
    acc_moments(Mk[1], rr, &u1, &trr, &tr);
    acc_moments(Mk[2], rl, &u1, &Apl, &tl);
    acc_moments(Mk[2], rr, &u1, &Apr, &tr);
    acc_moments(Vk[0], rl, &one, &one, &tl);
    acc_moments(Vk[0], rr, &one, &one, &tr);
    acc_moments(Vk[1], rl, &one, &trl, &tl);
    acc_moments(Vk[1], rr, &one, &trr, &tr);
    acc_moments(Vk[2], rl, &one, &Apl, &tl);
    acc_moments(Vk[2], rr, &one, &Apr, &tr);
    /* heat flux relative to g^c velocity (Prandtl fix) */
    double H[6] = {0, 0, 0, 0, 0, 0};
    int prfix = p->viscous && p->prandtl != 1.0;
    if (prfix) {
        poly h, cu, cv, cw, c2, t1;
        p_zero(&cu);
        p_term(&cu, 1.0, 1, 0, 0, 0);
        p_term(&cu, -Uc[0], 0, 0, 0, 0);
        p_zero(&cv);
        p_term(&cv, 1.0, 0, 1, 0, 0);
        p_term(&cv, -Uc[1], 0, 0, 0, 0);
        p_zero(&cw);
        p_term(&cw, 1.0, 0, 0, 1, 0);
        p_term(&cw, -Uc[2], 0, 0, 0, 0);
        p_zero(&c2);
        p_mul(&cu, &cu, &t1);
        p_axpy(&c2, 1.0, &t1);
        p_mul(&cv, &cv, &t1);
        p_axpy(&c2, 1.0, &t1);
        p_mul(&cw, &cw, &t1);
        p_axpy(&c2, 1.0, &t1);
        p_term(&c2, 1.0, 0, 0, 0, 1);
        p_mul(&cu, &c2, &h);
        for (int t = 0; t < h.n; ++t) h.c[t] *= 0.5;
        H[0] = acc_scalar(&h, &one, rc, &tc);
        H[1] = acc_scalar(&h, &trc, rc, &tc);
        H[2] = acc_scalar(&h, &Apc, rc, &tc);
        H[3] = acc_scalar(&h, &one, rl, &tl) + acc_scalar(&h, &one, rr, &tr);
        H[4] = acc_scalar(&h, &trl, rl, &tl) + acc_scalar(&h, &trr, rr, &tr);
        H[5] = acc_scalar(&h, &Apl, rl, &tl) + acc_scalar(&h, &Apr, rr, &tr);
    }
    /* time-integrated coefficients over [0,T] */
    double Ts[2] = {dt, 0.5 * dt};
    double *Fo[2] = {out->Fint, out->Fhalf};
    for (int s = 0; s < 2; ++s) {
        double T = Ts[s];
        double E = exp(-T / taun), omE = -expm1(-T / taun);
        double Ie = taun * omE;
        double Ite = taun * taun * omE - taun * T * E;
        double I1 = T - taun * omE;
        double I2 = Ite + tau * Ie - tau * T;
        double I3 = 0.5 * T * T - tau * T + tau * Ie;
        double Ik1 = tau * Ie + Ite;
        double Ik2 = tau * Ie;
        for (int c = 0; c < 5; ++c)
            Fo[s][c] = I1 * Mc[0][c] + I2 * Mc[1][c] + I3 * Mc[2][c] + Ie * Mk[0][c] - Ik1 * Mk[1][c] - Ik2 * Mk[2][c];
        if (prfix) {
            double q = I1 * H[0] + I2 * H[1] + I3 * H[2] + Ie * H[3] - Ik1 * H[4] - Ik2 * H[5];
            Fo[s][4] += (1.0 / p->prandtl - 1.0) * q;
        }
    }
    for (int c = 0; c < 5; ++c) out->F[c] = out->Fint[c] / dt;
    /* interface values at t = dt and dt/2 */
    double *Wo[2] = {out->Wdt, out->Whalf};
    for (int s = 0; s < 2; ++s) {
        double t = Ts[s];
        double e = exp(-t / taun);
        double C1 = -expm1(-t / taun);
        double C2 = (t + tau) * e - tau;
        double C3 = t - tau + tau * e;
        for (int c = 0; c < 5; ++c)
            Wo[s][c] = C1 * Vc[0][c] + C2 * Vc[1][c] + C3 * Vc[2][c] + e * Vk[0][c] - (tau + t) * e * Vk[1][c] -
                       tau * e * Vk[2][c];
    }
    for (int c = 0; c < 5; ++c) out->Wc[c] = Wc[c];
    return 0;
}

/* First-order kinetic flux vector splitting: F = rho_l <u psi>_{u>0} + rho_r <u psi>_{u<0} (local frame). */
void om_kfvs_point(const double *Wl, const double *Wr, double gamma, double *F)
{
    const double K = (5.0 - 3.0 * gamma) / (gamma - 1.0);
    double rl, rr, Ul[3], Ur[3], ll, lr;
    om_prim_from_cons(Wl, gamma, &rl, Ul, &ll);
    om_prim_from_cons(Wr, gamma, &rr, Ur, &lr);
    mtab tl, tr;
    mtab_build(&tl, Ul, ll, K, +1);
    mtab_build(&tr, Ur, lr, K, -1);
    poly one, u1;
    p_zero(&one);
    p_term(&one, 1.0, 0, 0, 0, 0);
    p_vel(0, &u1);
    for (int c = 0; c < 5; ++c) F[c] = 0;
    acc_moments(F, rl, &u1, &one, &tl);
    acc_moments(F, rr, &u1, &one, &tr);
}

/* exposed for pins: moment of u^i v^j w^k xi^(2l) of the normalised Maxwellian */
double om_monomial_moment(const double *U, double lam, double K, int half, int i, int j, int k, int l)
{
    mtab t;
    mtab_build(&t, U, lam, K, half);
    poly p;
    p_zero(&p);
    p_term(&p, 1.0, i, j, k, l);
    return p_moment(&p, &t);
}
