/*
 * CGKS CPU oracle -- third-order compact HWENO reconstruction of one cell.
 * TEST INFRASTRUCTURE ONLY (see om_internal.h).
 *
 * Paper Sec. 3:
 *  - large stencil p^2 (10 coefficients) on the cell and its face neighbours:
 *    neighbour averages exact, neighbour gradient averages in the least-squares
 *    sense, solved as a constrained least-squares (KKT) system (Sec. 3.1);
 *  - Green-Gauss linear p^1 on the sub-stencil, scaled by the compression
 *    factor of the previous evolution (Secs. 3.2, 3.3);
 *  - two-polynomial multi-resolution WENO: P2 = p^2/g2 - g1 p^1/g2, P1 = p^1,
 *    smoothness indicators, normalisation by Q0^2 + beta_1 + 1e-40, global
 *    indicator, nonlinear weights with eps = 1e-5 (Sec. 3.4).
 * Readings (listed in the design notes):
 *  - the reconstruction acts on each conservative component separately;
 *  - basis functions of p^2 have zero mean on the target cell, so its average
 *    is exact by construction; gradient rows are scaled by |Omega_0|^(1/3);
 *  - Green-Gauss gradient = (1/|Omega_0|) sum_m (Q_m + Q_0)/2 S_m n_m, evaluated
 *    with (x - x_0); boundary faces use the boundary ghost of Q_0;
 *  - beta_1,LS is the unweighted linear least-squares fit of neighbour averages;
 *    beta is evaluated on p^1 and p^2; each distinct multi-index counted once;
 *  - the global indicator is |beta~_2 - beta~_1|;
 *  - only interior face neighbours enter p^2 and the LS fit; a cell with fewer
 *    than three of them uses p^1 alone.
 */
#include "om_internal.h"
#include <math.h>
#include <string.h>

/* value and gradient of r0 + r.dx + quadratic terms; order r0, x, y, z, xx, yy, zz, xy, yz, xz */
void om_eval_poly(const double *r, const double *dx, double *val, double *grad)
{
    double x = dx[0], y = dx[1], z = dx[2];
    *val = r[0] + r[1] * x + r[2] * y + r[3] * z + r[4] * x * x + r[5] * y * y + r[6] * z * z + r[7] * x * y +
           r[8] * y * z + r[9] * x * z;
    grad[0] = r[1] + 2.0 * r[4] * x + r[7] * y + r[9] * z;
    grad[1] = r[2] + 2.0 * r[5] * y + r[7] * x + r[8] * z;
    grad[2] = r[3] + 2.0 * r[6] * z + r[8] * y + r[9] * x;
}

int om_reconstruct_cell(const om_mesh *m, const om_params *p, const double *W, const double *G, const double *alpha,
                        int64_t c, double *coef)
{
    const int64_t N = m->n_cells;
    const double V0 = m->vol[c];
    const double *x0 = &m->cen[3 * c];
    const double *I0 = &m->mom2[6 * c];
    int nb = 0;
    int64_t nbid[OM_MAXNF];
    double dxn[OM_MAXNF][3];
    double gg[5][3];
    memset(gg, 0, sizeof(gg));
    double Q0[5];
    for (int k = 0; k < 5; ++k) Q0[k] = W[k * N + c];
    for (int64_t q = m->cf_ptr[c]; q < m->cf_ptr[c + 1]; ++q) {
        int64_t f = m->cf_face[q];
        int s = m->cf_sign[q];
        double A[3];
        for (int d = 0; d < 3; ++d) A[d] = s * m->avec[3 * f + d];
        double Qm[5];
        if (m->fr[f] >= 0) {
            int64_t o = s > 0 ? m->fr[f] : m->fl[f];
            for (int k = 0; k < 5; ++k) Qm[k] = W[k * N + o];
            for (int d = 0; d < 3; ++d)
                dxn[nb][d] = m->cen[3 * o + d] + s * m->shift[3 * f + d] - x0[d];
            nbid[nb++] = o;
        } else {
            double na = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
            double nn[3] = {A[0] / na, A[1] / na, A[2] / na};
            om_bc_ghost_state(&m->bc[m->ftag[f] & 63], nn, Q0, p->gamma, Qm);
        }
        for (int k = 0; k < 5; ++k)
            for (int d = 0; d < 3; ++d) gg[k][d] += 0.5 * (Qm[k] + Q0[k]) * A[d];
    }
    const double a_prev = alpha ? alpha[c] : 1.0;
    for (int k = 0; k < 5; ++k)
        for (int d = 0; d < 3; ++d) gg[k][d] /= V0;
    /* p1 monomial coefficients */
    double p1[5][10];
    memset(p1, 0, sizeof(p1));
    for (int k = 0; k < 5; ++k) {
        p1[k][0] = Q0[k];
        for (int d = 0; d < 3; ++d) p1[k][1 + d] = a_prev * gg[k][d];
    }
    if (nb < 3) {
        memcpy(coef, p1, sizeof(p1));
        return 0;
    }
    /* least-squares linear gradient */
    double gls[5][3];
    {
        double A[9] = {0}, b[15] = {0};
        for (int j = 0; j < nb; ++j) {
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) A[3 * a + bb] += dxn[j][a] * dxn[j][bb];
            for (int k = 0; k < 5; ++k)
                for (int a = 0; a < 3; ++a) b[3 * k + a] += dxn[j][a] * (W[k * N + nbid[j]] - Q0[k]);
        }
        if (om_lu_solve(3, A, b, 5)) return -3;
        for (int k = 0; k < 5; ++k)
            for (int a = 0; a < 3; ++a) gls[k][a] = b[3 * k + a];
    }
    /* constrained least squares for p2: unknowns a1..a9 */
    const double h0 = cbrt(V0);
    const int nk = 9 + nb;
    double K[15 * 15];
    double rhs[5 * 15];
    memset(K, 0, sizeof(K));
    memset(rhs, 0, sizeof(rhs));
    double phi0[9] = {0, 0, 0, I0[0] / V0, I0[1] / V0, I0[2] / V0, I0[3] / V0, I0[4] / V0, I0[5] / V0};
    for (int j = 0; j < nb; ++j) {
        int64_t o = nbid[j];
        const double *Im = &m->mom2[6 * o];
        double Vm = m->vol[o];
        double X = dxn[j][0], Y = dxn[j][1], Z = dxn[j][2];
        double phim[9] = {X, Y, Z, Im[0] / Vm + X * X, Im[1] / Vm + Y * Y, Im[2] / Vm + Z * Z,
                          Im[3] / Vm + X * Y, Im[4] / Vm + Y * Z, Im[5] / Vm + X * Z};
        double Brow[3][9] = {{1, 0, 0, 2 * X, 0, 0, Y, 0, Z}, {0, 1, 0, 0, 2 * Y, 0, X, Z, 0}, {0, 0, 1, 0, 0, 2 * Z, 0, Y, X}};
        /* equality row */
        for (int k = 0; k < 9; ++k) {
            double cjk = phim[k] - phi0[k];
            K[(9 + j) * nk + k] = cjk;
            K[k * nk + 9 + j] = cjk;
        }
        for (int q = 0; q < 5; ++q) rhs[q * nk + 9 + j] = W[q * N + o] - Q0[q];
        /* least-squares rows, scaled by h0 */
        for (int d = 0; d < 3; ++d) {
            for (int a = 0; a < 9; ++a)
                for (int b = 0; b < 9; ++b) K[a * nk + b] += 2.0 * (h0 * Brow[d][a]) * (h0 * Brow[d][b]);
            for (int q = 0; q < 5; ++q) {
                double dv = h0 * G[(3 * q + d) * N + o];
                for (int a = 0; a < 9; ++a) rhs[q * nk + a] += 2.0 * (h0 * Brow[d][a]) * dv;
            }
        }
    }
    if (om_lu_solve(nk, K, rhs, 5)) return -3;
    const double g2 = p->gamma_lin, g1 = 1.0 - p->gamma_lin;
    const double V13 = cbrt(V0), V23 = V13 * V13;
    for (int q = 0; q < 5; ++q) {
        const double *a = &rhs[q * nk];
        double p2[10];
        p2[0] = Q0[q];
        for (int k = 0; k < 9; ++k) {
            p2[1 + k] = a[k];
            p2[0] -= a[k] * phi0[k];
        }
        /* smoothness indicators */
        double b1gg = V23 * (p1[q][1] * p1[q][1] + p1[q][2] * p1[q][2] + p1[q][3] * p1[q][3]);
        double b1ls = V23 * (gls[q][0] * gls[q][0] + gls[q][1] * gls[q][1] + gls[q][2] * gls[q][2]);
        double beta1 = b1gg < b1ls ? b1gg : b1ls;
        double gx[3] = {2 * a[3], a[6], a[8]}, gy[3] = {a[6], 2 * a[4], a[7]}, gz[3] = {a[8], a[7], 2 * a[5]};
        double lin[3] = {a[0], a[1], a[2]};
        double *gs[3] = {gx, gy, gz};
        double first = 0;
        for (int d = 0; d < 3; ++d) {
            double *g = gs[d];
            /* int (lin + g.dx)^2 dV = lin^2 V + g^T I g */
            double gIg = g[0] * g[0] * I0[0] + g[1] * g[1] * I0[1] + g[2] * g[2] * I0[2] +
                         2.0 * (g[0] * g[1] * I0[3] + g[1] * g[2] * I0[4] + g[0] * g[2] * I0[5]);
            first += lin[d] * lin[d] * V0 + gIg;
        }
        double second = 4 * a[3] * a[3] + 4 * a[4] * a[4] + 4 * a[5] * a[5] + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
        double beta2 = first / V13 + second * V0 * V13;
        double den = Q0[q] * Q0[q] + beta1 + 1e-40;
        double bt1 = beta1 / den, bt2 = beta2 / den;
        double sig = fabs(bt2 - bt1);
        double w1 = g1 * (1.0 + (sig / (p->weno_eps + bt1)) * (sig / (p->weno_eps + bt1)));
        double w2 = g2 * (1.0 + (sig / (p->weno_eps + bt2)) * (sig / (p->weno_eps + bt2)));
        double ws = w1 + w2;
        w1 /= ws;
        w2 /= ws;
        for (int k = 0; k < 10; ++k) {
            double P2 = p2[k] / g2 - g1 / g2 * p1[q][k];
            coef[q * 10 + k] = w2 * P2 + w1 * p1[q][k];
        }
    }
    return 0;
}
