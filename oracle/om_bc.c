/*
 * CGKS CPU oracle -- boundary ghost states.  TEST INFRASTRUCTURE ONLY.
 *
 * The paper names slip walls, adiabatic no-slip walls and Riemann-invariant
 * far fields (Sec. 5) without formulas.  Readings used here:
 *  - slip wall: mirror image of the interior field across the face plane
 *    (normal momentum reversed); gradients mirrored the same way;
 *  - adiabatic no-slip wall: same density and energy, momentum reversed;
 *    density/energy gradients mirrored, momentum field x -> -m(Rx);
 *  - far field: one-dimensional Riemann invariants along the outward normal,
 *    entropy and tangential velocity from the upwind side; zero gradients.
 */
#include "om_internal.h"
#include <math.h>

static void reflect_matrix(const double *n, double R[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = (i == j ? 1.0 : 0.0) - 2.0 * n[i] * n[j];
}

void om_bc_ghost_state(const om_bc *bc, const double *n, const double *Wi, double gamma, double *Wg)
{
    if (bc->kind == OM_BC_SLIP) {
        double mn = Wi[1] * n[0] + Wi[2] * n[1] + Wi[3] * n[2];
        Wg[0] = Wi[0];
        for (int d = 0; d < 3; ++d) Wg[1 + d] = Wi[1 + d] - 2.0 * mn * n[d];
        Wg[4] = Wi[4];
        return;
    }
    if (bc->kind == OM_BC_NOSLIP) {
        Wg[0] = Wi[0];
        for (int d = 0; d < 3; ++d) Wg[1 + d] = -Wi[1 + d];
        Wg[4] = Wi[4];
        return;
    }
    /* far field */
    double ri = Wi[0], ui[3], q2 = 0;
    for (int d = 0; d < 3; ++d) {
        ui[d] = Wi[1 + d] / ri;
        q2 += ui[d] * ui[d];
    }
    double pi = (gamma - 1.0) * (Wi[4] - 0.5 * ri * q2);
    double ci = sqrt(gamma * pi / ri);
    const double *pf = bc->prim;
    double rf = pf[0], uf[3] = {pf[1], pf[2], pf[3]}, pff = pf[4];
    double cf = sqrt(gamma * pff / rf);
    double uni = ui[0] * n[0] + ui[1] * n[1] + ui[2] * n[2];
    double unf = uf[0] * n[0] + uf[1] * n[1] + uf[2] * n[2];
    double rb, ub[3], pb;
    if (fabs(uni) >= ci) {
        if (uni >= 0) {
            rb = ri;
            pb = pi;
            for (int d = 0; d < 3; ++d) ub[d] = ui[d];
        } else {
            rb = rf;
            pb = pff;
            for (int d = 0; d < 3; ++d) ub[d] = uf[d];
        }
    } else {
        double Rp = uni + 2.0 * ci / (gamma - 1.0);
        double Rm = unf - 2.0 * cf / (gamma - 1.0);
        double unb = 0.5 * (Rp + Rm);
        double cb = 0.25 * (gamma - 1.0) * (Rp - Rm);
        double s, ut[3];
        if (unb >= 0) {
            s = pi / pow(ri, gamma);
            for (int d = 0; d < 3; ++d) ut[d] = ui[d] - uni * n[d];
        } else {
            s = pff / pow(rf, gamma);
            for (int d = 0; d < 3; ++d) ut[d] = uf[d] - unf * n[d];
        }
        rb = pow(cb * cb / (gamma * s), 1.0 / (gamma - 1.0));
        pb = rb * cb * cb / gamma;
        for (int d = 0; d < 3; ++d) ub[d] = ut[d] + unb * n[d];
    }
    Wg[0] = rb;
    double qb = 0;
    for (int d = 0; d < 3; ++d) {
        Wg[1 + d] = rb * ub[d];
        qb += ub[d] * ub[d];
    }
    Wg[4] = pb / (gamma - 1.0) + 0.5 * rb * qb;
}

void om_bc_ghost_grad(const om_bc *bc, const double *n, const double *Gi, double *Gg)
{
    if (bc->kind == OM_BC_FARFIELD) {
        for (int i = 0; i < 15; ++i) Gg[i] = 0.0;
        return;
    }
    double R[3][3];
    reflect_matrix(n, R);
    /* scalar components: grad_g = R grad */
    const int sc[2] = {0, 4};
    for (int s = 0; s < 2; ++s) {
        int c = sc[s];
        for (int d = 0; d < 3; ++d) {
            double v = 0;
            for (int e = 0; e < 3; ++e) v += R[d][e] * Gi[3 * c + e];
            Gg[3 * c + d] = v;
        }
    }
    /* momentum: M_ij = d m_i / d x_j */
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = Gi[3 * (1 + i) + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0;
            if (bc->kind == OM_BC_SLIP) {
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) v += R[i][k] * M[k][l] * R[l][j];
            } else {
                for (int l = 0; l < 3; ++l) v -= M[i][l] * R[l][j];
            }
            Gg[3 * (1 + i) + j] = v;
        }
}
