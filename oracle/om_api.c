/*
 * CGKS CPU oracle -- flat accessors for the Python test harness.
 * TEST INFRASTRUCTURE ONLY (see om_internal.h).
 */
#include "om_internal.h"
#include <string.h>

void om_mesh_sizes(const om_mesh *m, int64_t *out)
{
    out[0] = m->n_cells;
    out[1] = m->n_faces;
    out[2] = m->n_int;
    out[3] = m->n_nodes;
}

void om_mesh_cells(const om_mesh *m, double *vol, double *cen, double *mom2)
{
    if (vol) memcpy(vol, m->vol, sizeof(double) * m->n_cells);
    if (cen) memcpy(cen, m->cen, sizeof(double) * 3 * m->n_cells);
    if (mom2) memcpy(mom2, m->mom2, sizeof(double) * 6 * m->n_cells);
}

void om_mesh_faces(const om_mesh *m, int64_t *fl, int64_t *fr, int32_t *tag, double *area, double *avec,
                   double *fmom, double *shift, int32_t *ngp, double *gpx, double *gpw, double *gpn)
{
    int64_t F = m->n_faces;
    if (fl) memcpy(fl, m->fl, sizeof(int64_t) * F);
    if (fr) memcpy(fr, m->fr, sizeof(int64_t) * F);
    if (tag) memcpy(tag, m->ftag, sizeof(int32_t) * F);
    if (area) memcpy(area, m->area, sizeof(double) * F);
    if (avec) memcpy(avec, m->avec, sizeof(double) * 3 * F);
    if (fmom) memcpy(fmom, m->fmom, sizeof(double) * 3 * F);
    if (shift) memcpy(shift, m->shift, sizeof(double) * 3 * F);
    if (ngp)
        for (int64_t f = 0; f < F; ++f) ngp[f] = m->ngp[f];
    if (gpx) memcpy(gpx, m->gpx, sizeof(double) * 3 * OM_MAXGP * F);
    if (gpw) memcpy(gpw, m->gpw, sizeof(double) * OM_MAXGP * F);
    if (gpn) memcpy(gpn, m->gpn, sizeof(double) * 3 * OM_MAXGP * F);
}

int om_mesh_set_bc(om_mesh *m, int32_t tag, int kind, const double *prim)
{
    if (tag < 0 || tag >= 64) return -1;
    m->bc[tag].kind = kind;
    for (int k = 0; k < 5; ++k) m->bc[tag].prim[k] = prim ? prim[k] : 0.0;
    return 0;
}

/* single Gauss point in the local frame, for pins */
int om_gks_point_flat(const double *Wl, const double *dWl, const double *Wr, const double *dWr, double dt,
                      const om_params *p, double *out30)
{
    om_gks_out o;
    int e = om_gks_point(Wl, dWl, Wr, dWr, dt, p, &o);
    if (e) return e;
    memcpy(out30, o.F, 5 * sizeof(double));
    memcpy(out30 + 5, o.Fint, 5 * sizeof(double));
    memcpy(out30 + 10, o.Fhalf, 5 * sizeof(double));
    memcpy(out30 + 15, o.Wdt, 5 * sizeof(double));
    memcpy(out30 + 20, o.Whalf, 5 * sizeof(double));
    memcpy(out30 + 25, o.Wc, 5 * sizeof(double));
    return 0;
}

int om_slopes_flat(double rho, const double *U, double lam, double K, const double *dW /*3x5*/, double *a /*3x5*/,
                   double *A)
{
    double aa[3][5];
    for (int j = 0; j < 3; ++j) {
        if (om_micro_slope(rho, U, lam, K, &dW[5 * j], aa[j])) return -1;
        memcpy(&a[5 * j], aa[j], 5 * sizeof(double));
    }
    return om_time_slope(U, lam, K, aa, A);
}

void om_bc_ghost_flat(int kind, const double *prim, const double *n, const double *Wi, const double *Gi,
                      double gamma, double *Wg, double *Gg)
{
    om_bc bc;
    bc.kind = kind;
    for (int k = 0; k < 5; ++k) bc.prim[k] = prim ? prim[k] : 0.0;
    om_bc_ghost_state(&bc, n, Wi, gamma, Wg);
    if (Gi && Gg) om_bc_ghost_grad(&bc, n, Gi, Gg);
}
