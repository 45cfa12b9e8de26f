/*
 * CGKS CPU oracle -- mesh connectivity and geometry.
 * TEST INFRASTRUCTURE ONLY (see om_internal.h).
 *
 * Finite-volume framework on hybrid meshes (paper Sec. 2.2): cells are tets,
 * pyramids, prisms and hexahedra with linear iso-parametric faces; a triangle
 * carries 3 Gauss points and a quadrilateral 4.  Reading used here: triangles
 * use the interior degree-2 rule at barycentric (2/3,1/6,1/6) with weights
 * 1/3; quadrilaterals use 2x2 Gauss on the bilinear map.  Cell volume,
 * centroid and second moments come from a 3x3x3 Gauss rule on the trilinear
 * map of each element, written as a (possibly collapsed) hexahedron.
 */
#include "om_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

static const int FACE_N[9] = {0, 0, 0, 0, 4, 5, 5, 0, 6};
/* local faces, VTK node order; -1 pads triangles */
static const int TET_F[4][4] = {{0, 1, 3, -1}, {1, 2, 3, -1}, {2, 0, 3, -1}, {0, 2, 1, -1}};
static const int PYR_F[5][4] = {{0, 1, 2, 3}, {0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}};
static const int PRI_F[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
static const int HEX_F[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
/* element as collapsed hexahedron */
static const int TET_H[8] = {0, 1, 2, 2, 3, 3, 3, 3};
static const int PYR_H[8] = {0, 1, 2, 3, 4, 4, 4, 4};
static const int PRI_H[8] = {0, 1, 2, 2, 3, 4, 5, 5};
static const int HEX_H[8] = {0, 1, 2, 3, 4, 5, 6, 7};

static const int *local_face(int t, int f)
{
    switch (t) {
    case OM_TET: return TET_F[f];
    case OM_PYR: return PYR_F[f];
    case OM_PRISM: return PRI_F[f];
    default: return HEX_F[f];
    }
}

static const int *hex_map(int t)
{
    switch (t) {
    case OM_TET: return TET_H;
    case OM_PYR: return PYR_H;
    case OM_PRISM: return PRI_H;
    default: return HEX_H;
    }
}

static void cross(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Volume, centroid and central second moments by 3x3x3 Gauss on the trilinear map. */
static void cell_moments(const double *X /*8x3*/, double *vol, double *cen, double *m2)
{
    const double g[3] = {0.5 - 0.5 * sqrt(0.6), 0.5, 0.5 + 0.5 * sqrt(0.6)};
    const double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double qx[27][3], qw[27];
    int q = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c, ++q) {
                double s = g[a], t = g[b], r = g[c];
                double N[8] = {(1 - s) * (1 - t) * (1 - r), s * (1 - t) * (1 - r), s * t * (1 - r), (1 - s) * t * (1 - r),
                               (1 - s) * (1 - t) * r, s * (1 - t) * r, s * t * r, (1 - s) * t * r};
                double dNs[8] = {-(1 - t) * (1 - r), (1 - t) * (1 - r), t * (1 - r), -t * (1 - r),
                                 -(1 - t) * r, (1 - t) * r, t * r, -t * r};
                double dNt[8] = {-(1 - s) * (1 - r), -s * (1 - r), s * (1 - r), (1 - s) * (1 - r),
                                 -(1 - s) * r, -s * r, s * r, (1 - s) * r};
                double dNr[8] = {-(1 - s) * (1 - t), -s * (1 - t), -s * t, -(1 - s) * t,
                                 (1 - s) * (1 - t), s * (1 - t), s * t, (1 - s) * t};
                double x[3] = {0, 0, 0}, js[3] = {0, 0, 0}, jt[3] = {0, 0, 0}, jr[3] = {0, 0, 0};
                for (int i = 0; i < 8; ++i)
                    for (int d = 0; d < 3; ++d) {
                        x[d] += N[i] * X[3 * i + d];
                        js[d] += dNs[i] * X[3 * i + d];
                        jt[d] += dNt[i] * X[3 * i + d];
                        jr[d] += dNr[i] * X[3 * i + d];
                    }
                double c2[3];
                cross(jt, jr, c2);
                double det = dot3(js, c2);
                qx[q][0] = x[0];
                qx[q][1] = x[1];
                qx[q][2] = x[2];
                qw[q] = w[a] * w[b] * w[c] * det;
            }
    double V = 0, P[3] = {0, 0, 0};
    for (q = 0; q < 27; ++q) {
        V += qw[q];
        for (int d = 0; d < 3; ++d) P[d] += qw[q] * qx[q][d];
    }
    for (int d = 0; d < 3; ++d) cen[d] = P[d] / V;
    double M[6] = {0, 0, 0, 0, 0, 0};
    for (q = 0; q < 27; ++q) {
        double dx = qx[q][0] - cen[0], dy = qx[q][1] - cen[1], dz = qx[q][2] - cen[2];
        M[0] += qw[q] * dx * dx;
        M[1] += qw[q] * dy * dy;
        M[2] += qw[q] * dz * dz;
        M[3] += qw[q] * dx * dy;
        M[4] += qw[q] * dy * dz;
        M[5] += qw[q] * dx * dz;
    }
    double sgn = V < 0 ? -1.0 : 1.0;
    *vol = sgn * V;
    for (int i = 0; i < 6; ++i) m2[i] = sgn * M[i];
}

/* Gauss points of one face given its node coordinates in outward cyclic order. */
static void face_points(const double *P, int nn, int *ngp, double *gx, double *gw, double *gn,
                        double *S, double *avec, double *fmom)
{
    if (nn == 3) {
        double e1[3], e2[3], J[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = P[3 + d] - P[d];
            e2[d] = P[6 + d] - P[d];
        }
        cross(e1, e2, J);
        double nj = sqrt(dot3(J, J));
        const double b[3][3] = {{2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
        *ngp = 3;
        *S = 0.5 * nj;
        for (int d = 0; d < 3; ++d) {
            avec[d] = 0.5 * J[d];
            fmom[d] = 0;
        }
        for (int k = 0; k < 3; ++k) {
            for (int d = 0; d < 3; ++d) {
                gx[3 * k + d] = b[k][0] * P[d] + b[k][1] * P[3 + d] + b[k][2] * P[6 + d];
                gn[3 * k + d] = J[d] / nj;
                fmom[d] += (*S) * gx[3 * k + d] / 3.0;
            }
            gw[k] = 1.0 / 3.0;
        }
        gw[3] = 0;
        return;
    }
    const double g0 = 0.5 - 0.5 / sqrt(3.0), g1 = 0.5 + 0.5 / sqrt(3.0);
    const double st[4][2] = {{g0, g0}, {g1, g0}, {g1, g1}, {g0, g1}};
    double aj[4];
    *ngp = 4;
    *S = 0;
    for (int d = 0; d < 3; ++d) avec[d] = fmom[d] = 0;
    for (int k = 0; k < 4; ++k) {
        double s = st[k][0], t = st[k][1];
        double xs[3], xt[3], J[3];
        for (int d = 0; d < 3; ++d) {
            gx[3 * k + d] = (1 - s) * (1 - t) * P[d] + s * (1 - t) * P[3 + d] + s * t * P[6 + d] + (1 - s) * t * P[9 + d];
            xs[d] = (1 - t) * (P[3 + d] - P[d]) + t * (P[6 + d] - P[9 + d]);
            xt[d] = (1 - s) * (P[9 + d] - P[d]) + s * (P[6 + d] - P[3 + d]);
        }
        cross(xs, xt, J);
        aj[k] = sqrt(dot3(J, J));
        for (int d = 0; d < 3; ++d) {
            gn[3 * k + d] = J[d] / aj[k];
            avec[d] += 0.25 * J[d];
            fmom[d] += 0.25 * aj[k] * gx[3 * k + d];
        }
        *S += 0.25 * aj[k];
    }
    for (int k = 0; k < 4; ++k) gw[k] = 0.25 * aj[k] / (*S);
}

typedef struct {
    int64_t key[4];
    int64_t cell;
    int64_t nodes[4];
    int nn;
    int32_t btag; /* >0 for a boundary-face record */
} fside;

static int cmp_side(const void *a, const void *b)
{
    const fside *x = (const fside *)a, *y = (const fside *)b;
    for (int i = 0; i < 4; ++i) {
        if (x->key[i] < y->key[i]) return -1;
        if (x->key[i] > y->key[i]) return 1;
    }
    if (x->btag != y->btag) return x->btag < y->btag ? -1 : 1;
    if (x->cell < y->cell) return -1;
    if (x->cell > y->cell) return 1;
    return 0;
}

static void sort_key(int64_t *k, int n)
{
    for (int i = 0; i < 4; ++i)
        if (i >= n) k[i] = -1;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (k[j] < k[i]) {
                int64_t t = k[i];
                k[i] = k[j];
                k[j] = t;
            }
    /* put -1 pads last by shifting: keys of triangles are (a,b,c,-1) */
}

typedef struct {
    int64_t l, r;
    int64_t ln[4], rn[4];
    int nn;
    int32_t tag;
} frec;

static int cmp_frec(const void *a, const void *b)
{
    const frec *x = (const frec *)a, *y = (const frec *)b;
    int bx = x->r < 0, by = y->r < 0;
    if (bx != by) return bx - by;
    if (x->l != y->l) return x->l < y->l ? -1 : 1;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    for (int i = 0; i < 4; ++i)
        if (x->ln[i] != y->ln[i]) return x->ln[i] < y->ln[i] ? -1 : 1;
    return 0;
}

void om_mesh_free(om_mesh *m)
{
    if (!m) return;
    free(m->xyz);
    free(m->vol);
    free(m->cen);
    free(m->mom2);
    free(m->nface);
    free(m->fl);
    free(m->fr);
    free(m->ftag);
    free(m->shift);
    free(m->ngp);
    free(m->gpx);
    free(m->gpw);
    free(m->gpn);
    free(m->area);
    free(m->avec);
    free(m->fmom);
    free(m->cf_ptr);
    free(m->cf_face);
    free(m->cf_sign);
    free(m);
}

om_mesh *om_mesh_build(int64_t n_nodes, const double *xyz, int64_t n_cells, const uint8_t *ctype,
                       const int64_t *cptr, const int64_t *cnode, int64_t n_bf, const int64_t *bptr,
                       const int64_t *bnode, const int32_t *btag, const int64_t *canon, char *err)
{
    om_mesh *m = (om_mesh *)calloc(1, sizeof(om_mesh));
    m->n_nodes = n_nodes;
    m->n_cells = n_cells;
    m->xyz = (double *)malloc(sizeof(double) * 3 * n_nodes);
    memcpy(m->xyz, xyz, sizeof(double) * 3 * n_nodes);
    m->vol = (double *)malloc(sizeof(double) * n_cells);
    m->cen = (double *)malloc(sizeof(double) * 3 * n_cells);
    m->mom2 = (double *)malloc(sizeof(double) * 6 * n_cells);
    m->nface = (int *)malloc(sizeof(int) * n_cells);
    int64_t nside = 0;
    for (int64_t c = 0; c < n_cells; ++c) {
        int t = ctype[c];
        if ((t != 4 && t != 5 && t != 6 && t != 8) || cptr[c + 1] - cptr[c] != t) {
            snprintf(err, 256, "cell %lld: bad type %d", (long long)c, t);
            om_mesh_free(m);
            return NULL;
        }
        double X[24];
        const int *hm = hex_map(t);
        for (int i = 0; i < 8; ++i)
            for (int d = 0; d < 3; ++d) X[3 * i + d] = xyz[3 * cnode[cptr[c] + hm[i]] + d];
        cell_moments(X, &m->vol[c], &m->cen[3 * c], &m->mom2[6 * c]);
        if (!(m->vol[c] > 0)) {
            snprintf(err, 256, "cell %lld: non-positive volume", (long long)c);
            om_mesh_free(m);
            return NULL;
        }
        m->nface[c] = FACE_N[t];
        nside += FACE_N[t];
    }
    fside *S = (fside *)malloc(sizeof(fside) * (nside + n_bf));
    int64_t q = 0;
    for (int64_t c = 0; c < n_cells; ++c) {
        int t = ctype[c];
        for (int f = 0; f < FACE_N[t]; ++f, ++q) {
            const int *lf = local_face(t, f);
            int nn = lf[3] < 0 ? 3 : 4;
            for (int i = 0; i < 4; ++i) {
                S[q].nodes[i] = i < nn ? cnode[cptr[c] + lf[i]] : -1;
                S[q].key[i] = i < nn ? (canon ? canon[S[q].nodes[i]] : S[q].nodes[i]) : INT64_MAX;
            }
            sort_key(S[q].key, 4);
            S[q].cell = c;
            S[q].nn = nn;
            S[q].btag = 0;
        }
    }
    for (int64_t b = 0; b < n_bf; ++b, ++q) {
        int nn = (int)(bptr[b + 1] - bptr[b]);
        for (int i = 0; i < 4; ++i) {
            S[q].nodes[i] = i < nn ? bnode[bptr[b] + i] : -1;
            S[q].key[i] = i < nn ? (canon ? canon[S[q].nodes[i]] : S[q].nodes[i]) : INT64_MAX;
        }
        sort_key(S[q].key, 4);
        S[q].cell = -1;
        S[q].nn = nn;
        S[q].btag = btag[b] > 0 ? btag[b] : 1;
    }
    qsort(S, q, sizeof(fside), cmp_side);
    frec *F = (frec *)malloc(sizeof(frec) * q);
    int64_t nf = 0;
    for (int64_t i = 0; i < q;) {
        int64_t j = i;
        while (j < q && memcmp(S[j].key, S[i].key, sizeof(S[i].key)) == 0) ++j;
        int64_t cnt = j - i;
        /* sorted: boundary records (btag > 0) after cell sides (btag == 0) */
        if (cnt == 2 && S[i].btag == 0 && S[i + 1].btag == 0) {
            F[nf].l = S[i].cell;
            F[nf].r = S[i + 1].cell;
            memcpy(F[nf].ln, S[i].nodes, sizeof(F[nf].ln));
            memcpy(F[nf].rn, S[i + 1].nodes, sizeof(F[nf].rn));
            F[nf].nn = S[i].nn;
            F[nf].tag = 0;
            ++nf;
        } else if (cnt == 2 && S[i].btag == 0 && S[i + 1].btag > 0) {
            F[nf].l = S[i].cell;
            F[nf].r = -1;
            memcpy(F[nf].ln, S[i].nodes, sizeof(F[nf].ln));
            F[nf].nn = S[i].nn;
            F[nf].tag = S[i + 1].btag;
            ++nf;
        } else {
            snprintf(err, 256, "non-manifold or unmatched face (cell %lld, %lld records)", (long long)S[i].cell,
                     (long long)cnt);
            free(S);
            free(F);
            om_mesh_free(m);
            return NULL;
        }
        i = j;
    }
    free(S);
    qsort(F, nf, sizeof(frec), cmp_frec);
    m->n_faces = nf;
    m->n_int = 0;
    while (m->n_int < nf && F[m->n_int].r >= 0) ++m->n_int;
    m->fl = (int64_t *)malloc(sizeof(int64_t) * nf);
    m->fr = (int64_t *)malloc(sizeof(int64_t) * nf);
    m->ftag = (int32_t *)malloc(sizeof(int32_t) * nf);
    m->shift = (double *)calloc(3 * nf, sizeof(double));
    m->ngp = (int *)malloc(sizeof(int) * nf);
    m->gpx = (double *)calloc(3 * OM_MAXGP * nf, sizeof(double));
    m->gpw = (double *)calloc(OM_MAXGP * nf, sizeof(double));
    m->gpn = (double *)calloc(3 * OM_MAXGP * nf, sizeof(double));
    m->area = (double *)malloc(sizeof(double) * nf);
    m->avec = (double *)malloc(sizeof(double) * 3 * nf);
    m->fmom = (double *)malloc(sizeof(double) * 3 * nf);
    for (int64_t f = 0; f < nf; ++f) {
        m->fl[f] = F[f].l;
        m->fr[f] = F[f].r;
        m->ftag[f] = F[f].tag;
        int nn = F[f].nn;
        double P[12];
        for (int i = 0; i < nn; ++i)
            for (int d = 0; d < 3; ++d) P[3 * i + d] = xyz[3 * F[f].ln[i] + d];
        /* orient outward from L */
        double mid[3] = {0, 0, 0}, J[3];
        for (int i = 0; i < nn; ++i)
            for (int d = 0; d < 3; ++d) mid[d] += P[3 * i + d] / nn;
        {
            double e1[3], e2[3];
            for (int d = 0; d < 3; ++d) {
                e1[d] = P[3 * 2 + d] - P[d];
                e2[d] = P[3 * (nn - 1) + d] - P[3 + d];
            }
            if (nn == 3)
                for (int d = 0; d < 3; ++d) e2[d] = P[6 + d] - P[d], e1[d] = P[3 + d] - P[d];
            cross(e1, e2, J);
        }
        double rel[3] = {mid[0] - m->cen[3 * F[f].l], mid[1] - m->cen[3 * F[f].l + 1], mid[2] - m->cen[3 * F[f].l + 2]};
        if (dot3(J, rel) < 0) {
            /* reverse cyclic order keeping node 0 */
            double Q[12];
            memcpy(Q, P, sizeof(Q));
            for (int i = 1; i < nn; ++i)
                for (int d = 0; d < 3; ++d) P[3 * i + d] = Q[3 * (nn - i) + d];
        }
        face_points(P, nn, &m->ngp[f], &m->gpx[3 * OM_MAXGP * f], &m->gpw[OM_MAXGP * f], &m->gpn[3 * OM_MAXGP * f],
                    &m->area[f], &m->avec[3 * f], &m->fmom[3 * f]);
        if (F[f].r >= 0 && canon) {
            /* periodic translation from the node with the smallest canonical id */
            int64_t best = INT64_MAX;
            int il = 0;
            for (int i = 0; i < nn; ++i)
                if (canon[F[f].ln[i]] < best) best = canon[F[f].ln[i]], il = i;
            int ir = 0;
            for (int i = 0; i < nn; ++i)
                if (canon[F[f].rn[i]] == best) ir = i;
            for (int d = 0; d < 3; ++d) m->shift[3 * f + d] = xyz[3 * F[f].ln[il] + d] - xyz[3 * F[f].rn[ir] + d];
        }
    }
    free(F);
    /* cell -> face CSR */
    m->cf_ptr = (int64_t *)calloc(n_cells + 1, sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) {
        m->cf_ptr[m->fl[f] + 1]++;
        if (m->fr[f] >= 0) m->cf_ptr[m->fr[f] + 1]++;
    }
    for (int64_t c = 0; c < n_cells; ++c) m->cf_ptr[c + 1] += m->cf_ptr[c];
    m->cf_face = (int64_t *)malloc(sizeof(int64_t) * m->cf_ptr[n_cells]);
    m->cf_sign = (int *)malloc(sizeof(int) * m->cf_ptr[n_cells]);
    int64_t *fill = (int64_t *)calloc(n_cells, sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) {
        int64_t l = m->fl[f], r = m->fr[f];
        m->cf_face[m->cf_ptr[l] + fill[l]] = f;
        m->cf_sign[m->cf_ptr[l] + fill[l]++] = 1;
        if (r >= 0) {
            m->cf_face[m->cf_ptr[r] + fill[r]] = f;
            m->cf_sign[m->cf_ptr[r] + fill[r]++] = -1;
        }
    }
    free(fill);
    for (int64_t c = 0; c < n_cells; ++c)
        if (m->cf_ptr[c + 1] - m->cf_ptr[c] != m->nface[c]) {
            snprintf(err, 256, "cell %lld: %lld faces found, expected %d", (long long)c,
                     (long long)(m->cf_ptr[c + 1] - m->cf_ptr[c]), m->nface[c]);
            om_mesh_free(m);
            return NULL;
        }
    for (int i = 0; i < 64; ++i) m->bc[i].kind = OM_BC_SLIP;
    return m;
}

/* Orthonormal tangents for a unit normal: t1 from the axis least aligned with n. */
void om_frame(const double *n, double *t1, double *t2)
{
    double e[3] = {0, 0, 0};
    double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
    if (ax <= ay && ax <= az) e[0] = 1;
    else if (ay <= az) e[1] = 1;
    else e[2] = 1;
    double c[3];
    cross(n, e, c);
    double l = sqrt(dot3(c, c));
    for (int d = 0; d < 3; ++d) t1[d] = c[d] / l;
    cross(n, t1, t2);
}

void om_rotate_state(const double *W, const double *n, const double *t1, const double *t2, double *Wl)
{
    Wl[0] = W[0];
    Wl[1] = W[1] * n[0] + W[2] * n[1] + W[3] * n[2];
    Wl[2] = W[1] * t1[0] + W[2] * t1[1] + W[3] * t1[2];
    Wl[3] = W[1] * t2[0] + W[2] * t2[1] + W[3] * t2[2];
    Wl[4] = W[4];
}

void om_rotate_back(const double *Wl, const double *n, const double *t1, const double *t2, double *W)
{
    W[0] = Wl[0];
    for (int d = 0; d < 3; ++d) W[1 + d] = Wl[1] * n[d] + Wl[2] * t1[d] + Wl[3] * t2[d];
    W[4] = Wl[4];
}

/* G[3c+d] = dW_c/dx_d (global) -> Gl[j][c'] = dW'_c'/dx'_j in the (n,t1,t2) frame, stored [3][5]. */
void om_rotate_grad(const double *G, const double *n, const double *t1, const double *t2, double *Gl)
{
    const double *E[3] = {n, t1, t2};
    for (int j = 0; j < 3; ++j) {
        double dW[5];
        for (int c = 0; c < 5; ++c) dW[c] = G[3 * c] * E[j][0] + G[3 * c + 1] * E[j][1] + G[3 * c + 2] * E[j][2];
        om_rotate_state(dW, n, t1, t2, &Gl[5 * j]);
    }
}
