/*
 * CGKS CPU oracle -- two-step random-hash agglomeration, run sequentially.
 * TEST INFRASTRUCTURE ONLY (see om_internal.h).
 *
 * Paper Sec. 4.1 and Algorithm 1 (cell coarsening):
 *  - face hash h_f = [23 (N_l + N_r) + N_l N_r] % N_f over interior faces;
 *  - faces are visited in order; a face is a deletion candidate only if its
 *    hash value has not been seen before (first occurrence wins);
 *  - each candidate is checked for skewness against the virtual centre
 *    C_c = (V_l C_l + V_r C_r) / (V_l + V_r) and merged if acceptable;
 *  - boundary faces are never deleted;
 *  - coarse volume V_c = sum V_i, centre C_c = sum V_i C_i / V_c.
 * Readings (listed in the design notes):
 *  - the graph of a pass has one node per current agglomerate, numbered by its
 *    smallest member id, and one face per unordered adjacent pair (a < b) in
 *    lexicographic order; N_f is that pair count; the hash uses those ids and a
 *    seed multiplier s: h = (23 s (a+b) + a b) mod N_f in 64-bit unsigned;
 *  - merging is a greedy matching in ascending face order: a face merges its two
 *    agglomerates only if neither has merged in this pass;
 *  - skewness is tested without division: with e = V M - S P (V, P: summed
 *    volume and first moment of the two sides; S, M: summed area and first
 *    area moment of the pair's faces; A: summed area vector), accept iff
 *    (e.e)^3 <= delta^6 V^8 S^6 (virtual centre within delta V^(1/3) of the face
 *    centre) or (e.A)^2 >= s^2 (e.e)(A.A) (angle to the face plane >= asin s);
 *  - periodic faces are kept like boundary faces.
 */
#include "om_internal.h"
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t a, b, j;
    int rev;
} pkey;

static int cmp_pkey(const void *x, const void *y)
{
    const pkey *p = (const pkey *)x, *q = (const pkey *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->j != q->j) return p->j < q->j ? -1 : 1;
    return 0;
}

int om_skew_accept(double Va, double Vb, const double *Pa, const double *Pb, double S, const double *M,
                   const double *A, double delta, double smin)
{
    double V = Va + Vb;
    double P[3] = {Pa[0] + Pb[0], Pa[1] + Pb[1], Pa[2] + Pb[2]};
    double e[3];
    for (int d = 0; d < 3; ++d) e[d] = V * M[d] - S * P[d];
    double ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    double d2 = delta * delta;
    double d6 = d2 * d2 * d2;
    double V2 = V * V, V4 = V2 * V2, V8 = V4 * V4;
    double S2 = S * S, S6 = S2 * S2 * S2;
    if (ee * ee * ee <= d6 * V8 * S6) return 1;
    double ea = e[0] * A[0] + e[1] * A[1] + e[2] * A[2];
    double aa = A[0] * A[0] + A[1] * A[1] + A[2] * A[2];
    double s2 = smin * smin;
    return ea * ea >= s2 * ee * aa;
}

/*
 * One pass on the graph (n nodes, m pairs).  Writes map[n] (node -> new id) and the
 * new graph into the out arrays (sized n and m by the caller); returns the new node count,
 * writes the new pair count to *m_out and pass statistics to stats[4]
 * (selected, skew-accepted, merged, new pairs).
 */
int64_t om_agglo_pass(int64_t n, const double *V, const double *P, int64_t m, const int64_t *pa, const int64_t *pb,
                      const double *S, const double *M, const double *A, uint64_t seed, double delta, double smin,
                      int64_t *map, double *Vo, double *Po, int64_t *m_out, int64_t *pao, int64_t *pbo, double *So,
                      double *Mo, double *Ao, int64_t *stats)
{
    char *seen = (char *)calloc(m > 0 ? m : 1, 1);
    char *matched = (char *)calloc(n > 0 ? n : 1, 1);
    int64_t *mate = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) mate[i] = -1;
    int64_t nsel = 0, nacc = 0, nmerge = 0;
    const uint64_t Nf = (uint64_t)m;
    for (int64_t j = 0; j < m; ++j) {
        uint64_t a = (uint64_t)pa[j], b = (uint64_t)pb[j];
        uint64_t h = (23u * seed * (a + b) + a * b) % Nf;
        if (seen[h]) continue;
        seen[h] = 1;
        ++nsel;
        if (!om_skew_accept(V[pa[j]], V[pb[j]], &P[3 * pa[j]], &P[3 * pb[j]], S[j], &M[3 * j], &A[3 * j], delta, smin))
            continue;
        ++nacc;
        if (matched[pa[j]] || matched[pb[j]]) continue;
        matched[pa[j]] = matched[pb[j]] = 1;
        mate[pb[j]] = pa[j];
        ++nmerge;
    }
    int64_t nn = 0;
    for (int64_t i = 0; i < n; ++i)
        if (mate[i] < 0) map[i] = nn++;
    for (int64_t i = 0; i < n; ++i)
        if (mate[i] >= 0) map[i] = map[mate[i]];
    for (int64_t i = 0; i < n; ++i)
        if (mate[i] < 0) {
            Vo[map[i]] = V[i];
            for (int d = 0; d < 3; ++d) Po[3 * map[i] + d] = P[3 * i + d];
        }
    for (int64_t i = 0; i < n; ++i)
        if (mate[i] >= 0) {
            int64_t a = mate[i], k = map[i];
            Vo[k] = V[a] + V[i];
            for (int d = 0; d < 3; ++d) Po[3 * k + d] = P[3 * a + d] + P[3 * i + d];
        }
    pkey *K = (pkey *)malloc(sizeof(pkey) * (m > 0 ? m : 1));
    int64_t nk = 0;
    for (int64_t j = 0; j < m; ++j) {
        int64_t a = map[pa[j]], b = map[pb[j]];
        if (a == b) continue;
        K[nk].a = a < b ? a : b;
        K[nk].b = a < b ? b : a;
        K[nk].j = j;
        K[nk].rev = a > b;
        ++nk;
    }
    /* sort by new pair, then by face index of this pass */
    qsort(K, nk, sizeof(pkey), cmp_pkey);
    int64_t mo = 0;
    for (int64_t i = 0; i < nk;) {
        int64_t e = i;
        double s = 0, mm[3] = {0, 0, 0}, aa[3] = {0, 0, 0};
        while (e < nk && K[e].a == K[i].a && K[e].b == K[i].b) {
            int64_t j = K[e].j;
            s += S[j];
            for (int d = 0; d < 3; ++d) {
                mm[d] += M[3 * j + d];
                aa[d] += K[e].rev ? -A[3 * j + d] : A[3 * j + d];
            }
            ++e;
        }
        pao[mo] = K[i].a;
        pbo[mo] = K[i].b;
        So[mo] = s;
        for (int d = 0; d < 3; ++d) {
            Mo[3 * mo + d] = mm[d];
            Ao[3 * mo + d] = aa[d];
        }
        ++mo;
        i = e;
    }
    *m_out = mo;
    if (stats) {
        stats[0] = nsel;
        stats[1] = nacc;
        stats[2] = nmerge;
        stats[3] = mo;
    }
    free(K);
    free(seen);
    free(matched);
    free(mate);
    return nn;
}

/*
 * P passes on a graph; f2c[n] receives the composed map.  Output arrays are sized
 * like the input (n nodes, m pairs); returns the final node count.
 */
int64_t om_agglomerate_graph(int64_t n, const double *V, const double *P, int64_t m, const int64_t *pa,
                             const int64_t *pb, const double *S, const double *M, const double *A, uint64_t seed,
                             int passes, double delta, double smin, int64_t *f2c, double *Vo, double *Po,
                             int64_t *m_out, int64_t *pao, int64_t *pbo, double *So, double *Mo, double *Ao,
                             int64_t *stats /* 4 per pass */)
{
    int64_t cn = n, cm = m;
    double *cV = malloc(sizeof(double) * n), *cP = malloc(sizeof(double) * 3 * n);
    int64_t *ca = malloc(sizeof(int64_t) * (m + 1)), *cb = malloc(sizeof(int64_t) * (m + 1));
    double *cS = malloc(sizeof(double) * (m + 1)), *cM = malloc(sizeof(double) * 3 * (m + 1)),
           *cA = malloc(sizeof(double) * 3 * (m + 1));
    memcpy(cV, V, sizeof(double) * n);
    memcpy(cP, P, sizeof(double) * 3 * n);
    memcpy(ca, pa, sizeof(int64_t) * m);
    memcpy(cb, pb, sizeof(int64_t) * m);
    memcpy(cS, S, sizeof(double) * m);
    memcpy(cM, M, sizeof(double) * 3 * m);
    memcpy(cA, A, sizeof(double) * 3 * m);
    for (int64_t i = 0; i < n; ++i) f2c[i] = i;
    int64_t *map = malloc(sizeof(int64_t) * n);
    for (int pass = 0; pass < passes; ++pass) {
        int64_t nm = 0;
        int64_t nn = om_agglo_pass(cn, cV, cP, cm, ca, cb, cS, cM, cA, seed, delta, smin, map, Vo, Po, &nm, pao, pbo,
                                   So, Mo, Ao, stats ? &stats[4 * pass] : NULL);
        for (int64_t i = 0; i < n; ++i) f2c[i] = map[f2c[i]];
        cn = nn;
        cm = nm;
        memcpy(cV, Vo, sizeof(double) * nn);
        memcpy(cP, Po, sizeof(double) * 3 * nn);
        memcpy(ca, pao, sizeof(int64_t) * nm);
        memcpy(cb, pbo, sizeof(int64_t) * nm);
        memcpy(cS, So, sizeof(double) * nm);
        memcpy(cM, Mo, sizeof(double) * 3 * nm);
        memcpy(cA, Ao, sizeof(double) * 3 * nm);
    }
    if (passes == 0) {
        memcpy(Vo, V, sizeof(double) * n);
        memcpy(Po, P, sizeof(double) * 3 * n);
        memcpy(pao, pa, sizeof(int64_t) * m);
        memcpy(pbo, pb, sizeof(int64_t) * m);
        memcpy(So, S, sizeof(double) * m);
        memcpy(Mo, M, sizeof(double) * 3 * m);
        memcpy(Ao, A, sizeof(double) * 3 * m);
    }
    *m_out = cm;
    free(map);
    free(cV);
    free(cP);
    free(ca);
    free(cb);
    free(cS);
    free(cM);
    free(cA);
    return cn;
}

/* face hash of one pair, exposed for pins */
uint64_t om_face_hash(uint64_t a, uint64_t b, uint64_t nf, uint64_t seed)
{
    return (23u * seed * (a + b) + a * b) % nf;
}
