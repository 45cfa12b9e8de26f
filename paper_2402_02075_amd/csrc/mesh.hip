// Mesh ingest: face connectivity on the host (integer work), geometry and the
// reconstruction operators on the device.
//
// Paper Sec. 2.2: hybrid cells (tet, pyramid, prism, hexahedron) with linear
// iso-parametric faces; 3 Gauss points per triangle, 4 per quadrilateral, fluxes
// in the local face frame.  Sec. 3.1: the large-stencil quadratic p^2 is the
// constrained least-squares fit to the neighbour averages (exact) and neighbour
// gradient averages (least squares).  Because the fit is linear in the data, its
// solution operator is formed once per cell here (9 x 4 nb numbers), and the
// per-evaluation reconstruction only applies it.
//
// Readings: triangles use the degree-2 rule at barycentric (2/3,1/6,1/6) with
// weights 1/3, quadrilaterals 2x2 Gauss on the bilinear map; cell moments come
// from 3x3x3 Gauss on the trilinear map of the element written as a (possibly
// collapsed) hexahedron; gradient rows of p^2 are scaled by |Omega_0|^(1/3);
// cells with fewer than three interior neighbours use the linear p^1 alone.
#include <algorithm>
#include <numeric>
#include <parallel/algorithm>

#include "common.hpp"

namespace cgks {

namespace {

// local faces in VTK order; -1 pads triangles
const int kTetF[4][4] = {{0, 1, 3, -1}, {1, 2, 3, -1}, {2, 0, 3, -1}, {0, 2, 1, -1}};
const int kPyrF[5][4] = {{0, 1, 2, 3}, {0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}};
const int kPriF[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
const int kHexF[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
// element node -> collapsed hexahedron corner
const int kTetH[8] = {0, 1, 2, 2, 3, 3, 3, 3};
const int kPyrH[8] = {0, 1, 2, 3, 4, 4, 4, 4};
const int kPriH[8] = {0, 1, 2, 2, 3, 4, 5, 5};
const int kHexH[8] = {0, 1, 2, 3, 4, 5, 6, 7};

int faces_of(int t) { return t == 4 ? 4 : (t == 8 ? 6 : 5); }
const int *face_of(int t, int f)
{
    return t == 4 ? kTetF[f] : t == 5 ? kPyrF[f] : t == 6 ? kPriF[f] : kHexF[f];
}
const int *hex_of(int t) { return t == 4 ? kTetH : t == 5 ? kPyrH : t == 6 ? kPriH : kHexH; }

struct SideRec {
    uint64_t k0, k1;  // sorted canonical ids packed two by two; 0xffffffff pads a triangle
    int32_t cell;     // -1 for a boundary record
    int32_t aux;      // local face (cell side) or tag (boundary)
};

inline void pack_key(int64_t *ids, int nn, SideRec &r)
{
    uint32_t v[4];
    for (int i = 0; i < 4; ++i) v[i] = i < nn ? (uint32_t)ids[i] : 0xffffffffu;
    std::sort(v, v + 4);
    r.k0 = ((uint64_t)v[0] << 32) | v[1];
    r.k1 = ((uint64_t)v[2] << 32) | v[3];
}

struct FaceRec {
    int32_t L, R, lfL, lfR, tag;
};

}  // namespace

// ------------------------------------------------------------------ kernels
__global__ void k_cell_geom(int64_t N, const double *__restrict__ xyz, const int32_t *__restrict__ hexn,
                            double *__restrict__ vol, double *__restrict__ cen, double *__restrict__ mom2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double X[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int64_t nd = hexn[a * N + i];
#pragma unroll
        for (int d = 0; d < 3; ++d) X[a][d] = xyz[3 * nd + d];
    }
    const double r = 0.5 * sqrt(0.6);
    const double gp[3] = {0.5 - r, 0.5, 0.5 + r};
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    // two passes: volume and first moment, then central second moments
    double V = 0, P[3] = {0, 0, 0}, Q[6] = {0, 0, 0, 0, 0, 0};
    double c0[3] = {0, 0, 0};
    for (int pass = 0; pass < 2; ++pass) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int e = 0; e < 3; ++e) {
                    const double s = gp[a], t = gp[b], u = gp[e];
                    const double sm = 1 - s, tm = 1 - t, um = 1 - u;
                    // trilinear shape functions, hexahedron corners 0..7 (VTK)
                    const double Nf[8] = {sm * tm * um, s * tm * um, s * t * um, sm * t * um,
                                          sm * tm * u,  s * tm * u,  s * t * u,  sm * t * u};
                    const double Ns[8] = {-tm * um, tm * um, t * um, -t * um, -tm * u, tm * u, t * u, -t * u};
                    const double Nt[8] = {-sm * um, -s * um, s * um, sm * um, -sm * u, -s * u, s * u, sm * u};
                    const double Nu[8] = {-sm * tm, -s * tm, -s * t, -sm * t, sm * tm, s * tm, s * t, sm * t};
                    double x[3] = {0, 0, 0}, js[3] = {0, 0, 0}, jt[3] = {0, 0, 0}, ju[3] = {0, 0, 0};
#pragma unroll
                    for (int q = 0; q < 8; ++q)
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            x[d] += Nf[q] * X[q][d];
                            js[d] += Ns[q] * X[q][d];
                            jt[d] += Nt[q] * X[q][d];
                            ju[d] += Nu[q] * X[q][d];
                        }
                    const double det = js[0] * (jt[1] * ju[2] - jt[2] * ju[1]) - js[1] * (jt[0] * ju[2] - jt[2] * ju[0]) +
                                       js[2] * (jt[0] * ju[1] - jt[1] * ju[0]);
                    const double w = gw[a] * gw[b] * gw[e] * det;
                    if (pass == 0) {
                        V += w;
#pragma unroll
                        for (int d = 0; d < 3; ++d) P[d] += w * x[d];
                    } else {
                        const double dx = x[0] - c0[0], dy = x[1] - c0[1], dz = x[2] - c0[2];
                        Q[0] += w * dx * dx;
                        Q[1] += w * dy * dy;
                        Q[2] += w * dz * dz;
                        Q[3] += w * dx * dy;
                        Q[4] += w * dy * dz;
                        Q[5] += w * dx * dz;
                    }
                }
        if (pass == 0)
            for (int d = 0; d < 3; ++d) c0[d] = P[d] / V;
    }
    const double sg = V < 0 ? -1.0 : 1.0;
    vol[i] = sg * V;
#pragma unroll
    for (int d = 0; d < 3; ++d) cen[d * N + i] = c0[d];
#pragma unroll
    for (int q = 0; q < 6; ++q) mom2[q * N + i] = sg * Q[q];
}

__global__ void k_face_geom(int64_t F, int64_t N, const double *__restrict__ xyz, const int32_t *__restrict__ fnode,
                            const int32_t *__restrict__ fl, const double *__restrict__ cen,
                            const int32_t *__restrict__ fshiftn, int32_t *__restrict__ fngp, double *__restrict__ gpx,
                            double *__restrict__ gpw, double *__restrict__ gpn, double *__restrict__ farea,
                            double *__restrict__ favec, double *__restrict__ fmom, double *__restrict__ fshift)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int nn = fnode[3 * F + f] < 0 ? 3 : 4;
    double P[4][3];
    for (int a = 0; a < nn; ++a) {
        const int64_t nd = fnode[a * F + f];
        for (int d = 0; d < 3; ++d) P[a][d] = xyz[3 * nd + d];
    }
    // orientation: outward from L
    double J0[3], e1[3], e2[3], mid[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        e1[d] = nn == 3 ? P[1][d] - P[0][d] : P[2][d] - P[0][d];
        e2[d] = nn == 3 ? P[2][d] - P[0][d] : P[3][d] - P[1][d];
        for (int a = 0; a < nn; ++a) mid[d] += P[a][d];
        mid[d] /= nn;
    }
    J0[0] = e1[1] * e2[2] - e1[2] * e2[1];
    J0[1] = e1[2] * e2[0] - e1[0] * e2[2];
    J0[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const int L = fl[f];
    const double side = J0[0] * (mid[0] - cen[L]) + J0[1] * (mid[1] - cen[N + L]) + J0[2] * (mid[2] - cen[2 * N + L]);
    if (side < 0) {
        // reverse the cycle, keep node 0
        for (int d = 0; d < 3; ++d) {
            const double t = P[1][d];
            P[1][d] = P[nn - 1][d];
            P[nn - 1][d] = t;
        }
    }
    double S = 0, Av[3] = {0, 0, 0}, Mv[3] = {0, 0, 0};
    if (nn == 3) {
        double a[3], b[3], J[3];
        for (int d = 0; d < 3; ++d) {
            a[d] = P[1][d] - P[0][d];
            b[d] = P[2][d] - P[0][d];
        }
        J[0] = a[1] * b[2] - a[2] * b[1];
        J[1] = a[2] * b[0] - a[0] * b[2];
        J[2] = a[0] * b[1] - a[1] * b[0];
        const double nj = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
        S = 0.5 * nj;
        const double big = 2.0 / 3.0, sm = 1.0 / 6.0;
        for (int k = 0; k < 3; ++k) {
            const double w0 = k == 0 ? big : sm, w1 = k == 1 ? big : sm, w2 = k == 2 ? big : sm;
            for (int d = 0; d < 3; ++d) {
                const double x = w0 * P[0][d] + w1 * P[1][d] + w2 * P[2][d];
                gpx[(3 * k + d) * F + f] = x;
                gpn[(3 * k + d) * F + f] = J[d] / nj;
                Mv[d] += S * x / 3.0;
            }
            gpw[k * F + f] = S / 3.0;
        }
        for (int d = 0; d < 3; ++d) {
            gpx[(9 + d) * F + f] = 0;
            gpn[(9 + d) * F + f] = 0;
            Av[d] = 0.5 * J[d];
        }
        gpw[3 * F + f] = 0;
        fngp[f] = 3;
    } else {
        const double h = 0.5 / sqrt(3.0);
        const double st[4][2] = {{0.5 - h, 0.5 - h}, {0.5 + h, 0.5 - h}, {0.5 + h, 0.5 + h}, {0.5 - h, 0.5 + h}};
        for (int k = 0; k < 4; ++k) {
            const double s = st[k][0], t = st[k][1];
            double xs[3], xt[3], J[3], x[3];
            for (int d = 0; d < 3; ++d) {
                x[d] = (1 - s) * (1 - t) * P[0][d] + s * (1 - t) * P[1][d] + s * t * P[2][d] + (1 - s) * t * P[3][d];
                xs[d] = (1 - t) * (P[1][d] - P[0][d]) + t * (P[2][d] - P[3][d]);
                xt[d] = (1 - s) * (P[3][d] - P[0][d]) + s * (P[2][d] - P[1][d]);
            }
            J[0] = xs[1] * xt[2] - xs[2] * xt[1];
            J[1] = xs[2] * xt[0] - xs[0] * xt[2];
            J[2] = xs[0] * xt[1] - xs[1] * xt[0];
            const double nj = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
            const double w = 0.25 * nj;
            S += w;
            for (int d = 0; d < 3; ++d) {
                gpx[(3 * k + d) * F + f] = x[d];
                gpn[(3 * k + d) * F + f] = J[d] / nj;
                Av[d] += 0.25 * J[d];
                Mv[d] += w * x[d];
            }
            gpw[k * F + f] = w;
        }
        fngp[f] = 4;
    }
    farea[f] = S;
    for (int d = 0; d < 3; ++d) {
        favec[d * F + f] = Av[d];
        fmom[d * F + f] = Mv[d];
    }
    const int a0 = fshiftn[f], b0 = fshiftn[F + f];
    for (int d = 0; d < 3; ++d) fshift[d * F + f] = a0 >= 0 ? xyz[3 * a0 + d] - xyz[3 * b0 + d] : 0.0;
}

__global__ void k_slots(int64_t N, int64_t F, const int32_t *__restrict__ cf_ptr, const int32_t *__restrict__ cf_face,
                        const int32_t *__restrict__ fl, const int32_t *__restrict__ fr, const double *__restrict__ favec,
                        const double *__restrict__ vol, int32_t *__restrict__ slot_nb, double *__restrict__ slot_av)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = cf_ptr[i], e = cf_ptr[i + 1];
    const double iv = 1.0 / vol[i];
    for (int s = 0; s < 6; ++s) {
        if (b + s < e) {
            const int it = cf_face[b + s];
            const int f = it >> 1;
            const bool isR = it & 1;
            slot_nb[s * N + i] = fr[f] >= 0 ? (isR ? fl[f] : fr[f]) : -(f + 1);
            const double sg = isR ? -iv : iv;
            for (int d = 0; d < 3; ++d) slot_av[(3 * s + d) * N + i] = sg * favec[d * F + f];
        } else {
            slot_nb[s * N + i] = INT32_MIN;
            for (int d = 0; d < 3; ++d) slot_av[(3 * s + d) * N + i] = 0;
        }
    }
}

// Per face-kernel lane (lane-major, coalesced): Gauss point offsets from the left and right
// cell centroids (the right one through the periodic shift), unit normal, weight w_k S, and
// the packed indices {4 f + k, L, R, 8 tag + ngp}; idle lanes get zeros and f = -1.
__global__ void k_lane_geom(int64_t NL, int64_t F, int64_t N, const int32_t *__restrict__ lmap,
                            const double *__restrict__ gpx, const double *__restrict__ gpn,
                            const double *__restrict__ gpw, const double *__restrict__ fshift,
                            const double *__restrict__ cen, const int32_t *__restrict__ fl,
                            const int32_t *__restrict__ fr, const int32_t *__restrict__ ftag,
                            const int32_t *__restrict__ fngp, int4 *__restrict__ lidx, double *__restrict__ lgeo)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NL) return;
    const int lm = lmap[t];
    if (lm < 0) {
        lidx[t] = make_int4(-1, 0, 0, 0);
        for (int q = 0; q < 10; ++q) lgeo[q * NL + t] = 0.0;
        return;
    }
    const int64_t f = lm >> 2;
    const int k = lm & 3;
    const int L = fl[f], R = fr[f];
    lidx[t] = make_int4(lm, L, R, 8 * ftag[f] + fngp[f]);
    for (int d = 0; d < 3; ++d) {
        const double x = gpx[(3 * k + d) * F + f];
        lgeo[d * NL + t] = x - cen[d * N + L];
        lgeo[(3 + d) * NL + t] = R >= 0 ? x - fshift[d * F + f] - cen[d * N + R] : 0.0;
        lgeo[(6 + d) * NL + t] = gpn[(3 * k + d) * F + f];
    }
    lgeo[9 * NL + t] = gpw[k * F + f];
}

// Area vectors / |Omega| of each cell's interior faces in neighbour order (the slot vectors
// with the boundary slots left out), for the reconstruction's Green-Gauss term.
__global__ void k_iav(int64_t N, const int32_t *__restrict__ slot_nb, const double *__restrict__ slot_av,
                      double *__restrict__ iav)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int m = 0;
    for (int s = 0; s < 6; ++s) {
        const int nbv = slot_nb[s * N + i];
        if (nbv == INT32_MIN) break;
        if (nbv < 0) continue;
        for (int d = 0; d < 3; ++d) iav[(3 * m + d) * N + i] = slot_av[(3 * s + d) * N + i];
        ++m;
    }
    for (; m < 6; ++m)
        for (int d = 0; d < 3; ++d) iav[(3 * m + d) * N + i] = 0.0;
}

// Per cell: solution operator of the constrained least-squares system of p^2 and the
// linear least-squares operator used by the smoothness indicator beta_1,LS.
//  unknowns a_1..a_9 of sum_k a_k (phi_k - avg_0 phi_k), phi = dx dy dz dx^2 dy^2 dz^2 dxdy dydz dxdz;
//  rows: neighbour averages exactly (Lagrange multipliers), h0-scaled gradient averages in LS.
//  Solution columns: col < nb multiplies (Q_m - Q_0), col = nb + 3m + d multiplies (dQ/dx_d)_m;
//  stored per interior neighbour m as 39 entries (see the reconstruction kernel), stride 64.
__global__ void k_op_build(int64_t N, int64_t F, const int32_t *__restrict__ cf_ptr, const int32_t *__restrict__ cf_face,
                           const int32_t *__restrict__ fl, const int32_t *__restrict__ fr,
                           const double *__restrict__ fshift, const double *__restrict__ vol,
                           const double *__restrict__ cen, const double *__restrict__ mom2,
                           const int64_t *__restrict__ op_off, double *__restrict__ op, int32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t off = op_off[i];
    if (off < 0) return;
    double D[6][3];
    int nbr[6];
    int nb = 0;
    for (int k = cf_ptr[i]; k < cf_ptr[i + 1]; ++k) {
        const int it = cf_face[k];
        const int f = it >> 1;
        if (fr[f] < 0) continue;
        const bool isR = it & 1;
        const int o = isR ? fl[f] : fr[f];
        const double sg = isR ? -1.0 : 1.0;
        for (int d = 0; d < 3; ++d) D[nb][d] = cen[d * N + o] + sg * fshift[d * F + f] - cen[d * N + i];
        nbr[nb++] = o;
    }
    const int n = 9 + nb, nc = 4 * nb;
    double K[15][15];
    double B[15][24];
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) K[r][c] = 0;
        for (int c = 0; c < nc; ++c) B[r][c] = 0;
    }
    const double V0 = vol[i];
    const double h0 = cbrt(V0), h2 = h0 * h0;
    double avg0[9] = {0, 0, 0, mom2[0 * N + i] / V0, mom2[1 * N + i] / V0, mom2[2 * N + i] / V0,
                      mom2[3 * N + i] / V0, mom2[4 * N + i] / V0, mom2[5 * N + i] / V0};
    for (int m = 0; m < nb; ++m) {
        const int o = nbr[m];
        const double Vm = vol[o];
        const double X = D[m][0], Y = D[m][1], Z = D[m][2];
        const double avgm[9] = {X, Y, Z, mom2[0 * N + o] / Vm + X * X, mom2[1 * N + o] / Vm + Y * Y,
                                mom2[2 * N + o] / Vm + Z * Z, mom2[3 * N + o] / Vm + X * Y,
                                mom2[4 * N + o] / Vm + Y * Z, mom2[5 * N + o] / Vm + X * Z};
        const double g[3][9] = {{1, 0, 0, 2 * X, 0, 0, Y, 0, Z}, {0, 1, 0, 0, 2 * Y, 0, X, Z, 0}, {0, 0, 1, 0, 0, 2 * Z, 0, Y, X}};
        for (int k = 0; k < 9; ++k) {
            K[9 + m][k] = avgm[k] - avg0[k];
            K[k][9 + m] = avgm[k] - avg0[k];
        }
        B[9 + m][m] = 1.0;
        for (int d = 0; d < 3; ++d) {
            for (int a = 0; a < 9; ++a) {
                for (int b = 0; b < 9; ++b) K[a][b] += 2.0 * h2 * g[d][a] * g[d][b];
                B[a][nb + 3 * m + d] = 2.0 * h2 * g[d][a];
            }
        }
    }
    // Gaussian elimination with partial pivoting on [K | B]
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(K[c][c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(K[r][c]) > best) best = fabs(K[r][c]), p = r;
        if (best == 0.0) {
            atomicMin(bad, (int32_t)i);
            return;
        }
        if (p != c) {
            for (int q = 0; q < n; ++q) {
                const double t = K[c][q];
                K[c][q] = K[p][q];
                K[p][q] = t;
            }
            for (int q = 0; q < nc; ++q) {
                const double t = B[c][q];
                B[c][q] = B[p][q];
                B[p][q] = t;
            }
        }
        const double piv = 1.0 / K[c][c];
        for (int r = c + 1; r < n; ++r) {
            const double f = K[r][c] * piv;
            if (f == 0.0) continue;
            for (int q = c; q < n; ++q) K[r][q] -= f * K[c][q];
            for (int q = 0; q < nc; ++q) B[r][q] -= f * B[c][q];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int q = 0; q < nc; ++q) {
            double s = B[c][q];
            for (int r = c + 1; r < n; ++r) s -= K[c][r] * B[r][q];
            B[c][q] = s / K[c][c];
        }
    }
    // entry m*39 + j of the cell, stride 64 (group-interleaved)
    for (int m = 0; m < nb; ++m)
        for (int k = 0; k < 9; ++k) {
            op[off + 64 * (39 * m + k)] = B[k][m];
            for (int d = 0; d < 3; ++d) op[off + 64 * (39 * m + 9 + 3 * k + d)] = B[k][nb + 3 * m + d];
        }
    // linear least squares: (sum D D^T)^-1 D_m
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int m = 0; m < nb; ++m)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] += D[m][a] * D[m][b];
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (det == 0.0) {
        atomicMin(bad, (int32_t)i);
        return;
    }
    double Ai[3][3];
    Ai[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    Ai[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    Ai[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < nb; ++m)
            op[off + 64 * (39 * m + 36 + d)] = Ai[d][0] * D[m][0] + Ai[d][1] * D[m][1] + Ai[d][2] * D[m][2];
}

// ------------------------------------------------------------------ host ingest
void mesh_build(cgks_ctx *c, int64_t n_nodes, const double *xyz, int64_t N, const uint8_t *ctype, const int64_t *cptr,
                const int64_t *cnode, int64_t n_bf, const int64_t *bptr, const int64_t *bnode, const int32_t *btag,
                const int64_t *canon)
{
    if (N <= 0 || n_nodes <= 0 || N > INT32_MAX / 2 || n_nodes > INT32_MAX)
        throw Error{CGKS_E_ARG, "mesh sizes out of range"};
    hipStream_t s = c->stream;
    // per-cell corner map and face sides
    std::vector<int32_t> hexn(8 * N);
    int64_t nside = 0;
    for (int64_t i = 0; i < N; ++i) {
        const int t = ctype[i];
        if ((t != 4 && t != 5 && t != 6 && t != 8) || cptr[i + 1] - cptr[i] != t)
            throw Error{CGKS_E_MESH, "cell " + std::to_string(c->caller_cell(i)) + ": unsupported type or node count"};
        const int *hm = hex_of(t);
        for (int a = 0; a < 8; ++a) {
            const int64_t nd = cnode[cptr[i] + hm[a]];
            if (nd < 0 || nd >= n_nodes)
                throw Error{CGKS_E_MESH, "cell " + std::to_string(c->caller_cell(i)) + ": node out of range"};
            hexn[a * N + i] = (int32_t)nd;
        }
        nside += faces_of(t);
    }
    std::vector<SideRec> sides(nside + n_bf);
    {
        int64_t q = 0;
        for (int64_t i = 0; i < N; ++i) {
            const int t = ctype[i];
            for (int f = 0; f < faces_of(t); ++f, ++q) {
                const int *lf = face_of(t, f);
                const int nn = lf[3] < 0 ? 3 : 4;
                int64_t ids[4];
                for (int a = 0; a < nn; ++a) {
                    const int64_t nd = cnode[cptr[i] + lf[a]];
                    ids[a] = canon ? canon[nd] : nd;
                }
                pack_key(ids, nn, sides[q]);
                sides[q].cell = (int32_t)i;
                sides[q].aux = f;
            }
        }
        for (int64_t b = 0; b < n_bf; ++b, ++q) {
            const int nn = (int)(bptr[b + 1] - bptr[b]);
            if (nn != 3 && nn != 4) throw Error{CGKS_E_MESH, "boundary face " + std::to_string(b) + ": not 3 or 4 nodes"};
            if (btag[b] < 1 || btag[b] > 63) throw Error{CGKS_E_MESH, "boundary face " + std::to_string(b) + ": tag not in 1..63"};
            int64_t ids[4];
            for (int a = 0; a < nn; ++a) ids[a] = canon ? canon[bnode[bptr[b] + a]] : bnode[bptr[b] + a];
            pack_key(ids, nn, sides[q]);
            sides[q].cell = -1;
            sides[q].aux = btag[b];
        }
    }
    __gnu_parallel::sort(sides.begin(), sides.end(), [](const SideRec &a, const SideRec &b) {
        if (a.k0 != b.k0) return a.k0 < b.k0;
        if (a.k1 != b.k1) return a.k1 < b.k1;
        // cell sides (cell >= 0) before boundary records, then by cell
        const bool ba = a.cell < 0, bb = b.cell < 0;
        if (ba != bb) return bb;
        return a.cell < b.cell;
    });
    std::vector<FaceRec> faces;
    faces.reserve(nside / 2 + n_bf);
    for (size_t i = 0; i < sides.size();) {
        size_t j = i;
        while (j < sides.size() && sides[j].k0 == sides[i].k0 && sides[j].k1 == sides[i].k1) ++j;
        const size_t cnt = j - i;
        if (cnt == 2 && sides[i].cell >= 0 && sides[i + 1].cell >= 0) {
            faces.push_back({sides[i].cell, sides[i + 1].cell, sides[i].aux, sides[i + 1].aux, 0});
        } else if (cnt == 2 && sides[i].cell >= 0 && sides[i + 1].cell < 0) {
            faces.push_back({sides[i].cell, -1, sides[i].aux, -1, sides[i + 1].aux});
        } else {
            throw Error{CGKS_E_MESH, "non-conforming face at cell " + std::to_string(c->caller_cell(sides[i].cell)) + " (" +
                                         std::to_string(cnt) + " records)"};
        }
        i = j;
    }
    std::vector<SideRec>().swap(sides);
    __gnu_parallel::sort(faces.begin(), faces.end(), [](const FaceRec &a, const FaceRec &b) {
        const bool ba = a.R < 0, bb = b.R < 0;
        if (ba != bb) return bb;
        if (a.L != b.L) return a.L < b.L;
        if (a.R != b.R) return a.R < b.R;
        return a.lfL < b.lfL;
    });
    const int64_t F = (int64_t)faces.size();
    int64_t Fi = 0;
    while (Fi < F && faces[Fi].R >= 0) ++Fi;
    std::vector<int32_t> hfl(F), hfr(F), htag(F), fnode(4 * F), fshn(2 * F, -1);
    std::vector<int32_t> deg(N + 1, 0);
    int64_t ngp = 0;
    std::vector<int32_t> gpoff(F);  // first Gauss point of each face in a compact numbering
    std::vector<int32_t> lmap;  // face-kernel lanes: 4 f + k, or -1 for an idle lane
    lmap.reserve(4 * F + 256);
    for (int64_t f = 0; f < F; ++f) {
        const FaceRec &r = faces[f];
        hfl[f] = r.L;
        hfr[f] = r.R;
        htag[f] = r.tag;
        const int *lf = face_of(ctype[r.L], r.lfL);
        const int nn = lf[3] < 0 ? 3 : 4;
        gpoff[f] = (int32_t)ngp;
        ngp += nn;
        // pack faces into 64-lane waves, nn lanes each, never splitting a face across waves
        if ((int64_t)(lmap.size() % 64) + nn > 64)
            while (lmap.size() % 64) lmap.push_back(-1);
        for (int k = 0; k < nn; ++k) lmap.push_back((int32_t)(4 * f + k));
        for (int a = 0; a < 4; ++a) fnode[a * F + f] = a < nn ? (int32_t)cnode[cptr[r.L] + lf[a]] : -1;
        deg[r.L + 1]++;
        if (r.R >= 0) {
            deg[r.R + 1]++;
            if (canon) {
                // translation between the two images of a periodic face
                const int *rf = face_of(ctype[r.R], r.lfR);
                int64_t best = INT64_MAX;
                int32_t nl = -1;
                for (int a = 0; a < nn; ++a) {
                    const int64_t nd = cnode[cptr[r.L] + lf[a]];
                    if (canon[nd] < best) best = canon[nd], nl = (int32_t)nd;
                }
                int32_t nr = -1;
                for (int a = 0; a < nn; ++a) {
                    const int64_t nd = cnode[cptr[r.R] + rf[a]];
                    if (canon[nd] == best) nr = (int32_t)nd;
                }
                if (nl != nr) {
                    fshn[f] = nl;
                    fshn[F + f] = nr;
                }
            }
        }
    }
    for (int64_t i = 0; i < N; ++i) deg[i + 1] += deg[i];
    std::vector<int32_t> cfp(deg.begin(), deg.end()), cff(deg[N]);
    {
        std::vector<int32_t> fill(N, 0);
        for (int64_t f = 0; f < F; ++f) {
            const int L = hfl[f], R = hfr[f];
            cff[cfp[L] + fill[L]++] = (int32_t)(2 * f);
            if (R >= 0) cff[cfp[R] + fill[R]++] = (int32_t)(2 * f + 1);
        }
    }
    for (int64_t i = 0; i < N; ++i)
        if (cfp[i + 1] - cfp[i] != faces_of(ctype[i]))
            throw Error{CGKS_E_MESH, "cell " + std::to_string(c->caller_cell(i)) + ": face count mismatch"};
    // interior neighbour counts and operator offsets
    std::vector<uint8_t> nint(N, 0);
    for (int64_t f = 0; f < Fi; ++f) {
        nint[hfl[f]]++;
        nint[hfr[f]]++;
    }
    // Operators are interleaved over groups of 64 consecutive cells: entry e of cell i is
    // at op_off[i] + 64 e, each group sized for its largest interior-neighbour count.
    std::vector<int64_t> off(N), gbase((N + 63) / 64);
    std::vector<int32_t> gnb((N + 63) / 64), gmx((N + 63) / 64);
    int64_t tot = 0;
    for (int64_t g0 = 0; g0 < N; g0 += 64) {
        const int64_t g1 = std::min<int64_t>(N, g0 + 64);
        int nbmax = 0;
        for (int64_t i = g0; i < g1; ++i)
            if (nint[i] >= 3) nbmax = std::max<int>(nbmax, nint[i]);
        for (int64_t i = g0; i < g1; ++i) off[i] = nint[i] >= 3 ? tot + (i - g0) : -1;
        gbase[g0 / 64] = tot;
        gnb[g0 / 64] = nbmax;
        int am = 0;
        for (int64_t i = g0; i < g1; ++i) am = std::max<int>(am, nint[i]);
        gmx[g0 / 64] = am;
        tot += 64 * 39 * (int64_t)nbmax;
    }
    // interior neighbours of each cell in face (slot) order, the order of the operator columns
    std::vector<int32_t> inbh(6 * N, -1);
    for (int64_t i = 0; i < N; ++i) {
        int m = 0;
        for (int32_t k = cfp[i]; k < cfp[i + 1]; ++k) {
            const int64_t f = cff[k] >> 1;
            if (hfr[f] < 0) continue;
            inbh[m++ * N + i] = (cff[k] & 1) ? hfl[f] : hfr[f];
        }
    }
    // upload and compute geometry
    c->N = N;
    c->F = F;
    c->Fi = Fi;
    c->Fb = F - Fi;
    c->NGP = ngp;
    while (lmap.size() % 256) lmap.push_back(-1);
    c->NL = (int64_t)lmap.size();
    c->lmap.upload(lmap, s);
    c->gpoff.upload(gpoff, s);
    DBuf<double> dxyz;
    DBuf<int32_t> dhexn, dfnode, dfsh;
    dxyz.upload(xyz, 3 * n_nodes, s);
    dhexn.upload(hexn, s);
    dfnode.upload(fnode, s);
    dfsh.upload(fshn, s);
    c->fl.upload(hfl, s);
    c->fr.upload(hfr, s);
    c->ftag.upload(htag, s);
    c->tags_used = 0;
    for (int64_t f = Fi; f < F; ++f) c->tags_used |= uint64_t(1) << (htag[f] & 63);
    c->cf_ptr.upload(cfp, s);
    c->cf_face.upload(cff, s);
    c->n_int.upload(nint, s);
    c->op_off.upload(off, s);
    c->op_gbase.upload(gbase, s);
    c->op_gnb.upload(gnb, s);
    c->op_gmax.upload(gmx, s);
    c->inb.upload(inbh, s);
    {
        std::vector<uint8_t> nf(N);
        for (int64_t i = 0; i < N; ++i) nf[i] = (uint8_t)(cfp[i + 1] - cfp[i]);
        c->nface.upload(nf, s);
    }
    c->vol.alloc(N);
    c->cen.alloc(3 * N);
    c->mom2.alloc(6 * N);
    c->fngp.alloc(F);
    c->gpx.alloc(12 * F);
    c->gpw.alloc(4 * F);
    c->gpn.alloc(12 * F);
    c->farea.alloc(F);
    c->favec.alloc(3 * F);
    c->fmom.alloc(3 * F);
    c->fshift.alloc(3 * F);
    c->slot_nb.alloc(6 * N);
    c->slot_av.alloc(18 * N);
    c->op.alloc(tot > 0 ? tot : 1);
    c->bad.alloc(1);
    const int32_t big = INT32_MAX;
    CGKS_HIP(hipMemcpyAsync(c->bad.p, &big, sizeof(int32_t), hipMemcpyHostToDevice, s));
    const int bs = 128;
    hipLaunchKernelGGL(k_cell_geom, dim3(blocks_for(N, bs)), dim3(bs), 0, s, N, dxyz.p, dhexn.p, c->vol.p, c->cen.p,
                       c->mom2.p);
    hipLaunchKernelGGL(k_face_geom, dim3(blocks_for(F, bs)), dim3(bs), 0, s, F, N, dxyz.p, dfnode.p, c->fl.p, c->cen.p,
                       dfsh.p, c->fngp.p, c->gpx.p, c->gpw.p, c->gpn.p, c->farea.p, c->favec.p, c->fmom.p,
                       c->fshift.p);
    c->lidx.alloc(c->NL);
    c->lgeo.alloc(10 * c->NL);
    hipLaunchKernelGGL(k_lane_geom, dim3(blocks_for(c->NL, bs)), dim3(bs), 0, s, c->NL, F, N, c->lmap.p, c->gpx.p,
                       c->gpn.p, c->gpw.p, c->fshift.p, c->cen.p, c->fl.p, c->fr.p, c->ftag.p, c->fngp.p, c->lidx.p,
                       c->lgeo.p);
    hipLaunchKernelGGL(k_slots, dim3(blocks_for(N, bs)), dim3(bs), 0, s, N, F, c->cf_ptr.p, c->cf_face.p, c->fl.p,
                       c->fr.p, c->favec.p, c->vol.p, c->slot_nb.p, c->slot_av.p);
    c->iav.alloc(18 * N);
    c->bgq.alloc(5 * (F > Fi ? F - Fi : 1));
    hipLaunchKernelGGL(k_iav, dim3(blocks_for(N, bs)), dim3(bs), 0, s, N, c->slot_nb.p, c->slot_av.p, c->iav.p);
    hipLaunchKernelGGL(k_op_build, dim3(blocks_for(N, 64)), dim3(64), 0, s, N, F, c->cf_ptr.p, c->cf_face.p, c->fl.p,
                       c->fr.p, c->fshift.p, c->vol.p, c->cen.p, c->mom2.p, c->op_off.p, c->op.p, c->bad.p);
    CGKS_HIP(hipGetLastError());
    int32_t hb = 0;
    CGKS_HIP(hipMemcpyAsync(&hb, c->bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CGKS_HIP(hipStreamSynchronize(s));
    if (hb != INT32_MAX)
        throw Error{CGKS_E_MESH, "singular reconstruction stencil at cell " + std::to_string(c->caller_cell(hb))};
    // negative volumes are a mesh error
    std::vector<double> hv = c->vol.download(N, s);
    for (int64_t i = 0; i < N; ++i)
        if (!(hv[i] > 0)) throw Error{CGKS_E_MESH, "cell " + std::to_string(c->caller_cell(i)) + ": non-positive volume"};
    // work buffers
    c->coef.alloc(50 * N);
    c->dtc.alloc(N);
    c->fout.alloc(41 * F);
    c->Rw.alloc(5 * N);
    c->Gw.alloc(15 * N);
    c->aw.alloc(N);
    c->Ws.alloc(5 * N);
    c->Gs.alloc(15 * N);
    c->L1.alloc(5 * N);
    c->Lt1.alloc(5 * N);
    c->Gc1.alloc(15 * N);
    c->partial.alloc(4096);
    c->scal.alloc(16);
    c->has_mesh = true;
}

}  // namespace cgks
