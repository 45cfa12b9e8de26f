// HWENO reconstruction: kernel arguments, operator layout, and a scalar-generic
// per-(cell, component) reconstruction used where derivatives are needed.
//
// Paper Sec. 3: p^2 from the constrained least-squares operator (neighbour
// averages exact, neighbour gradients in least squares), p^1 by Green-Gauss
// scaled with the previous compression factor, smoothness indicators beta_1
// (min of the Green-Gauss and linear least-squares gradients) and beta_2,
// nonlinear weights, R = w2 (p2 - g1 p1)/g2 + w1 p1.
#pragma once
#include "common.hpp"
#include "gks_device.hpp"
#include "bc_device.hpp"

namespace cgks {

struct ReconArgs {
    int64_t N, F;
    double gam, weno_eps, g2;
    const double *W, *G, *alpha, *vol, *mom2, *slot_av, *op;
    const int32_t *slot_nb, *ftag;
    const int64_t *op_off;
    const BcTable *bc;
    const int64_t *gbase;   // per 64-cell group: first operator entry
    const int32_t *gnb;     // per group: largest interior-neighbour count of its p^2 cells
    const int32_t *gmax;    // per group: largest interior-neighbour count of all its cells
    const int32_t *inb;     // [6][N] interior neighbours in slot order (-1 past the last)
    const double *iav;      // [6*3][N] outward area vector / |Omega| of those faces
    const uint8_t *n_int;   // [N] interior neighbours
    const uint8_t *nface;   // [N] faces
    const double *bgq;      // [5][Fb] ghost states of the boundary faces at W (face ids Fi..F-1)
    int64_t Fi, Fb;
    double *coef;
    const float *opf;  // FP32 copy of op (FP32 storage instantiation)
    float *coeff;      // FP32 cell-major coefficients (FP32 storage instantiation)
};

// Operator entries of one interior neighbour m of a cell, 39 per neighbour: 9 multiply the
// average difference, 27 the neighbour gradient (row k, direction d at 9 + 3k + d), 3 the
// linear least-squares gradient (36 + d).  Cells are interleaved in groups of 64, so entry
// e of cell i sits at op_off[i] + 64 e and a wave reads each entry with one coalesced load.
constexpr int OP_PER_NB = 39;
constexpr int OP_GROUP = 64;

// Inputs of the reconstruction of component C of one cell, by position:
//   0..4   own averages of all five components (the boundary ghosts couple them),
//   5      own compression factor of the previous update,
//   6+4s   average of component C of the interior neighbour in slot s,
//   7+4s.. its three gradient components (x, y, z).
constexpr int RECON_IN = 30;

// The same arithmetic as the reconstruction kernel, in the scalar type T (double
// or a dual number); the inputs come in as values, the mesh data from A.
template <class T, int C>
__device__ inline void recon_generic(const ReconArgs &A, int64_t i, const T w0[5], T al, const T nbw[6],
                                     const T nbg[6][3], T r[10])
{
    const int64_t N = A.N;
    const T q0 = w0[C];
    const int64_t off = A.op_off[i];
    T gg[3] = {T(0.0), T(0.0), T(0.0)}, gl[3] = {T(0.0), T(0.0), T(0.0)}, a[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = T(0.0);
    int m = 0;
    for (int s = 0; s < 6; ++s) {
        const int nbv = A.slot_nb[s * N + i];
        if (nbv == INT32_MIN) break;
        const double av[3] = {A.slot_av[(3 * s) * N + i], A.slot_av[(3 * s + 1) * N + i], A.slot_av[(3 * s + 2) * N + i]};
        T qm;
        if (nbv >= 0) {
            qm = nbw[s];
            if (off >= 0) {
                const double *op = A.op + off + (int64_t)OP_GROUP * OP_PER_NB * m;
                const T e = qm - q0;
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    a[k] += op[OP_GROUP * k] * e + op[OP_GROUP * (9 + 3 * k)] * nbg[s][0] +
                            op[OP_GROUP * (10 + 3 * k)] * nbg[s][1] + op[OP_GROUP * (11 + 3 * k)] * nbg[s][2];
#pragma unroll
                for (int d = 0; d < 3; ++d) gl[d] += op[OP_GROUP * (36 + d)] * e;
            }
            ++m;
        } else {
            const int f = -nbv - 1;
            const double na = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
            const double n[3] = {av[0] / na, av[1] / na, av[2] / na};
            T Qg[5];
            ghost_state(*A.bc, A.ftag[f], n, w0, A.gam, Qg);
            qm = Qg[C];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[d] += 0.5 * (qm + q0) * av[d];
    }
    const T p1x = al * gg[0], p1y = al * gg[1], p1z = al * gg[2];
    if (off < 0) {
        r[0] = q0;
        r[1] = p1x;
        r[2] = p1y;
        r[3] = p1z;
#pragma unroll
        for (int k = 4; k < 10; ++k) r[k] = T(0.0);
        return;
    }
    const double V = A.vol[i];
    const double V13 = cbrt(V), V23 = V13 * V13;
    double I[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) I[q] = A.mom2[q * N + i];
    const double g2 = A.g2, g1 = 1.0 - A.g2;
    const T bgg = V23 * (p1x * p1x + p1y * p1y + p1z * p1z);
    const T bls = V23 * (gl[0] * gl[0] + gl[1] * gl[1] + gl[2] * gl[2]);
    const T b1 = bgg <= bls ? bgg : bls;
    const T hx[3] = {2.0 * a[3], a[6], a[8]};
    const T hy[3] = {a[6], 2.0 * a[4], a[7]};
    const T hz[3] = {a[8], a[7], 2.0 * a[5]};
    const T *hh[3] = {hx, hy, hz};
    T first = T(0.0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T *h = hh[d];
        first += a[d] * a[d] * V + h[0] * h[0] * I[0] + h[1] * h[1] * I[1] + h[2] * h[2] * I[2] +
                 2.0 * (h[0] * h[1] * I[3] + h[1] * h[2] * I[4] + h[0] * h[2] * I[5]);
    }
    const T second = 4.0 * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]) + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
    const T b2 = first / V13 + second * V * V13;
    const T den = q0 * q0 + b1 + 1e-40;
    const T t1 = b1 / den, t2 = b2 / den;
    const T sg = abs_(t2 - t1);
    const T r1 = sg / (A.weno_eps + t1), r2 = sg / (A.weno_eps + t2);
    T w1 = g1 * (1.0 + r1 * r1), w2 = g2 * (1.0 + r2 * r2);
    const T ws = 1.0 / (w1 + w2);
    w1 *= ws;
    w2 *= ws;
    const T c2 = w2 / g2, c1 = w1 - w2 * g1 / g2;
    T rr0 = q0;
#pragma unroll
    for (int k = 3; k < 9; ++k) rr0 -= a[k] * I[k - 3] / V;
    r[0] = c2 * rr0 + c1 * q0;
    r[1] = c2 * a[0] + c1 * p1x;
    r[2] = c2 * a[1] + c1 * p1y;
    r[3] = c2 * a[2] + c1 * p1z;
#pragma unroll
    for (int k = 3; k < 9; ++k) r[1 + k] = c2 * a[k];
}

}  // namespace cgks
