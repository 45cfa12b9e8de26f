// Boundary ghost states for the fine Gauss points and the coarse cell averages.
#pragma once
#include "common.hpp"
#include "gks_device.hpp"

namespace cgks {

// Readings: slip = mirror across the face plane; adiabatic no-slip = density and
// energy kept, momentum reversed (momentum field x -> -m(Rx)); far field =
// one-dimensional Riemann invariants along the outward normal, zero gradients.
// Templated on the state type so the adjoint can differentiate through it; n and gamma are data.
template <class T>
__device__ inline void ghost_state(const BcTable &bc, int tag, const double n[3], const T wi[5], double gam, T wg[5])
{
    const int kind = bc.kind[tag & 63];
    if (kind == CGKS_BC_SLIP) {
        const T mn = wi[1] * n[0] + wi[2] * n[1] + wi[3] * n[2];
        wg[0] = wi[0];
        wg[1] = wi[1] - 2.0 * mn * n[0];
        wg[2] = wi[2] - 2.0 * mn * n[1];
        wg[3] = wi[3] - 2.0 * mn * n[2];
        wg[4] = wi[4];
        return;
    }
    if (kind == CGKS_BC_NOSLIP_ADIABATIC) {
        wg[0] = wi[0];
        wg[1] = -wi[1];
        wg[2] = -wi[2];
        wg[3] = -wi[3];
        wg[4] = wi[4];
        return;
    }
    const double *pf = bc.prim[tag & 63];
    const T ri = wi[0];
    const T ui[3] = {wi[1] / ri, wi[2] / ri, wi[3] / ri};
    const T pi = (gam - 1.0) * (wi[4] - 0.5 * ri * (ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2]));
    const T ci = Fp<T>::sqrt_(gam * pi / ri);
    const double cf = sqrt(gam * pf[4] / pf[0]);
    const T uni = ui[0] * n[0] + ui[1] * n[1] + ui[2] * n[2];
    const double unf = pf[1] * n[0] + pf[2] * n[1] + pf[3] * n[2];
    T rb, pb, ub[3];
    if (abs_(uni) >= ci) {
        const bool out = uni >= 0.0;
        rb = out ? ri : T(pf[0]);
        pb = out ? pi : T(pf[4]);
        for (int d = 0; d < 3; ++d) ub[d] = out ? ui[d] : T(pf[1 + d]);
    } else {
        const T rp = uni + 2.0 * ci / (gam - 1.0);
        const T rm = T(unf - 2.0 * cf / (gam - 1.0));
        const T unb = 0.5 * (rp + rm);
        const T cb = 0.25 * (gam - 1.0) * (rp - rm);
        const bool out = unb >= 0.0;
        const T ent = out ? pi / powc_(ri, gam) : T(pf[4] / pow(pf[0], gam));
        for (int d = 0; d < 3; ++d) ub[d] = (out ? ui[d] - uni * n[d] : T(pf[1 + d] - unf * n[d])) + unb * n[d];
        rb = powc_(cb * cb / (gam * ent), 1.0 / (gam - 1.0));
        pb = rb * cb * cb / gam;
    }
    wg[0] = rb;
    wg[1] = rb * ub[0];
    wg[2] = rb * ub[1];
    wg[3] = rb * ub[2];
    wg[4] = pb / (gam - 1.0) + 0.5 * rb * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
}

// G[3c+d] = dW_c/dx_d
template <class T>
__device__ inline void ghost_grad(const BcTable &bc, int tag, const double n[3], const T gi[15], T gg[15])
{
    const int kind = bc.kind[tag & 63];
    if (kind == CGKS_BC_FARFIELD) {
#pragma unroll
        for (int q = 0; q < 15; ++q) gg[q] = T(0.0);
        return;
    }
    // mirrored direction derivative: R v = v - 2 (v.n) n
#pragma unroll
    for (int c = 0; c < 5; c += 4) {
        const T dn = gi[3 * c] * n[0] + gi[3 * c + 1] * n[1] + gi[3 * c + 2] * n[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[3 * c + d] = gi[3 * c + d] - 2.0 * dn * n[d];
    }
    // momentum gradient M_ij = dm_i/dx_j: slip R M R, no-slip -M R
    T MR[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T rn = gi[3 * (1 + i)] * n[0] + gi[3 * (1 + i) + 1] * n[1] + gi[3 * (1 + i) + 2] * n[2];
#pragma unroll
        for (int j = 0; j < 3; ++j) MR[i][j] = gi[3 * (1 + i) + j] - 2.0 * rn * n[j];
    }
    if (kind == CGKS_BC_SLIP) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T cn = MR[0][j] * n[0] + MR[1][j] * n[1] + MR[2][j] * n[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) gg[3 * (1 + i) + j] = MR[i][j] - 2.0 * n[i] * cn;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) gg[3 * (1 + i) + j] = -MR[i][j];
    }
}

}  // namespace cgks
