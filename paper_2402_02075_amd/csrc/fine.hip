// Fine-level CGKS kernels: local time step, HWENO reconstruction, BGK flux at
// face Gauss points, deterministic cell gathers and the residual norm.
//
// Paper: Sec. 2.2 (semi-discrete finite volume, Eq. semidiscrete), Sec. 2.3
// (Eq. 2nd-flux), Sec. 2.4 (Eq. gauss-formula), Sec. 3 (HWENO, compression
// factor, WENO weights), Sec. 4.2 (Eq. smo), local time stepping (Secs. 1, 4.3).
//
// Data layout (HBM): per-cell states and geometry are structure-of-arrays,
// component-major, so consecutive lanes touch consecutive addresses; the
// polynomial coefficients are cell-major (50 per cell, read by the Gauss-point
// lanes) and the face records face-major (read by both cells' gathers).  Faces are
// ordered by (left cell, right cell), cells keep the caller's order, and each
// cell gathers its faces through a CSR list in a fixed order: sums are
// deterministic without atomics.
#include "common.hpp"
#include "gks_device.hpp"
#include "bc_device.hpp"
#include "recon_ops.hpp"

namespace cgks {

// ---------------------------------------------------------------- local time step
__device__ __forceinline__ void local_dt_one(int64_t i, int64_t N, int64_t F, double gam, double cfl, double mu,
                                             int viscous, const double *__restrict__ W,
                                             const int32_t *__restrict__ cf_ptr, const int32_t *__restrict__ cf_face,
                                             const double *__restrict__ favec, const double *__restrict__ farea,
                                             const double *__restrict__ vol, double *__restrict__ dt)
{
    const double rho = W[i], ir = 1.0 / rho;
    const double u = W[N + i] * ir, v = W[2 * N + i] * ir, w = W[3 * N + i] * ir;
    const double p = (gam - 1.0) * (W[4 * N + i] - 0.5 * rho * (u * u + v * v + w * w));
    const double cs = sqrt(gam * p * ir);
    const double V = vol[i];
    double sum = 0.0;
    for (int k = cf_ptr[i]; k < cf_ptr[i + 1]; ++k) {
        const int f = cf_face[k] >> 1;
        const double ax = favec[f], ay = favec[F + f], az = favec[2 * F + f];
        const double S = farea[f];
        const double un = fabs(u * ax + v * ay + w * az) / sqrt(ax * ax + ay * ay + az * az);
        const double lam = un + cs + (viscous ? 2.0 * mu * S / (rho * V) : 0.0);
        sum += lam * S;
    }
    dt[i] = cfl * V / sum;
}

__global__ void k_local_dt(int64_t N, int64_t F, double gam, double cfl, double mu, int viscous,
                           const double *__restrict__ W, const int32_t *__restrict__ cf_ptr,
                           const int32_t *__restrict__ cf_face, const double *__restrict__ favec,
                           const double *__restrict__ farea, const double *__restrict__ vol, double *__restrict__ dt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    local_dt_one(i, N, F, gam, cfl, mu, viscous, W, cf_ptr, cf_face, favec, farea, vol, dt);
}

// ---------------------------------------------------------------- reconstruction
// One thread per (cell, conservative component): the reconstruction acts on each
// component separately, so a block holds 64 consecutive cells (one operator group) and five
// waves, one per component.  The operator entries of the group's m-th interior neighbours
// (39 x 64 doubles) are staged in LDS once per block and shared by the five waves, so every
// operator byte crosses the memory hierarchy once.

// Ghost state of boundary face Fi + b at the current state, for the reconstruction's
// Green-Gauss term (each face's ghost is computed once, not per component).
__device__ __forceinline__ void bnd_ghost_one(int64_t b, int64_t N, int64_t F, int64_t Fi, const double *__restrict__ W,
                                              const int32_t *__restrict__ fl, const int32_t *__restrict__ ftag,
                                              const double *__restrict__ favec, const BcTable *__restrict__ bc,
                                              double gam, double *__restrict__ bgq)
{
    const int64_t Fb = F - Fi;
    const int64_t f = Fi + b;
    const int o = fl[f];
    const double av[3] = {favec[f], favec[F + f], favec[2 * F + f]};
    const double na = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
    const double n[3] = {av[0] / na, av[1] / na, av[2] / na};
    double Q0[5], Qg[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) Q0[c] = W[c * N + o];
    ghost_state(*bc, ftag[f], n, Q0, gam, Qg);
#pragma unroll
    for (int c = 0; c < 5; ++c) bgq[c * Fb + b] = Qg[c];
}

// One thread per boundary face.
__global__ void k_bnd_ghost(int64_t N, int64_t F, int64_t Fi, const double *__restrict__ W,
                            const int32_t *__restrict__ fl, const int32_t *__restrict__ ftag,
                            const double *__restrict__ favec, const BcTable *__restrict__ bc, double gam,
                            double *__restrict__ bgq)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= F - Fi) return;
    bnd_ghost_one(b, N, F, Fi, W, fl, ftag, favec, bc, gam, bgq);
}

// The local steps of the cells and, in threads N.., the boundary ghost states at the same W
// (both read only W and geometry): one launch before the reconstruction instead of two.
__global__ void k_local_dt_ghost(int64_t N, int64_t F, int64_t Fi, double gam, double cfl, double mu, int viscous,
                                 const double *__restrict__ W, const int32_t *__restrict__ cf_ptr,
                                 const int32_t *__restrict__ cf_face, const double *__restrict__ favec,
                                 const double *__restrict__ farea, const double *__restrict__ vol,
                                 double *__restrict__ dt, const int32_t *__restrict__ fl,
                                 const int32_t *__restrict__ ftag, const BcTable *__restrict__ bc,
                                 double *__restrict__ bgq)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) local_dt_one(t, N, F, gam, cfl, mu, viscous, W, cf_ptr, cf_face, favec, farea, vol, dt);
    else if (t - N < F - Fi) bnd_ghost_one(t - N, N, F, Fi, W, fl, ftag, favec, bc, gam, bgq);
}

// Green-Gauss contribution of a cell's boundary faces to component C, ghost states precomputed.
template <int C>
__device__ __forceinline__ void recon_gg_boundary(const ReconArgs &A, int64_t i, double q0, double gg[3])
{
    const int64_t N = A.N;
    for (int s = 0; s < 6; ++s) {
        const int nbv = A.slot_nb[s * N + i];
        if (nbv == INT32_MIN) break;
        if (nbv >= 0) continue;
        const double av[3] = {A.slot_av[(3 * s) * N + i], A.slot_av[(3 * s + 1) * N + i], A.slot_av[(3 * s + 2) * N + i]};
        const int64_t f = -(int64_t)nbv - 1;
        const double qm = A.bgq[C * A.Fb + (f - A.Fi)];
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[d] += 0.5 * (qm + q0) * av[d];
    }
}

// TS: storage type of the operator entries and of the coefficients written (double, or float in
// the mixed-precision flux phase, which halves the two largest streams); the arithmetic is FP64.
template <class TS> __device__ __forceinline__ const TS *recon_op(const ReconArgs &A);
template <> __device__ __forceinline__ const double *recon_op<double>(const ReconArgs &A) { return A.op; }
template <> __device__ __forceinline__ const float *recon_op<float>(const ReconArgs &A) { return A.opf; }

template <bool CELL_MAJOR, class TS = double> __global__ __launch_bounds__(320) void k_recon(ReconArgs A)
{
    __shared__ TS sop[OP_PER_NB * OP_GROUP];
    const int lane = threadIdx.x & (OP_GROUP - 1);
    const int C = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform over a wave
    const int64_t N = A.N;
    const int64_t i = (int64_t)blockIdx.x * OP_GROUP + lane;
    const bool live = i < N;
    const int64_t ic = live ? i : N - 1;
    const double q0 = A.W[C * N + ic];
    const int64_t off = A.op_off[ic];
    double gg[3] = {0.0, 0.0, 0.0};
    const int nint = A.n_int[ic];
    if (live && nint < A.nface[ic]) {
        switch (C) {
        case 0: recon_gg_boundary<0>(A, i, q0, gg); break;
        case 1: recon_gg_boundary<1>(A, i, q0, gg); break;
        case 2: recon_gg_boundary<2>(A, i, q0, gg); break;
        case 3: recon_gg_boundary<3>(A, i, q0, gg); break;
        default: recon_gg_boundary<4>(A, i, q0, gg); break;
        }
    }
    // interior neighbours one at a time: Green-Gauss term and, for p^2 cells, the operator
    // products with the entries staged in LDS; the neighbour's data are requested before
    // the staging so that both loads are in flight together
    double a[9], gl[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = 0.0;
    const int gnb = A.gnb[blockIdx.x], gmax = A.gmax[blockIdx.x];
    const TS *gop = recon_op<TS>(A) + A.gbase[blockIdx.x];
    int nb_next = (live && nint > 0) ? A.inb[i] : 0;
    for (int m = 0; m < gmax; ++m) {
        const bool use = live && m < nint;
        const int nb = use ? nb_next : 0;
        nb_next = (live && m + 1 < nint) ? A.inb[(m + 1) * N + i] : 0;  // one neighbour ahead
        const double qm = A.W[C * N + nb];
        const double av[3] = {A.iav[(3 * m) * N + ic], A.iav[(3 * m + 1) * N + ic], A.iav[(3 * m + 2) * N + ic]};
        const bool p2 = use && off >= 0;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        if (p2) {
            gx = A.G[(3 * C) * N + nb];
            gy = A.G[(3 * C + 1) * N + nb];
            gz = A.G[(3 * C + 2) * N + nb];
        }
        if (m < gnb) {
            // 2,496 entries over 320 threads in 8-byte units (one double or two floats; group
            // bases are multiples of 64 entries): all loads in flight before the stores
            using U = typename std::conditional<sizeof(TS) == 8, double, float2>::type;
            const U *src = reinterpret_cast<const U *>(gop + (int64_t)OP_GROUP * OP_PER_NB * m);
            U *dst = reinterpret_cast<U *>(sop);
            constexpr int NT = 5 * OP_GROUP, NE = OP_PER_NB * OP_GROUP * (int)sizeof(TS) / 8,
                          NR = (NE + NT - 1) / NT;
            U v[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int t = threadIdx.x + r * NT;
                v[r] = t < NE ? src[t] : U{};
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int t = threadIdx.x + r * NT;
                if (t < NE) dst[t] = v[r];
            }
        }
        __syncthreads();
        if (use) {
#pragma unroll
            for (int d = 0; d < 3; ++d) gg[d] += 0.5 * (qm + q0) * av[d];
        }
        if (p2) {
            const double e = qm - q0;
            const TS *o = sop + lane;
#pragma unroll
            for (int k = 0; k < 9; ++k)
                a[k] += double(o[OP_GROUP * k]) * e + double(o[OP_GROUP * (9 + 3 * k)]) * gx +
                        double(o[OP_GROUP * (10 + 3 * k)]) * gy + double(o[OP_GROUP * (11 + 3 * k)]) * gz;
#pragma unroll
            for (int d = 0; d < 3; ++d) gl[d] += double(o[OP_GROUP * (36 + d)]) * e;
        }
        __syncthreads();
    }
    if (!live) return;
    const double al = A.alpha ? A.alpha[i] : 1.0;
    double r[10];
    const double p1x = al * gg[0], p1y = al * gg[1], p1z = al * gg[2];
    if (off < 0) {
        r[0] = q0;
        r[1] = p1x;
        r[2] = p1y;
        r[3] = p1z;
#pragma unroll
        for (int k = 4; k < 10; ++k) r[k] = 0.0;
    } else {
        const double V = A.vol[i];
        const double V13 = cbrt(V), V23 = V13 * V13;
        double I[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) I[q] = A.mom2[q * N + i];
        const double g2 = A.g2, g1 = 1.0 - A.g2;
        const double bgg = V23 * (p1x * p1x + p1y * p1y + p1z * p1z);
        const double bls = V23 * (gl[0] * gl[0] + gl[1] * gl[1] + gl[2] * gl[2]);
        const double b1 = fmin(bgg, bls);
        // beta_2: first derivatives (linear in dx) squared and integrated, plus constant second derivatives
        const double hx[3] = {2.0 * a[3], a[6], a[8]};
        const double hy[3] = {a[6], 2.0 * a[4], a[7]};
        const double hz[3] = {a[8], a[7], 2.0 * a[5]};
        const double *hh[3] = {hx, hy, hz};
        double first = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double *h = hh[d];
            first += a[d] * a[d] * V + h[0] * h[0] * I[0] + h[1] * h[1] * I[1] + h[2] * h[2] * I[2] +
                     2.0 * (h[0] * h[1] * I[3] + h[1] * h[2] * I[4] + h[0] * h[2] * I[5]);
        }
        const double second = 4.0 * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]) + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
        const double b2 = first / V13 + second * V * V13;
        const double den = q0 * q0 + b1 + 1e-40;
        const double t1 = b1 / den, t2 = b2 / den;
        const double sg = fabs(t2 - t1);
        const double r1 = sg / (A.weno_eps + t1), r2 = sg / (A.weno_eps + t2);
        double w1 = g1 * (1.0 + r1 * r1), w2 = g2 * (1.0 + r2 * r2);
        const double ws = 1.0 / (w1 + w2);
        w1 *= ws;
        w2 *= ws;
        // R = w2 (p2/g2 - g1/g2 p1) + w1 p1
        const double c2 = w2 / g2, c1 = w1 - w2 * g1 / g2;
        double r0 = q0;
#pragma unroll
        for (int k = 3; k < 9; ++k) r0 -= a[k] * I[k - 3] / V;
        r[0] = c2 * r0 + c1 * q0;
        r[1] = c2 * a[0] + c1 * p1x;
        r[2] = c2 * a[1] + c1 * p1y;
        r[3] = c2 * a[2] + c1 * p1z;
#pragma unroll
        for (int k = 3; k < 9; ++k) r[1 + k] = c2 * a[k];
    }
    if constexpr (sizeof(TS) == 4) {
#pragma unroll
        for (int k = 0; k < 10; ++k) A.coeff[i * 50 + 10 * C + k] = float(r[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            if (CELL_MAJOR) A.coef[i * 50 + 10 * C + k] = r[k];
            else A.coef[(10 * C + k) * N + i] = r[k];
        }
    }
}

// ---------------------------------------------------------------- face flux
struct FaceArgs {
    int64_t N, F;
    GksCfg cfg;
    double dt_global;
    const double *coef, *dtc;
    const float *coeff;  // FP32 coefficients (FP32 flux)
    const int4 *lidx;    // per lane {4 f + k, L, R, 8 tag + ngp}, f = -1 idle
    const double *lgeo;  // per lane dx_L, dx_R, n, w S ([10][NL])
    const float *lgeof;  // the same in FP32 (FP32 flux)
    int64_t NL;
    const BcTable *bc;
    double *out;  // [F][nq], face-major
    int32_t *bad;
};

template <class T>
__device__ __forceinline__ void eval_poly(const T *__restrict__ coef, int64_t cell, const T dx[3], T w[5], T g[15])
{
    const T *cc = coef + cell * 50;  // cell-major: 10 coefficients per component
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        T r[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) r[k] = cc[10 * c + k];
        poly_eval(r, dx, w[c], &g[3 * c]);
    }
}

// Sums (products) over the lanes of one face: the face's lanes are consecutive within the
// wave, starting at its first Gauss point's lane; the result is valid on that lane.
__device__ __forceinline__ double face_sum(double v, int ln, int ngp)
{
    const double v1 = __shfl(v, ln + 1, 64), v2 = __shfl(v, ln + 2, 64), v3 = __shfl(v, ln + 3, 64);
    return ((v + v1) + v2) + (ngp == 4 ? v3 : 0.0);
}
__device__ __forceinline__ double face_prod(double v, int ln, int ngp)
{
    const double v1 = __shfl(v, ln + 1, 64), v2 = __shfl(v, ln + 2, 64), v3 = __shfl(v, ln + 3, 64);
    return ((v * v1) * v2) * (ngp == 4 ? v3 : 1.0);
}

// The work of one lane: its face's Gauss point k, given the lane's indices and geometry.
// FOLD: 0 = moment vectors then combination (all modes), 1 = time coefficients folded into the
// moment sums, inviscid, 2 = folded, viscous (steady modes only).
// T is the type of the whole per-point evaluation: polynomials, rotations, flux and compression
// factor (FP32 reads FP32 coefficients and lane geometry); the face sums are FP64.
template <class T> __device__ __forceinline__ const T *face_coef(const FaceArgs &A);
template <> __device__ __forceinline__ const double *face_coef<double>(const FaceArgs &A) { return A.coef; }
template <> __device__ __forceinline__ const float *face_coef<float>(const FaceArgs &A) { return A.coeff; }

template <class T, int MODE, bool VAL, int FOLD>
__device__ __forceinline__ void face_lane(const FaceArgs &A, const int4 id, const T g[10], int ln)
{
    const int64_t N = A.N;
    const bool act = id.x >= 0;
    const int64_t f = id.x >> 2;
    const int k = id.x & 3;
    const int L = id.y, R = id.z;
    const int ngp = id.w & 7;
    constexpr int NQ = MODE == MODE_RES ? 21 : MODE == MODE_RESONLY ? 5 : MODE == MODE_S1 ? 41 : 26;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    double alpha_k = 1.0;
    if (act) {
        const T n[3] = {g[6], g[7], g[8]};
        const double wS = g[9];
        double dtf = A.dt_global;
        if (dtf <= 0.0) dtf = R >= 0 ? fmin(A.dtc[L], A.dtc[R]) : A.dtc[L];
        T WL[5], GL[15], WR[5], GR[15];
        {
            const T dx[3] = {g[0], g[1], g[2]};
            eval_poly<T>(face_coef<T>(A), L, dx, WL, GL);
        }
        if (R >= 0) {
            const T dx[3] = {g[3], g[4], g[5]};
            eval_poly<T>(face_coef<T>(A), R, dx, WR, GR);
        } else {
            const int tag = id.w >> 3;
            const double nd[3] = {n[0], n[1], n[2]};
            ghost_state(*A.bc, tag, nd, WL, A.cfg.gamma, WR);
            ghost_grad(*A.bc, tag, nd, GL, GR);
        }
        T t1[3], t2[3];
        onb(n, t1, t2);
        T wl[5], wr[5], gl[3][5], gr[3][5];
        to_local(WL, GL, n, t1, t2, wl, gl);
        to_local(WR, GR, n, t1, t2, wr, gr);
        if constexpr (FOLD > 0) {
            // steady residual modes: time coefficients folded into the moment sums
            T Fl[5], Wt[5], pl, pr;
            if (!gks_flux_folded<T, MODE == MODE_RES, FOLD == 2>(wl, gl, wr, gr, T(A.cfg.gamma), T(A.cfg.K), T(dtf),
                                                                A.cfg, Fl, Wt, pl, pr)) {
                atomicMin(A.bad, L);
            } else {
                T Fg[5];
                to_global(Fl, n, t1, t2, Fg);
                const double s = wS / dtf;
#pragma unroll
                for (int q = 0; q < 5; ++q) acc[q] = s * double(Fg[q]);
                if (MODE == MODE_RES) {
                    T Wg[5];
                    to_global(Wt, n, t1, t2, Wg);
#pragma unroll
                    for (int q = 0; q < 5; ++q)
#pragma unroll
                        for (int d = 0; d < 3; ++d) acc[5 + 3 * q + d] = wS * double(Wg[q]) * double(n[d]);
                    if (R >= 0) {
                        if constexpr (sizeof(T) == 8) alpha_k = cf_factor(wl, wr, double(pl), double(pr), A.cfg.gamma);
                        else alpha_k = double(cf_factor(wl, wr, pl, pr, T(A.cfg.gamma)));
                    }
                }
            }
        } else {
        GksMoments<T> mo;
        if (!gks_moments<T>(wl, gl, wr, gr, T(A.cfg.gamma), T(A.cfg.K), mo, VAL)) {
            atomicMin(A.bad, L);
        } else {
            T tau, taun;
            collision_times(mo, T(dtf), A.cfg, tau, taun);
            T Fl[5];
            double Fg[5];
            flux_integrated(mo, T(dtf), tau, taun, A.cfg, Fl);
            to_global(Fl, n, t1, t2, Fg);
            if (MODE == MODE_RES || MODE == MODE_RESONLY) {
                const double s = wS / dtf;
#pragma unroll
                for (int q = 0; q < 5; ++q) acc[q] = s * Fg[q];
            } else {
#pragma unroll
                for (int q = 0; q < 5; ++q) acc[q] = wS * Fg[q];
                T Fh[5];
                double Fhg[5];
                flux_integrated(mo, T(0.5 * dtf), tau, taun, A.cfg, Fh);
                to_global(Fh, n, t1, t2, Fhg);
#pragma unroll
                for (int q = 0; q < 5; ++q) acc[5 + q] = wS * Fhg[q];
            }
            if (MODE == MODE_RES) {
                T Wt[5];
                double Wg[5];
                value_at(mo, T(dtf), tau, taun, Wt);
                to_global(Wt, n, t1, t2, Wg);
#pragma unroll
                for (int q = 0; q < 5; ++q)
#pragma unroll
                    for (int d = 0; d < 3; ++d) acc[5 + 3 * q + d] = wS * Wg[q] * n[d];
            } else if (MODE == MODE_S1) {
                T Wt[5];
                double Wg[5], Wc[5];
                value_at(mo, T(0.5 * dtf), tau, taun, Wt);
                to_global(Wt, n, t1, t2, Wg);
                T wc[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) wc[q] = mo.Vc[0][q];
                to_global(wc, n, t1, t2, Wc);
#pragma unroll
                for (int q = 0; q < 5; ++q)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        acc[10 + 3 * q + d] = wS * Wg[q] * n[d];
                        acc[25 + 3 * q + d] = wS * Wc[q] * n[d];
                    }
            } else if (MODE == MODE_S2) {
                T Wt[5];
                double Wg[5];
                value_at(mo, T(dtf), tau, taun, Wt);
#pragma unroll
                for (int q = 0; q < 5; ++q) Wt[q] -= mo.Vc[0][q];
                to_global(Wt, n, t1, t2, Wg);
#pragma unroll
                for (int q = 0; q < 5; ++q)
#pragma unroll
                    for (int d = 0; d < 3; ++d) acc[10 + 3 * q + d] = wS * Wg[q] * n[d];
            }
            if (MODE != MODE_RESONLY && R >= 0)
                alpha_k = cf_factor(wl, wr, double(mo.pl), double(mo.pr), A.cfg.gamma);
        }
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = face_sum(acc[q], ln, ngp);
    if (MODE != MODE_RESONLY) alpha_k = face_prod(alpha_k, ln, ngp);
    // face-major record of NQ values (flux sums, interface-value sums, CF product last)
    if (act && k == 0) {
        double *o = A.out + f * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) o[q] = acc[q];
        if (MODE != MODE_RESONLY) o[NQ - 1] = alpha_k;
    }
}


template <class T, int MODE, bool VAL, int FOLD> __device__ __forceinline__ void face_kernel(const FaceArgs &A)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t NL = A.NL;
    const int4 id = A.lidx[gid];  // the grid covers the padded lane map exactly
    T g[10];
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < 10; ++q) g[q] = A.lgeof[q * NL + gid];
    } else {
#pragma unroll
        for (int q = 0; q < 10; ++q) g[q] = A.lgeo[q * NL + gid];
    }
    face_lane<T, MODE, VAL, FOLD>(A, id, g, (int)(threadIdx.x & 63));
}

// One lane per face Gauss point, faces packed into waves with 3 or 4 lanes each (lane map
// built at set-up), face sums by lane shuffles.  The FP64 instantiations need more than 256
// registers: one wave per SIMD.
template <class T, int MODE, bool VAL, int FOLD = 0> __global__ __launch_bounds__(256) void k_face(FaceArgs A)
{
    face_kernel<T, MODE, VAL, FOLD>(A);
}

// The inviscid residual-only flux held to 256 registers for two waves per SIMD (its natural
// allocation is a little above 256; the few spills cost less than the second wave gains).
template <class T> __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_face_res2(FaceArgs A)
{
    face_kernel<T, MODE_RESONLY, false, 1>(A);
}

// ---------------------------------------------------------------- gathers
struct GatherArgs {
    int64_t N, F;
    const int32_t *cf_ptr, *cf_face;
    const double *fout, *vol;
};

// R = -sum s F, Gn = alpha S/V, alpha = prod; optionally W += dt/V R (FE) and norm partials.
// Four lanes per cell (lane g takes the cell's faces g, g + 4, ...), partial sums and products
// combined in a fixed xor tree: deterministic, and four times the waves of a thread per cell.
constexpr int CG = 4;
__device__ __forceinline__ double cell_sum(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}
__device__ __forceinline__ double cell_prod(double v)
{
    v *= __shfl_xor(v, 1, 64);
    v *= __shfl_xor(v, 2, 64);
    return v;
}

template <bool FE, bool GRAD>
__global__ __launch_bounds__(256) void k_gather(GatherArgs A, double *__restrict__ R, double *__restrict__ Gn,
                                                double *__restrict__ an, double *__restrict__ W,
                                                const double *__restrict__ dt, double *__restrict__ part)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / CG;
    const int g = (int)(t % CG);
    const int64_t N = A.N;
    double r2 = 0.0;
    if (i < N) {  // whole cell groups take the same branch
        // the cell's own inputs, requested before the face loop so that their latency overlaps it
        const double vi = A.vol[i];
        double dti = 0.0, w0[5] = {0, 0, 0, 0, 0};
        if (FE && g == 0) {
            dti = dt[i];
#pragma unroll
            for (int q = 0; q < 5; ++q) w0[q] = W[q * N + i];
        }
        double r[5] = {0, 0, 0, 0, 0};
        double gs[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) gs[q] = 0.0;
        double al = 1.0;
        constexpr int NQ = GRAD ? 21 : 5;
        for (int k = A.cf_ptr[i] + g; k < A.cf_ptr[i + 1]; k += CG) {
            const int it = A.cf_face[k];
            const double *o = A.fout + (int64_t)(it >> 1) * NQ;
            const double s = (it & 1) ? -1.0 : 1.0;
#pragma unroll
            for (int q = 0; q < 5; ++q) r[q] -= s * o[q];
            if (GRAD) {
#pragma unroll
                for (int q = 0; q < 15; ++q) gs[q] += s * o[5 + q];
                al *= o[20];
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) r[q] = cell_sum(r[q]);
        if (GRAD) {
#pragma unroll
            for (int q = 0; q < 15; ++q) gs[q] = cell_sum(gs[q]);
            al = cell_prod(al);
        }
        const double iv = 1.0 / vi;
        if (g == 0) {
#pragma unroll
            for (int q = 0; q < 5; ++q) R[q * N + i] = r[q];
            if (GRAD) {
#pragma unroll
                for (int q = 0; q < 15; ++q) Gn[q * N + i] = al * gs[q] * iv;
                an[i] = al;
            }
            if (FE) {
                const double h = dti * iv;
#pragma unroll
                for (int q = 0; q < 5; ++q) W[q * N + i] = w0[q] + h * r[q];
            }
            const double rr = r[0] * iv;
            r2 = rr * rr;
        }
    }
    if (part) {
        // deterministic block reduction in a fixed tree
        __shared__ double sm[256];
        sm[threadIdx.x] = r2;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
    }
}

__global__ __launch_bounds__(256) void k_gather_s2o4(GatherArgs A, int stage, double dt, double *__restrict__ W,
                                                     double *__restrict__ G, double *__restrict__ alpha,
                                                     double *__restrict__ Ws, double *__restrict__ Gs,
                                                     double *__restrict__ as, double *__restrict__ L1,
                                                     double *__restrict__ Lt1, double *__restrict__ Gc1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = A.N, F = A.F;
    if (i >= N) return;
    double ri[5] = {0, 0, 0, 0, 0}, rh[5] = {0, 0, 0, 0, 0}, g1[15], g2[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) g1[q] = g2[q] = 0.0;
    double al = 1.0;
    const int NQ = stage == 1 ? 41 : 26;
    for (int k = A.cf_ptr[i]; k < A.cf_ptr[i + 1]; ++k) {
        const int it = A.cf_face[k];
        const double *o = A.fout + (int64_t)(it >> 1) * NQ;
        const double s = (it & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            ri[q] -= s * o[q];
            rh[q] -= s * o[5 + q];
        }
#pragma unroll
        for (int q = 0; q < 15; ++q) g1[q] += s * o[10 + q];
        if (stage == 1) {
#pragma unroll
            for (int q = 0; q < 15; ++q) g2[q] += s * o[25 + q];
            al *= o[40];
        } else {
            al *= o[25];
        }
    }
    const double V = A.vol[i], iv = 1.0 / V;
    if (stage == 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double L = (4.0 * rh[q] - ri[q]) / (dt * V);
            const double Lt = 4.0 * (ri[q] - 2.0 * rh[q]) / (dt * dt * V);
            L1[q * N + i] = L;
            Lt1[q * N + i] = Lt;
            Ws[q * N + i] = W[q * N + i] + 0.5 * dt * L + 0.125 * dt * dt * Lt;
        }
#pragma unroll
        for (int q = 0; q < 15; ++q) {
            Gs[q * N + i] = al * g1[q] * iv;
            Gc1[q * N + i] = g2[q] * iv;
        }
        as[i] = al;
    } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double Lt2 = 4.0 * (ri[q] - 2.0 * rh[q]) / (dt * dt * V);
            W[q * N + i] += dt * L1[q * N + i] + dt * dt / 6.0 * (Lt1[q * N + i] + 2.0 * Lt2);
        }
#pragma unroll
        for (int q = 0; q < 15; ++q) G[q * N + i] = al * (Gc1[q * N + i] + g1[q] * iv);
        alpha[i] = al;
    }
}

// ---------------------------------------------------------------- wall force
// One work-group: each thread sums a fixed stride of the boundary faces, then a fixed tree.
__global__ __launch_bounds__(256) void k_wall_force(int64_t f0, int64_t f1, int32_t tag, int nq,
                                                     const int32_t *__restrict__ ftag, const double *__restrict__ fout,
                                                     double *__restrict__ out)
{
    __shared__ double sm[3][256];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t f = f0 + threadIdx.x; f < f1; f += 256)
        if (ftag[f] == tag)
#pragma unroll
            for (int d = 0; d < 3; ++d) acc[d] += fout[f * nq + 1 + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) sm[d][threadIdx.x] = acc[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int d = 0; d < 3; ++d) sm[d][threadIdx.x] += sm[d][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = sm[threadIdx.x][0];
}

void launch_wall_force(cgks_ctx *c, int32_t tag, double *out)
{
    // face records of the last residual-only face launch (5 values per face)
    hipLaunchKernelGGL(k_wall_force, dim3(1), dim3(256), 0, c->stream, c->Fi, c->F, tag, 5, c->ftag.p, c->fout.p, out);
}

// ---------------------------------------------------------------- norm
__global__ __launch_bounds__(256) void k_norm_part(int64_t n, const double *__restrict__ R,
                                                   const double *__restrict__ vol, double *__restrict__ part)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double r = R[i] / vol[i];
        v = r * r;
    }
    __shared__ double sm[256];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_norm_final(int nb, int64_t n, const double *__restrict__ part,
                                                    double *__restrict__ out)
{
    __shared__ double sm[256];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[b];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(sm[0] / (double)n);
}

__global__ void k_fill(double *p, double v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- launchers
GksCfg cfg_of(const cgks_ctx *c)
{
    GksCfg g;
    g.gamma = c->prm.gamma;
    g.K = (5.0 - 3.0 * c->prm.gamma) / (c->prm.gamma - 1.0);
    g.mu = c->prm.mu;
    g.prandtl = c->prm.prandtl;
    g.eps_tau = c->prm.eps_tau;
    g.c_tau = c->prm.c_tau;
    g.viscous = c->prm.viscous;
    return g;
}

void launch_fill(double *p, double v, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
}

void launch_local_dt(cgks_ctx *c, const double *W, double *dt)
{
    hipLaunchKernelGGL(k_local_dt, dim3(blocks_for(c->N, 256)), dim3(256), 0, c->stream, c->N, c->F, c->prm.gamma,
                       c->prm.cfl, c->prm.mu, c->prm.viscous, W, c->cf_ptr.p, c->cf_face.p, c->favec.p, c->farea.p,
                       c->vol.p, dt);
}

void launch_local_dt_recon(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *dt,
                           double *coef, double *bgq, float *coef32)
{
    const int64_t Fb = c->F - c->Fi;
    if (!bgq) bgq = c->bgq.p;
    hipLaunchKernelGGL(k_local_dt_ghost, dim3(blocks_for(c->N + Fb, 256)), dim3(256), 0, c->stream, c->N, c->F, c->Fi,
                       c->prm.gamma, c->prm.cfl, c->prm.mu, c->prm.viscous, W, c->cf_ptr.p, c->cf_face.p, c->favec.p,
                       c->farea.p, c->vol.p, dt, c->fl.p, c->ftag.p, c->bc.p, bgq);
    launch_recon(c, W, G, alpha, coef, true, true, bgq, coef32);
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = float(a[i]);
}

void ensure_fp32_front(cgks_ctx *c)
{
    if (!c->has_mesh || (c->opf.p && c->lgeof.p && c->coeff.p)) return;
    try {
        c->opf.alloc(c->op.n);
        c->lgeof.alloc(10 * c->NL);
        c->coeff.alloc(50 * c->N);
    } catch (...) {  // all three or none
        c->opf.release();
        c->lgeof.release();
        c->coeff.release();
        throw;
    }
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(c->op.n, 256)), dim3(256), 0, c->stream, (int64_t)c->op.n, c->op.p,
                       c->opf.p);
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(10 * c->NL, 256)), dim3(256), 0, c->stream, 10 * c->NL, c->lgeo.p,
                       c->lgeof.p);
    CGKS_HIP(hipGetLastError());
}

void launch_recon(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *coef, bool cell_major,
                  bool ghosts_ready, double *bgq, float *coef32)
{
    if (!bgq) bgq = c->bgq.p;
    ReconArgs A{};
    A.N = c->N;
    A.F = c->F;
    A.gam = c->prm.gamma;
    A.weno_eps = c->prm.weno_eps;
    A.g2 = c->prm.gamma_lin;
    A.W = W;
    A.G = G;
    A.alpha = alpha;
    A.vol = c->vol.p;
    A.mom2 = c->mom2.p;
    A.slot_av = c->slot_av.p;
    A.op = c->op.p;
    A.slot_nb = c->slot_nb.p;
    A.ftag = c->ftag.p;
    A.op_off = c->op_off.p;
    A.bc = c->bc.p;
    A.coef = coef;
    A.opf = c->opf.p;
    A.coeff = coef32;
    A.gbase = c->op_gbase.p;
    A.gnb = c->op_gnb.p;
    A.gmax = c->op_gmax.p;
    A.inb = c->inb.p;
    A.iav = c->iav.p;
    A.n_int = c->n_int.p;
    A.nface = c->nface.p;
    A.Fi = c->Fi;
    A.Fb = c->F - c->Fi;
    A.bgq = bgq;
    if (A.Fb > 0 && !ghosts_ready)
        hipLaunchKernelGGL(k_bnd_ghost, dim3(blocks_for(A.Fb, 256)), dim3(256), 0, c->stream, c->N, c->F, c->Fi, W,
                           c->fl.p, c->ftag.p, c->favec.p, c->bc.p, c->prm.gamma, bgq);
    const dim3 grid(blocks_for(c->N, OP_GROUP)), blk(5 * OP_GROUP);
    if (coef32) {
        if (!c->opf.p) throw Error{CGKS_E_STATE, "FP32 reconstruction without its operator copy"};
        hipLaunchKernelGGL((k_recon<true, float>), grid, blk, 0, c->stream, A);
    } else if (cell_major) {
        hipLaunchKernelGGL((k_recon<true>), grid, blk, 0, c->stream, A);
    } else {
        hipLaunchKernelGGL((k_recon<false>), grid, blk, 0, c->stream, A);
    }
}

void launch_face(cgks_ctx *c, int mode, const double *coef, const double *dt_cell, double dt_global, bool fp32,
                 double *out, const float *coef32)
{
    FaceArgs A;
    A.N = c->N;
    A.F = c->F;
    A.cfg = cfg_of(c);
    A.dt_global = dt_global;
    A.coef = coef;
    A.dtc = dt_cell;
    A.lidx = c->lidx.p;
    A.lgeo = c->lgeo.p;
    A.coeff = coef32 ? coef32 : c->coeff.p;
    A.lgeof = c->lgeof.p;
    if (fp32 && (!c->lgeof.p || !A.coeff)) throw Error{CGKS_E_STATE, "FP32 flux without its FP32 buffers"};
    A.NL = c->NL;
    A.bc = c->bc.p;
    A.out = out ? out : c->fout.p;
    A.bad = c->bad.p;
    const dim3 grid(blocks_for(c->NL, 256)), blk(256);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = c->timing && mode == MODE_RES && !out;
    if (timed) {
        while (c->ev_pool.size() < c->ev_used + 2) {
            hipEvent_t e;
            CGKS_HIP(hipEventCreate(&e));
            c->ev_pool.push_back(e);
        }
        e0 = c->ev_pool[c->ev_used++];
        e1 = c->ev_pool[c->ev_used++];
        CGKS_HIP(hipEventRecord(e0, c->stream));
    }
    // steady modes: time coefficients folded into the moment sums (inviscid: known before the
    // moments; viscous: after a first pass for the interface state)
    const bool inv = !c->prm.viscous;
    if (fp32) {
        switch (mode) {
        case MODE_RES:
            if (inv) hipLaunchKernelGGL((k_face<float, MODE_RES, true, 1>), grid, blk, 0, c->stream, A);
            else hipLaunchKernelGGL((k_face<float, MODE_RES, true, 2>), grid, blk, 0, c->stream, A);
            break;
        case MODE_RESONLY:
            if (inv) hipLaunchKernelGGL((k_face<float, MODE_RESONLY, false, 1>), grid, blk, 0, c->stream, A);
            else hipLaunchKernelGGL((k_face<float, MODE_RESONLY, false, 2>), grid, blk, 0, c->stream, A);
            break;
        default: throw Error{CGKS_E_ARG, "FP32 flux supports the steady modes only"};
        }
    } else {
        switch (mode) {
        case MODE_RES:
            if (inv) hipLaunchKernelGGL((k_face<double, MODE_RES, true, 1>), grid, blk, 0, c->stream, A);
            else hipLaunchKernelGGL((k_face<double, MODE_RES, true, 2>), grid, blk, 0, c->stream, A);
            break;
        case MODE_RESONLY:
            if (inv) hipLaunchKernelGGL((k_face_res2<double>), grid, blk, 0, c->stream, A);
            else hipLaunchKernelGGL((k_face<double, MODE_RESONLY, false, 2>), grid, blk, 0, c->stream, A);
            break;
        case MODE_S1: hipLaunchKernelGGL((k_face<double, MODE_S1, true>), grid, blk, 0, c->stream, A); break;
        default: hipLaunchKernelGGL((k_face<double, MODE_S2, true>), grid, blk, 0, c->stream, A); break;
        }
    }
    if (timed) CGKS_HIP(hipEventRecord(e1, c->stream));
}

static GatherArgs gargs(cgks_ctx *c, const double *fout = nullptr)
{
    GatherArgs g;
    g.N = c->N;
    g.F = c->F;
    g.cf_ptr = c->cf_ptr.p;
    g.cf_face = c->cf_face.p;
    g.fout = fout ? fout : c->fout.p;
    g.vol = c->vol.p;
    return g;
}

int norm_blocks(int64_t n) { return blocks_for(n, 256); }
int gather_blocks(int64_t n) { return blocks_for(CG * n, 256); }

void launch_gather_res(cgks_ctx *c, double *R, double *Gn, double *an, int mode, const double *fout)
{
    const dim3 grid(blocks_for(CG * c->N, 256)), blk(256);
    if (mode == MODE_RES)
        hipLaunchKernelGGL((k_gather<false, true>), grid, blk, 0, c->stream, gargs(c, fout), R, Gn, an, nullptr, nullptr,
                           nullptr);
    else
        hipLaunchKernelGGL((k_gather<false, false>), grid, blk, 0, c->stream, gargs(c, fout), R, nullptr, nullptr,
                           nullptr, nullptr, nullptr);
}

void launch_gather_fe(cgks_ctx *c, double *W, double *G, double *alpha, const double *dt, double *Rout, double *part)
{
    const dim3 grid(blocks_for(CG * c->N, 256)), blk(256);
    hipLaunchKernelGGL((k_gather<true, true>), grid, blk, 0, c->stream, gargs(c), Rout, G, alpha, W, dt, part);
}

void launch_gather_s2o4(cgks_ctx *c, int stage, double dt, double *W, double *G, double *alpha)
{
    const dim3 grid(blocks_for(c->N, 256)), blk(256);
    hipLaunchKernelGGL(k_gather_s2o4, grid, blk, 0, c->stream, gargs(c), stage, dt, W, G, alpha, c->Ws.p, c->Gs.p,
                       c->aw.p, c->L1.p, c->Lt1.p, c->Gc1.p);
}

void launch_norm(cgks_ctx *c, const double *R, const double *vol, int64_t n, double *out)
{
    const int nb = norm_blocks(n);
    c->partial.ensure(nb);
    hipLaunchKernelGGL(k_norm_part, dim3(nb), dim3(256), 0, c->stream, n, R, vol, c->partial.p);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, c->stream, nb, n, c->partial.p, out);
}

void finish_norm(cgks_ctx *c, const double *partials, int nblocks, int64_t n, double *out)
{
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, c->stream, nblocks, n, partials, out);
}

}  // namespace cgks
