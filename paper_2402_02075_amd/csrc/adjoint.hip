// Discrete adjoint of the fine CGKS operator and of the coarse KFVS operator,
// and the adjoint fixed-point iteration through the transposed V-cycle.
//
// Fine operator (Sec. 2.2 Eq. semidiscrete, Sec. 2.3 Eq. 2nd-flux, Sec. 2.4,
// Sec. 3): E(W, G, alpha) = (R, G_new, alpha_new) with the local face step
// dt_f = min(dt_L, dt_R) of the local time steps.  Its linearisation is taken once
// at a state and kept in HBM:
//   * per Gauss-point slot the 11 x 41 Jacobian of (time-averaged flux, interface
//     value W(dt_f), compression factor) with respect to (W_L, dW_L, W_R, dW_R,
//     dt_f), computed exactly with dual numbers (boundary faces differentiate
//     through the ghost state);
//   * per (cell, component) the 10 x 30 Jacobian of the HWENO coefficients with
//     respect to the own averages, the own compression factor and the neighbours'
//     averages and gradients of that component;
//   * per cell the derivative of the local time step with respect to its state.
// A vector-Jacobian product is then a chain of coalesced transposed products and
// deterministic cell gathers (no atomics): record cotangents per face -> Gauss-
// point cotangents -> polynomial coefficients -> reconstruction inputs -> cells.
//
// Coarse operator (Sec. 4.2): first-order KFVS residual on an agglomerated level;
// its face Jacobians are recomputed on the fly with dual numbers (cheap).
//
// Fixed point: one V-cycle U -> Phi(U) at fixed agglomeration (fine smoother with
// local steps, fine residual at the smoothed state, restriction, delta-form coarse
// sweeps with forcing, prolongation).  At a converged state every term that
// multiplies a residual vanishes, and the transposed linearised cycle is
//   X_1 = P_1^T lam_W, X_{l+1} = P_{l+1}^T X_l, Rs_L = (dt/V)_L X_L,
//   t = R_{l+1}^T Rs_{l+1}, D_l = X_l + dK_l^T t, Rs_l = t + (dt/V)_l D_l,
//   lam_r = R_1^T Rs_1, lam_1 = lam + dR^T lam_r,
//   lam' = (lam_1,W, 0, 0) + dE^T((dt/V) lam_1,W, lam_1,G, lam_1,alpha) + dJ/dU,
// iterated to a fixed point; P = injection prolongation, R = summing restriction.
#include <algorithm>
#include <cmath>

#include <memory>

#include "common.hpp"
#include "gks_device.hpp"
#include "dual.hpp"
#include "bc_device.hpp"
#include "recon_ops.hpp"

namespace cgks {

constexpr int GP_IN = 41, GP_OUT = 11;

// The Gauss-point Jacobians are stored in tiles of 64 columns (the compact Gauss points), and
// within a tile in runs of JG = 16 / (entry size) consecutive entries of one column: entry r of
// column s at ((s / 64) JRP + (r / JG) JG) 64 + (s % 64) JG + r % JG, with the 451 entries of a
// column padded to JRP = 452.  The lanes of a wave, which handle consecutive columns, then read
// 16 bytes each per load and stream through one contiguous tile (JRP x 64 entries) instead of 451
// rows far apart (48 to 64 columns per wave would leave short unaligned pieces of each row).  The
// reconstruction Jacobians need no tiles (a wave there covers 64 consecutive columns exactly):
// jr_at below keeps them row-major over the columns, in the same 16-byte runs.
constexpr int JRP = 452;
template <int JG> __host__ __device__ constexpr int64_t jf_at(int64_t s, int64_t r)
{
    return ((s >> 6) * JRP + (r / JG) * JG) * 64 + (s & 63) * JG + (r % JG);
}
__host__ __device__ constexpr size_t jf_size(int64_t n) { return (size_t)((n + 63) >> 6) * 64 * JRP; }
// The reconstruction Jacobians: entry r = 30 o + q of column t = 5 i + c (cell i, component c) at
// ((r / JG) 5N + t) JG + r % JG: row-major over the columns, so that the 64 consecutive columns of
// a wave read one contiguous kilobyte per load, in runs of JG = 16 / (entry size) entries; the
// columns are cell-major, so that the cotangents they produce are cell-major too.
template <int JG> __host__ __device__ constexpr int64_t jr_at(int64_t t, int64_t r, int64_t N5)
{
    return ((r / JG) * N5 + t) * JG + (r % JG);
}
__device__ __forceinline__ void unpack(const float4 &v, float e[4])
{
    e[0] = v.x;
    e[1] = v.y;
    e[2] = v.z;
    e[3] = v.w;
}
__device__ __forceinline__ void unpack(const double2 &v, double e[2])
{
    e[0] = v.x;
    e[1] = v.y;
}
// tangent directions per pass of the Gauss-point Jacobian: one (41 passes) keeps each lane's
// dual numbers to twice the flux's own registers, so a pass spills 2.3 KB per lane; four tangents
// spill 12 KB and eight 18.5 KB, and the whole linearisation takes 2.7 and 4.3 times as long
constexpr int K_FACE = 1;
constexpr int K_RECON = 6;  // tangent directions per pass of the reconstruction Jacobian

static inline dim3 B1(int64_t n, int bs = 256) { return dim3(blocks_for(n > 0 ? n : 1, bs)); }

// ---------------------------------------------------------------- local time step derivative
template <class T>
__device__ inline T local_dt_t(int64_t i, int64_t F, double gam, double cfl, double mu, int viscous, const T w[5],
                               const int32_t *cf_ptr, const int32_t *cf_face, const double *favec, const double *farea,
                               double V)
{
    const T rho = w[0], ir = 1.0 / rho;
    const T u = w[1] * ir, v = w[2] * ir, ww = w[3] * ir;
    const T p = (gam - 1.0) * (w[4] - 0.5 * rho * (u * u + v * v + ww * ww));
    const T cs = Fp<T>::sqrt_(gam * p * ir);
    T sum = T(0.0);
    for (int k = cf_ptr[i]; k < cf_ptr[i + 1]; ++k) {
        const int f = cf_face[k] >> 1;
        const double ax = favec[f], ay = favec[F + f], az = favec[2 * F + f];
        const double S = farea[f];
        const T un = abs_(u * ax + v * ay + ww * az) / sqrt(ax * ax + ay * ay + az * az);
        const T lam = viscous ? un + cs + 2.0 * mu * S / (rho * V) : un + cs;
        sum += lam * S;
    }
    return cfl * V / sum;
}

__global__ void k_dt_jac(int64_t N, int64_t F, double gam, double cfl, double mu, int viscous, const double *W,
                         const int32_t *cf_ptr, const int32_t *cf_face, const double *favec, const double *farea,
                         const double *vol, double *ddt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    Dual<5> w[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        w[c] = Dual<5>(W[c * N + i]);
        w[c].d[c] = 1.0;
    }
    const Dual<5> dt = local_dt_t(i, F, gam, cfl, mu, viscous, w, cf_ptr, cf_face, favec, farea, vol[i]);
#pragma unroll
    for (int c = 0; c < 5; ++c) ddt[c * N + i] = dt.d[c];
}

__global__ void k_dt_side(int64_t F, const int32_t *fl, const int32_t *fr, const double *dt, uint8_t *dtL)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int L = fl[f], R = fr[f];
    dtL[f] = (R < 0 || dt[L] <= dt[R]) ? 1 : 0;
}

// slot of the same face in the neighbour's slot list
__global__ void k_rev_slots(int64_t N, int64_t Fi, const int32_t *cf_ptr, const int32_t *cf_face, const int32_t *fl,
                            const int32_t *fr, int8_t *rev)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = cf_ptr[i], e = cf_ptr[i + 1];
    for (int s = 0; s < 6; ++s) {
        int8_t r = -1;
        if (b + s < e) {
            const int it = cf_face[b + s];
            const int f = it >> 1;
            if (fr[f] >= 0) {
                const int o = (it & 1) ? fl[f] : fr[f];
                for (int k = cf_ptr[o]; k < cf_ptr[o + 1]; ++k)
                    if ((cf_face[k] >> 1) == f && (cf_face[k] & 1) != (it & 1)) r = (int8_t)(k - cf_ptr[o]);
            }
        }
        rev[s * N + i] = r;
    }
}

// ---------------------------------------------------------------- Gauss-point outputs
struct GpArgs {
    int64_t N, F, NGP;
    GksCfg cfg;
    const double *coef, *dt, *cen, *gpx, *gpw, *gpn, *fshift;
    const uint8_t *dtL;
    const int32_t *fl, *fr, *ftag, *fngp, *gpoff;
    const BcTable *bc;
    double *Jf, *agp;  // Jf: 11*41 per compact Gauss point (jf_at<2>) in FP64, or
    float *Jf32;       // the same in FP32 (jf_at<4>; when not null)
    int32_t *bad;
};

// Outputs of one Gauss point in the global frame: time-averaged flux (5), interface value
// W(dt_f) (5), compression factor (1); the same arithmetic as the face kernel.
template <class T>
__device__ inline bool gp_outputs(const GpArgs &A, int f, int R, const double n[3], const T WL[5], const T GL[15],
                                  const T WRi[5], const T GRi[15], const T &dtf, T out[GP_OUT])
{
    T WR[5], GR[15];
    if (R >= 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) WR[q] = WRi[q];
#pragma unroll
        for (int q = 0; q < 15; ++q) GR[q] = GRi[q];
    } else {
        const int tag = A.ftag[f];
        ghost_state(*A.bc, tag, n, WL, A.cfg.gamma, WR);
        ghost_grad(*A.bc, tag, n, GL, GR);
    }
    double t1[3], t2[3];
    onb(n, t1, t2);
    T wl[5], wr[5], gl[3][5], gr[3][5];
    to_local(WL, GL, n, t1, t2, wl, gl);
    to_local(WR, GR, n, t1, t2, wr, gr);
    GksMoments<T> mo;
    if (!gks_moments<T>(wl, gl, wr, gr, T(A.cfg.gamma), T(A.cfg.K), mo, true)) return false;
    T tau, taun;
    collision_times(mo, dtf, A.cfg, tau, taun);
    T Fl[5], Fg[5];
    flux_integrated(mo, dtf, tau, taun, A.cfg, Fl);
    to_global(Fl, n, t1, t2, Fg);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = Fg[q] / dtf;
    T Wt[5], Wg[5];
    value_at(mo, dtf, tau, taun, Wt);
    to_global(Wt, n, t1, t2, Wg);
#pragma unroll
    for (int q = 0; q < 5; ++q) out[5 + q] = Wg[q];
    out[10] = R >= 0 ? cf_factor(wl, wr, mo.pl, mo.pr, T(A.cfg.gamma)) : T(1.0);
    return true;
}

__device__ inline void eval_cell(const double *coef, int64_t cell, const double dx[3], double w[5], double g[15])
{
    const double *cc = coef + cell * 50;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double r[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) r[k] = cc[10 * c + k];
        poly_eval(r, dx, w[c], &g[3 * c]);
    }
}

// One lane per Gauss-point slot (4 per face); pass p differentiates along inputs [pK, pK + K).
// Jacobian columns are the compact Gauss-point numbers gpoff[f] + k (3 per triangle, 4 per quad).
template <int K> __global__ __launch_bounds__(64) void k_face_jac(GpArgs A, int pass)
{
    const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t f = gp >> 2;
    const int k = (int)(gp & 3);
    if (f >= A.F || k >= A.fngp[f]) return;
    const int64_t F = A.F, N = A.N, NGP = A.NGP;
    const int64_t col = (int64_t)A.gpoff[f] + k;
    const int L = A.fl[f], R = A.fr[f];
    const double x[3] = {A.gpx[(3 * k) * F + f], A.gpx[(3 * k + 1) * F + f], A.gpx[(3 * k + 2) * F + f]};
    const double n[3] = {A.gpn[(3 * k) * F + f], A.gpn[(3 * k + 1) * F + f], A.gpn[(3 * k + 2) * F + f]};
    const double dtv = A.dtL[f] ? A.dt[L] : A.dt[R];
    double v[GP_IN];
    {
        const double dx[3] = {x[0] - A.cen[L], x[1] - A.cen[N + L], x[2] - A.cen[2 * N + L]};
        eval_cell(A.coef, L, dx, v, v + 5);
    }
    if (R >= 0) {
        const double dx[3] = {x[0] - A.fshift[f] - A.cen[R], x[1] - A.fshift[F + f] - A.cen[N + R],
                              x[2] - A.fshift[2 * F + f] - A.cen[2 * N + R]};
        eval_cell(A.coef, R, dx, v + 20, v + 25);
    } else {
#pragma unroll
        for (int q = 20; q < 40; ++q) v[q] = 0.0;
    }
    v[40] = dtv;
    using D = Dual<K>;
    D in[GP_IN];
#pragma unroll
    for (int q = 0; q < GP_IN; ++q) {
        in[q] = D(v[q]);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (q == pass * K + j) in[q].d[j] = 1.0;
    }
    D out[GP_OUT];
    const bool ok = gp_outputs(A, (int)f, R, n, in, in + 5, in + 20, in + 25, in[40], out);
    if (!ok) atomicMin(A.bad, L);
#pragma unroll
    for (int o = 0; o < GP_OUT; ++o)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int q = pass * K + j;
            if (q < GP_IN) {
                const double v = ok ? out[o].d[j] : 0.0;
                const int r = o * GP_IN + q;
                if (A.Jf32) A.Jf32[jf_at<4>(col, r)] = (float)v;
                else A.Jf[jf_at<2>(col, r)] = v;
            }
        }
    if (pass == 0) A.agp[gp] = ok ? out[10].v : 1.0;
}

// ---------------------------------------------------------------- face VJP
struct FvArgs {
    int64_t N, F, NGP;
    const double *cen, *gpx, *gpw, *gpn, *fshift, *agp, *brec;
    const int32_t *fl, *fr, *fngp, *gpoff;
    double *bface;  // [F][101]: coefficient cotangents of L (50) and R (50), face step (1)
};

__device__ __forceinline__ double sum4(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}

// cotangent of R(x) = sum_k r_k phi_k(dx) from cotangents of its value (bw) and gradient (bg)
__device__ __forceinline__ void poly_vjp(const double dx[3], double bw, const double bg[3], double b[10])
{
    const double x = dx[0], y = dx[1], z = dx[2];
    b[0] += bw;
    b[1] += bw * x + bg[0];
    b[2] += bw * y + bg[1];
    b[3] += bw * z + bg[2];
    b[4] += bw * x * x + 2.0 * x * bg[0];
    b[5] += bw * y * y + 2.0 * y * bg[1];
    b[6] += bw * z * z + 2.0 * z * bg[2];
    b[7] += bw * x * y + y * bg[0] + x * bg[1];
    b[8] += bw * y * z + z * bg[1] + y * bg[2];
    b[9] += bw * x * z + z * bg[0] + x * bg[2];
}

// TJ: the Jacobians' storage type (double or float); the products accumulate in FP64
template <class TJ> __global__ __launch_bounds__(256) void k_face_vjp(FvArgs A, const TJ *Jf)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t f = gid >> 2;
    const int k = (int)(gid & 3);
    if (f >= A.F) return;  // whole groups of four leave together
    const int64_t F = A.F, N = A.N, NGP = A.NGP;
    const bool act = k < A.fngp[f];
    const int L = A.fl[f], R = A.fr[f];
    const double *br = A.brec + f * 21;
    const double a = act ? A.agp[gid] : 1.0;
    const double others = __shfl_xor(a, 1, 64) * __shfl_xor(a, 2, 64) * __shfl_xor(a, 3, 64);
    // Gauss-point input cotangents = J^T (output cotangents); zero on idle lanes
    double bi[GP_IN];
    double dxl[3] = {0.0, 0.0, 0.0}, dxr[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < GP_IN; ++q) bi[q] = 0.0;
    if (act) {
        const double wS = A.gpw[k * F + f];
        const double x[3] = {A.gpx[(3 * k) * F + f], A.gpx[(3 * k + 1) * F + f], A.gpx[(3 * k + 2) * F + f]};
        const double n[3] = {A.gpn[(3 * k) * F + f], A.gpn[(3 * k + 1) * F + f], A.gpn[(3 * k + 2) * F + f]};
        double bo[GP_OUT];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            bo[q] = wS * br[q];
            bo[5 + q] = wS * (n[0] * br[5 + 3 * q] + n[1] * br[6 + 3 * q] + n[2] * br[7 + 3 * q]);
        }
        bo[10] = br[20] * others;
        // the column's entries in memory order, 16 bytes per load, about 20 entries in flight at a
        // time, not all 451 (keeps the wave count up); each bi[q] still sums over o in order
        constexpr int JG = 16 / sizeof(TJ);
        using V = typename std::conditional<sizeof(TJ) == 4, float4, double2>::type;
        const V *J = reinterpret_cast<const V *>(Jf + jf_at<JG>((int64_t)A.gpoff[f] + k, 0));
        constexpr int NG = (GP_OUT * GP_IN + JG - 1) / JG, BATCH = 20 / JG;
#pragma unroll
        for (int g0 = 0; g0 < NG; g0 += BATCH) {
#pragma unroll
            for (int g = g0; g < g0 + BATCH && g < NG; ++g) {
                TJ e[JG];
                unpack(J[g * 64], e);
#pragma unroll
                for (int t = 0; t < JG; ++t) {
                    const int r = g * JG + t;
                    if (r < GP_OUT * GP_IN) bi[r % GP_IN] += (double)e[t] * bo[r / GP_IN];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) dxl[d] = x[d] - A.cen[d * N + L];
        if (R >= 0)
#pragma unroll
            for (int d = 0; d < 3; ++d) dxr[d] = x[d] - A.fshift[d * F + f] - A.cen[d * N + R];
    }
    // polynomial transpose one component at a time (10 live sums), face sums by shuffles
    double *o = A.bface + f * 101;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double *dx = side == 0 ? dxl : dxr;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            double b[10];
#pragma unroll
            for (int j = 0; j < 10; ++j) b[j] = 0.0;
            poly_vjp(dx, bi[20 * side + c], bi + 20 * side + 5 + 3 * c, b);
#pragma unroll
            for (int j = 0; j < 10; ++j) {
                const double v = sum4(b[j]);
                if (k == 0) o[50 * side + 10 * c + j] = v;
            }
        }
    }
    const double bdt = sum4(bi[40]);
    if (k == 0) o[100] = bdt;
}

// per (component, cell): the component's 10 coefficient cotangents from the cell's faces, CSR
// order; the density threads also collect the time-step cotangent
__global__ __launch_bounds__(256) void k_coef_gather(int64_t N, const int32_t *cf_ptr, const int32_t *cf_face,
                                                     const int32_t *fr, const uint8_t *dtL, const double *bface,
                                                     double *bcoef, double *bdt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 5 * N) return;
    const int64_t i = t / 5;  // the five component threads of a cell are neighbouring lanes
    const int c = (int)(t - 5 * i);
    double b[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) b[j] = 0.0;
    double tt = 0.0;
    for (int k = cf_ptr[i]; k < cf_ptr[i + 1]; ++k) {
        const int it = cf_face[k];
        const int f = it >> 1;
        const bool isR = it & 1;
        const double *o = bface + (int64_t)f * 101 + (isR ? 50 : 0) + 10 * c;
#pragma unroll
        for (int j = 0; j < 10; ++j) b[j] += o[j];
        if (c == 0) {
            const bool fromL = fr[f] < 0 || dtL[f];
            if (isR != fromL) tt += bface[(int64_t)f * 101 + 100];
        }
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) bcoef[i * 50 + 10 * c + j] = b[j];
    if (c == 0) bdt[i] = tt;
}

// ---------------------------------------------------------------- reconstruction Jacobian and VJP
template <int K, int C, class TJ> __device__ __forceinline__ void recon_jac_comp(const ReconArgs &A, int64_t i, int pass, TJ *Jr)
{
    const int64_t N = A.N;
    using D = Dual<K>;
    double v[RECON_IN];
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = A.W[c * N + i];
    v[5] = A.alpha ? A.alpha[i] : 1.0;
    for (int s = 0; s < 6; ++s) {
        const int nbv = A.slot_nb[s * N + i];
        const bool in = nbv >= 0;
        v[6 + 4 * s] = in ? A.W[C * N + nbv] : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) v[7 + 4 * s + d] = in ? A.G[(3 * C + d) * N + nbv] : 0.0;
    }
    D x[RECON_IN];
#pragma unroll
    for (int q = 0; q < RECON_IN; ++q) {
        x[q] = D(v[q]);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (q == pass * K + j) x[q].d[j] = 1.0;
    }
    D nbw[6], nbg[6][3];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        nbw[s] = x[6 + 4 * s];
#pragma unroll
        for (int d = 0; d < 3; ++d) nbg[s][d] = x[7 + 4 * s + d];
    }
    D r[10];
    recon_generic<D, C>(A, i, x, x[5], nbw, nbg, r);
#pragma unroll
    for (int o = 0; o < 10; ++o)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int q = pass * K + j;
            if (q < RECON_IN) Jr[jr_at<16 / sizeof(TJ)>(5 * i + C, o * RECON_IN + q, 5 * N)] = (TJ)r[o].d[j];
        }
}

template <int K, class TJ> __global__ __launch_bounds__(320) void k_recon_jac(ReconArgs A, int pass, TJ *Jr)
{
    const int64_t i = (int64_t)blockIdx.x * OP_GROUP + (threadIdx.x & (OP_GROUP - 1));
    if (i >= A.N) return;
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: recon_jac_comp<K, 0, TJ>(A, i, pass, Jr); break;
    case 1: recon_jac_comp<K, 1, TJ>(A, i, pass, Jr); break;
    case 2: recon_jac_comp<K, 2, TJ>(A, i, pass, Jr); break;
    case 3: recon_jac_comp<K, 3, TJ>(A, i, pass, Jr); break;
    default: recon_jac_comp<K, 4, TJ>(A, i, pass, Jr); break;
    }
}

// per (cell, component): input cotangents = Jr^T (coefficient cotangents).  Outputs cell-major:
// bown[30 i + 6 c + q] (own state, compression factor), bslot[120 i + 20 s + 4 c + d] (value and
// gradient of the neighbour in slot s), so that a cell's 20 values for one slot are contiguous
template <class TJ>
__global__ __launch_bounds__(256) void k_recon_vjp(int64_t N, const TJ *Jr, const double *bcoef, double *bown,
                                                   double *bslot)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 5 * N) return;
    const int64_t i = t / 5;  // the five component threads of a cell are neighbouring lanes
    const int C = (int)(t - 5 * i);
    double br[10];
#pragma unroll
    for (int o = 0; o < 10; ++o) br[o] = bcoef[i * 50 + 10 * C + o];
    // the column's entries in memory order, 16 bytes per load, in batches; each s[q] still sums
    // over o in order
    constexpr int JG = 16 / sizeof(TJ), NG = 10 * RECON_IN / JG, BATCH = 32 / JG;
    using V = typename std::conditional<sizeof(TJ) == 4, float4, double2>::type;
    const V *Jv = reinterpret_cast<const V *>(Jr) + t;  // run g at Jv[g 5N]
    double s[RECON_IN];
#pragma unroll
    for (int q = 0; q < RECON_IN; ++q) s[q] = 0.0;
#pragma unroll
    for (int g0 = 0; g0 < NG; g0 += BATCH) {
#pragma unroll
        for (int g = g0; g < g0 + BATCH && g < NG; ++g) {
            TJ e[JG];
            unpack(Jv[(int64_t)g * 5 * N], e);
#pragma unroll
            for (int u = 0; u < JG; ++u) {
                const int r = g * JG + u;
                s[r % RECON_IN] += (double)e[u] * br[r / RECON_IN];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < RECON_IN; ++q) {
        if (q < 6) bown[i * 30 + C * 6 + q] = s[q];
        else bslot[i * 120 + ((q - 6) / 4) * 20 + C * 4 + (q - 6) % 4] = s[q];
    }
}

// per cell: state, gradient and compression-factor cotangents from the own and the
// neighbours' reconstructions and from the local time step
__global__ __launch_bounds__(256) void k_recon_gather(int64_t N, const int32_t *slot_nb, const int8_t *rev,
                                                      const double *bown, const double *bslot, const double *bdt,
                                                      const double *ddt, double *oW, double *oG, double *oA, int acc)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double bw[5], bg[15], ba = 0.0;
    const double t = bdt[j];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double s = 0.0;
#pragma unroll
        for (int C = 0; C < 5; ++C) s += bown[j * 30 + C * 6 + c];
        bw[c] = s + t * ddt[c * N + j];
    }
#pragma unroll
    for (int C = 0; C < 5; ++C) ba += bown[j * 30 + C * 6 + 5];
#pragma unroll
    for (int q = 0; q < 15; ++q) bg[q] = 0.0;
    for (int s = 0; s < 6; ++s) {
        const int nbv = slot_nb[s * N + j];
        if (nbv == INT32_MIN) break;
        if (nbv < 0) continue;
        const int rs = rev[s * N + j];
        if (rs < 0) continue;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const double *b = bslot + (int64_t)nbv * 120 + rs * 20 + c * 4;
            bw[c] += b[0];
#pragma unroll
            for (int d = 0; d < 3; ++d) bg[3 * c + d] += b[1 + d];
        }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) oW[c * N + j] = acc ? oW[c * N + j] + bw[c] : bw[c];
    if (oG)
#pragma unroll
        for (int q = 0; q < 15; ++q) oG[q * N + j] = acc ? oG[q * N + j] + bg[q] : bg[q];
    if (oA) oA[j] = acc ? oA[j] + ba : ba;
}

// ---------------------------------------------------------------- operator outputs -> face records
__global__ void k_bat(int64_t N, const double *bG, const double *bA, const double *Sgv, double *bat)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = bA ? bA[i] : 0.0;
    if (bG)
#pragma unroll
        for (int q = 0; q < 15; ++q) s += bG[q * N + i] * Sgv[q * N + i];
    bat[i] = s;
}

// R_i = -sum s rec_flux, G_new,i = alpha_i / V_i sum s rec_val, alpha_i = prod rec_cf (s = +1 left, -1 right)
__global__ void k_brec(int64_t N, int64_t F, const int32_t *fl, const int32_t *fr, const double *vol,
                       const double *Anew, const double *rec, const double *bR, const double *bG, const double *bat,
                       double *brec)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int L = fl[f], R = fr[f];
    double *o = brec + f * 21;
#pragma unroll
    for (int q = 0; q < 5; ++q) o[q] = (bR ? -bR[q * N + L] + (R >= 0 ? bR[q * N + R] : 0.0) : 0.0);
    if (bG) {
        const double hl = Anew[L] / vol[L], hr = R >= 0 ? Anew[R] / vol[R] : 0.0;
#pragma unroll
        for (int q = 0; q < 15; ++q) o[5 + q] = hl * bG[q * N + L] - (R >= 0 ? hr * bG[q * N + R] : 0.0);
    } else {
#pragma unroll
        for (int q = 0; q < 15; ++q) o[5 + q] = 0.0;
    }
    o[20] = (bat && R >= 0) ? (bat[L] * Anew[L] + bat[R] * Anew[R]) / rec[f * 21 + 20] : 0.0;
}

// objective e . (force on the boundary faces with tag)
__global__ void k_brec_wall(int64_t F, const int32_t *fr, const int32_t *ftag, int32_t tag, double e0, double e1,
                            double e2, double *brec)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double *o = brec + f * 21;
    const bool on = fr[f] < 0 && ftag[f] == tag;
#pragma unroll
    for (int q = 0; q < 21; ++q) o[q] = 0.0;
    if (on) {
        o[1] = e0;
        o[2] = e1;
        o[3] = e2;
    }
}

// ---------------------------------------------------------------- coarse KFVS VJP
struct KvArgs {
    int64_t n, m, nb;
    double gam, K;
    const double *W, *bR, *A, *bA;
    const int32_t *pa, *pb, *bown, *btag;
    const BcTable *bc;
    double *kb;  // [m + nb][10]
};

__global__ __launch_bounds__(128) void k_kfvs_vjp_face(KvArgs A)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = A.m + A.nb;
    if (j >= tot) return;
    using D = Dual<10>;
    double av[3];
    int a, b = -1;
    if (j < A.m) {
        for (int d = 0; d < 3; ++d) av[d] = A.A[d * A.m + j];
        a = A.pa[j];
        b = A.pb[j];
    } else {
        for (int d = 0; d < 3; ++d) av[d] = A.bA[d * A.nb + (j - A.m)];
        a = A.bown[j - A.m];
    }
    double *o = A.kb + j * 10;
    const double S = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
    if (S == 0.0) {
#pragma unroll
        for (int q = 0; q < 10; ++q) o[q] = 0.0;
        return;
    }
    double bff[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) bff[q] = -A.bR[q * A.n + a] + (b >= 0 ? A.bR[q * A.n + b] : 0.0);
    const double n[3] = {av[0] / S, av[1] / S, av[2] / S};
    D wa[5], wb[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        wa[q] = D(A.W[q * A.n + a]);
        wa[q].d[q] = 1.0;
        if (b >= 0) {
            wb[q] = D(A.W[q * A.n + b]);
            wb[q].d[5 + q] = 1.0;
        }
    }
    if (b < 0) ghost_state(*A.bc, A.btag[j - A.m], n, wa, A.gam, wb);
    double t1[3], t2[3];
    onb(n, t1, t2);
    D la[5], lb[5];
    la[0] = wa[0];
    la[1] = wa[1] * n[0] + wa[2] * n[1] + wa[3] * n[2];
    la[2] = wa[1] * t1[0] + wa[2] * t1[1] + wa[3] * t1[2];
    la[3] = wa[1] * t2[0] + wa[2] * t2[1] + wa[3] * t2[2];
    la[4] = wa[4];
    lb[0] = wb[0];
    lb[1] = wb[1] * n[0] + wb[2] * n[1] + wb[3] * n[2];
    lb[2] = wb[1] * t1[0] + wb[2] * t1[1] + wb[3] * t1[2];
    lb[3] = wb[1] * t2[0] + wb[2] * t2[1] + wb[3] * t2[2];
    lb[4] = wb[4];
    D Fl[5];
    kfvs_local(la, lb, D(A.gam), D(A.K), Fl);
    D ff[5];
    ff[0] = S * Fl[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) ff[1 + d] = S * (Fl[1] * n[d] + Fl[2] * t1[d] + Fl[3] * t2[d]);
    ff[4] = S * Fl[4];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < 5; ++p) s += ff[p].d[q] * bff[p];
        o[q] = s;
    }
}

__global__ __launch_bounds__(256) void k_kfvs_vjp_gather(int64_t n, int64_t m, const int32_t *ptr, const int32_t *item,
                                                         const double *kb, double *oW, int acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r[5] = {0, 0, 0, 0, 0};
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int it = item[k];
        const double *o = it >= 0 ? kb + (int64_t)(it >> 1) * 10 + ((it & 1) ? 5 : 0) : kb + (m + (-it - 1)) * 10;
#pragma unroll
        for (int q = 0; q < 5; ++q) r[q] += o[q];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) oW[q * n + i] = acc ? oW[q * n + i] + r[q] : r[q];
}

// ---------------------------------------------------------------- transfers and vector helpers
// transpose of the summing restriction: fine cell takes its coarse value
__global__ void k_restrict_t(int64_t nf, int64_t nc, const int32_t *f2c, const double *bc, double *bf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int k = f2c[i];
#pragma unroll
    for (int q = 0; q < 5; ++q) bf[q * nf + i] = bc[q * nc + k];
}

// transpose of the injection prolongation: coarse cell sums its fine members (ascending order)
__global__ void k_prolong_t(int64_t nc, int64_t nf, const int32_t *ptr, const int32_t *idx, const double *bf, double *bc)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    double s[5] = {0, 0, 0, 0, 0};
    for (int q = ptr[k]; q < ptr[k + 1]; ++q) {
        const int i = idx[q];
#pragma unroll
        for (int c = 0; c < 5; ++c) s[c] += bf[c * nf + i];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) bc[c * nc + k] = s[c];
}

// y = x * dt / V per cell (5 components); y may alias x
__global__ void k_scale_dtv(int64_t n, const double *dt, const double *V, const double *x, double *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = dt[i] / V[i];
#pragma unroll
    for (int q = 0; q < 5; ++q) y[q * n + i] = h * x[q * n + i];
}

// y = a + b * dt / V (5 components)
__global__ void k_add_scaled_dtv(int64_t n, const double *dt, const double *V, const double *a, const double *b,
                                 double *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = dt[i] / V[i];
#pragma unroll
    for (int q = 0; q < 5; ++q) y[q * n + i] = a[q * n + i] + h * b[q * n + i];
}

__global__ void k_copy(int64_t n, const double *a, double *b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_axpy(int64_t n, double s, const double *a, double *b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] += s * a[i];
}

__global__ void k_div(int64_t n, const double *a, const double *den, int64_t ncol, double *b)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * ncol) b[t] = a[t] / den[t % n];
}

// deterministic partial sums of |a - b|^2 and |a|^2 (fixed tree per block)
__global__ __launch_bounds__(256) void k_diff_part(int64_t n, const double *a, const double *b, double *part)
{
    __shared__ double s1[256], s2[256];
    double x = 0.0, y = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double d = a[i] - b[i];
        x += d * d;
        y += a[i] * a[i];
    }
    s1[threadIdx.x] = x;
    s2[threadIdx.x] = y;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// ---------------------------------------------------------------- host side
static AdjTape &tape(cgks_ctx *c)
{
    if (!c->adj || !c->adj->ready) throw Error{CGKS_E_STATE, "no linearisation: call cgks_linearize first"};
    return *c->adj;
}

static ReconArgs recon_args(cgks_ctx *c, const double *W, const double *G, const double *al)
{
    ReconArgs A{};
    A.N = c->N;
    A.F = c->F;
    A.gam = c->prm.gamma;
    A.weno_eps = c->prm.weno_eps;
    A.g2 = c->prm.gamma_lin;
    A.W = W;
    A.G = G;
    A.alpha = al;
    A.vol = c->vol.p;
    A.mom2 = c->mom2.p;
    A.slot_av = c->slot_av.p;
    A.op = c->op.p;
    A.slot_nb = c->slot_nb.p;
    A.ftag = c->ftag.p;
    A.op_off = c->op_off.p;
    A.bc = c->bc.p;
    A.coef = nullptr;
    return A;
}

void adj_linearize(cgks_ctx *c, const double *W, const double *G, const double *alpha)
{
    if (!c->adj) c->adj = new AdjTape();
    AdjTape &T = *c->adj;
    T.ready = false;
    hipStream_t st = c->stream;
    const int64_t N = c->N, F = c->F, NS = 4 * F, NGP = c->NGP;
    T.W.ensure(5 * N);
    T.G.ensure(15 * N);
    T.al.ensure(N);
    CGKS_HIP(hipMemcpyAsync(T.W.p, W, sizeof(double) * 5 * N, hipMemcpyDeviceToDevice, st));
    CGKS_HIP(hipMemcpyAsync(T.G.p, G, sizeof(double) * 15 * N, hipMemcpyDeviceToDevice, st));
    if (alpha) CGKS_HIP(hipMemcpyAsync(T.al.p, alpha, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    else launch_fill(T.al.p, 1.0, N, st);
    // local steps and their derivatives
    T.dt.ensure(N);
    T.ddt.ensure(5 * N);
    T.dtL.ensure(F);
    launch_local_dt(c, T.W.p, T.dt.p);
    hipLaunchKernelGGL(k_dt_jac, B1(N), dim3(256), 0, st, N, F, c->prm.gamma, c->prm.cfl, c->prm.mu, c->prm.viscous,
                       T.W.p, c->cf_ptr.p, c->cf_face.p, c->favec.p, c->farea.p, c->vol.p, T.ddt.p);
    hipLaunchKernelGGL(k_dt_side, B1(F), dim3(256), 0, st, F, c->fl.p, c->fr.p, T.dt.p, T.dtL.p);
    // primal pass: coefficients, face records, G_new, alpha_new
    T.coef.ensure(50 * N);
    launch_recon(c, T.W.p, T.G.p, T.al.p, T.coef.p);
    launch_face(c, MODE_RES, T.coef.p, T.dt.p, -1.0, false);
    T.rec.ensure(21 * F);
    CGKS_HIP(hipMemcpyAsync(T.rec.p, c->fout.p, sizeof(double) * 21 * F, hipMemcpyDeviceToDevice, st));
    T.Anew.ensure(N);
    T.Sgv.ensure(15 * N);
    c->Rw.ensure(5 * N);
    launch_gather_res(c, c->Rw.p, T.Sgv.p, T.Anew.p, MODE_RES);
    hipLaunchKernelGGL(k_div, B1(15 * N), dim3(256), 0, st, N, T.Sgv.p, T.Anew.p, (int64_t)15, T.Sgv.p);
    // Gauss-point Jacobians, in the precision params.adjoint_tape asks for (the other copy released)
    T.fp32 = c->prm.adjoint_tape == 1;
    const size_t nJf = jf_size(NGP), nJr = (size_t)10 * RECON_IN * 5 * N;
    try {
        if (T.fp32) {
            T.Jf.release();
            T.Jr.release();
            T.Jf32.ensure(nJf);
            T.Jr32.ensure(nJr);
        } else {
            T.Jf32.release();
            T.Jr32.release();
            T.Jf.ensure(nJf);
            T.Jr.ensure(nJr);
        }
    } catch (const Error &e) {
        // out of device memory: hold none of the Jacobians, and say what they need
        T.Jf.release();
        T.Jr.release();
        T.Jf32.release();
        T.Jr32.release();
        const double gb = double(nJf + nJr) * (T.fp32 ? 4.0 : 8.0) / 1e9;
        throw Error{e.code, e.msg + " (the recorded Jacobians need " + std::to_string(gb) + " GB" +
                                (T.fp32 ? ")" : "; params.adjoint_tape = 1 stores them in FP32, in half of that)")};
    }
    T.agp.ensure(NS);
    GpArgs A;
    A.N = N;
    A.F = F;
    A.NGP = NGP;
    A.cfg = cfg_of(c);
    A.coef = T.coef.p;
    A.dt = T.dt.p;
    A.cen = c->cen.p;
    A.gpx = c->gpx.p;
    A.gpw = c->gpw.p;
    A.gpn = c->gpn.p;
    A.fshift = c->fshift.p;
    A.dtL = T.dtL.p;
    A.fl = c->fl.p;
    A.fr = c->fr.p;
    A.ftag = c->ftag.p;
    A.fngp = c->fngp.p;
    A.gpoff = c->gpoff.p;
    A.bc = c->bc.p;
    A.Jf = T.Jf.p;
    A.Jf32 = T.fp32 ? T.Jf32.p : nullptr;
    A.agp = T.agp.p;
    A.bad = c->bad.p;
    for (int p = 0; p * K_FACE < GP_IN; ++p)
        hipLaunchKernelGGL(k_face_jac<K_FACE>, B1(NS, 64), dim3(64), 0, st, A, p);
    // reconstruction Jacobians
    const ReconArgs RA = recon_args(c, T.W.p, T.G.p, T.al.p);
    for (int p = 0; p * K_RECON < RECON_IN; ++p) {
        if (T.fp32)
            hipLaunchKernelGGL((k_recon_jac<K_RECON, float>), dim3(blocks_for(N, OP_GROUP)), dim3(5 * OP_GROUP), 0,
                               st, RA, p, T.Jr32.p);
        else
            hipLaunchKernelGGL((k_recon_jac<K_RECON, double>), dim3(blocks_for(N, OP_GROUP)), dim3(5 * OP_GROUP), 0,
                               st, RA, p, T.Jr.p);
    }
    T.rev.ensure(6 * N);
    hipLaunchKernelGGL(k_rev_slots, B1(N), dim3(256), 0, st, N, c->Fi, c->cf_ptr.p, c->cf_face.p, c->fl.p, c->fr.p,
                       T.rev.p);
    // work buffers
    T.brec.ensure(21 * F);
    T.bface.ensure(101 * F);
    T.bcoef.ensure(50 * N);
    T.bdt.ensure(N);
    T.bown.ensure(30 * N);
    T.bslot.ensure(120 * N);
    T.bat.ensure(N);
    // coarse states at the linearisation point: restricted fine state, level by level
    const int nl = (int)c->lev.size();
    while ((int)T.cW.size() < nl) {
        T.cW.push_back(new DBuf<double>());
        T.cdt.push_back(new DBuf<double>());
        T.cD.push_back(new DBuf<double>());
        T.cRs.push_back(new DBuf<double>());
        T.cX.push_back(new DBuf<double>());
    }
    for (int l = 1; l < nl; ++l) {
        Level *Lv = c->lev[l];
        T.cW[l]->ensure(5 * Lv->n);
        T.cdt[l]->ensure(Lv->n);
        restrict_level(c, l, l == 1 ? T.W.p : T.cW[l - 1]->p, nullptr, T.cW[l]->p, nullptr);
        coarse_dt_level(c, l, T.cW[l]->p, T.cdt[l]->p);
    }
    CGKS_HIP(hipGetLastError());
    int32_t hb = 0;
    CGKS_HIP(hipMemcpyAsync(&hb, c->bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CGKS_HIP(hipStreamSynchronize(st));
    if (hb != INT32_MAX) {
        const int32_t big = INT32_MAX;
        CGKS_HIP(hipMemcpy(c->bad.p, &big, sizeof(int32_t), hipMemcpyHostToDevice));
        throw Error{CGKS_E_PHYS, "non-physical Gauss-point state while linearising, cell " + std::to_string(c->caller_cell(hb))};
    }
    T.ready = true;
}

// face-record cotangents in T.brec -> state cotangents
static void vjp_from_records(cgks_ctx *c, double *oW, double *oG, double *oA, bool acc)
{
    AdjTape &T = tape(c);
    hipStream_t st = c->stream;
    const int64_t N = c->N, F = c->F;
    FvArgs A;
    A.N = N;
    A.F = F;
    A.NGP = c->NGP;
    A.cen = c->cen.p;
    A.gpx = c->gpx.p;
    A.gpw = c->gpw.p;
    A.gpn = c->gpn.p;
    A.fshift = c->fshift.p;
    A.agp = T.agp.p;
    A.brec = T.brec.p;
    A.fl = c->fl.p;
    A.fr = c->fr.p;
    A.fngp = c->fngp.p;
    A.gpoff = c->gpoff.p;
    A.bface = T.bface.p;
    if (T.fp32) hipLaunchKernelGGL(k_face_vjp<float>, B1(4 * F), dim3(256), 0, st, A, T.Jf32.p);
    else hipLaunchKernelGGL(k_face_vjp<double>, B1(4 * F), dim3(256), 0, st, A, T.Jf.p);
    hipLaunchKernelGGL(k_coef_gather, B1(5 * N), dim3(256), 0, st, N, c->cf_ptr.p, c->cf_face.p, c->fr.p, T.dtL.p,
                       T.bface.p, T.bcoef.p, T.bdt.p);
    if (T.fp32) hipLaunchKernelGGL(k_recon_vjp<float>, B1(5 * N), dim3(256), 0, st, N, T.Jr32.p, T.bcoef.p, T.bown.p, T.bslot.p);
    else hipLaunchKernelGGL(k_recon_vjp<double>, B1(5 * N), dim3(256), 0, st, N, T.Jr.p, T.bcoef.p, T.bown.p, T.bslot.p);
    hipLaunchKernelGGL(k_recon_gather, B1(N), dim3(256), 0, st, N, c->slot_nb.p, T.rev.p, T.bown.p, T.bslot.p,
                       T.bdt.p, T.ddt.p, oW, oG, oA, acc ? 1 : 0);
}

void adj_vjp_residual(cgks_ctx *c, const double *bR, const double *bG, const double *bA, double *oW, double *oG,
                      double *oA, bool acc)
{
    AdjTape &T = tape(c);
    hipStream_t st = c->stream;
    const int64_t N = c->N, F = c->F;
    const bool full = bG || bA;
    if (full) hipLaunchKernelGGL(k_bat, B1(N), dim3(256), 0, st, N, bG, bA, T.Sgv.p, T.bat.p);
    hipLaunchKernelGGL(k_brec, B1(F), dim3(256), 0, st, N, F, c->fl.p, c->fr.p, c->vol.p, T.Anew.p, T.rec.p, bR, bG,
                       full ? T.bat.p : nullptr, T.brec.p);
    vjp_from_records(c, oW, oG, oA, acc);
}

void adj_vjp_wall(cgks_ctx *c, int32_t tag, const double e[3], double *oW, double *oG, double *oA, bool acc)
{
    AdjTape &T = tape(c);
    hipLaunchKernelGGL(k_brec_wall, B1(c->F), dim3(256), 0, c->stream, c->F, c->fr.p, c->ftag.p, tag, e[0], e[1], e[2],
                       T.brec.p);
    vjp_from_records(c, oW, oG, oA, acc);
}

void adj_vjp_kfvs(cgks_ctx *c, int level, const double *Wc, const double *bR, double *oW, bool acc)
{
    if (level < 1 || level >= (int)c->lev.size()) throw Error{CGKS_E_STATE, "no such level: call cgks_agglomerate"};
    Level *L = c->lev[level];
    if (!c->adj) c->adj = new AdjTape();
    AdjTape &T = *c->adj;
    const int64_t tot = L->m + L->nb;
    T.bface.ensure(10 * tot + 10);  // shares the face-cotangent buffer
    KvArgs A;
    A.n = L->n;
    A.m = L->m;
    A.nb = L->nb;
    A.gam = c->prm.gamma;
    A.K = (5.0 - 3.0 * c->prm.gamma) / (c->prm.gamma - 1.0);
    A.W = Wc;
    A.bR = bR;
    A.A = L->A.p;
    A.bA = L->bA.p;
    A.pa = L->pa.p;
    A.pb = L->pb.p;
    A.bown = L->bown.p;
    A.btag = L->btag.p;
    A.bc = c->bc.p;
    A.kb = T.bface.p;
    hipLaunchKernelGGL(k_kfvs_vjp_face, B1(tot, 128), dim3(128), 0, c->stream, A);
    hipLaunchKernelGGL(k_kfvs_vjp_gather, B1(L->n), dim3(256), 0, c->stream, L->n, L->m, L->cf_ptr.p, L->cf_item.p,
                       T.bface.p, oW, acc ? 1 : 0);
}

int adj_solve(cgks_ctx *c, int32_t tag, const double e[3], int max_iter, double tol, double *lamW, double *lamG,
              double *lamA, double *cR, double *cG, double *cA, double *hist)
{
    AdjTape &T = tape(c);
    const cgks_params &p = c->prm;
    if (p.precision != 0) throw Error{CGKS_E_STATE, "the adjoint runs in FP64 (precision 0)"};
    if (p.coarse_smoother != 0) throw Error{CGKS_E_STATE, "the adjoint transposes the forward-Euler coarse smoother"};
    if (p.cycle_gamma != 1) throw Error{CGKS_E_STATE, "the adjoint transposes the V-cycle (cycle_gamma 1)"};
    const int nl = (int)c->lev.size();
    if (std::max(1, p.nu_pre[0]) != 1) throw Error{CGKS_E_STATE, "the adjoint supports one fine pre-sweep"};
    for (int l = 0; l < std::max(nl, 1); ++l)
        if (p.nu_post[l] != 0 || (l > 0 && p.nu_pre[l] != 1))
            throw Error{CGKS_E_STATE, "the adjoint supports one pre-sweep and no post-sweeps per level"};
    hipStream_t st = c->stream;
    const int64_t N = c->N, n21 = 21 * N;
    T.lam.ensure(n21);
    T.lam1.ensure(n21);
    T.tmp.ensure(n21);
    T.jv.ensure(n21);
    T.bR.ensure(5 * N);
    T.cR.ensure(5 * N);
    const int nbk = 512;
    T.part.ensure(2 * nbk);
    for (int l = 1; l < nl; ++l) {
        const int64_t n = c->lev[l]->n;
        T.cD[l]->ensure(5 * n);
        T.cRs[l]->ensure(5 * n);
        T.cX[l]->ensure(5 * n);
    }
    // dJ/dU, layout (W 5N, G 15N, alpha N)
    double *jW = T.jv.p, *jG = jW + 5 * N, *jA = jG + 15 * N;
    adj_vjp_wall(c, tag, e, jW, jG, jA, false);
    hipLaunchKernelGGL(k_copy, B1(n21), dim3(256), 0, st, n21, T.jv.p, T.lam.p);
    double *lW = T.lam.p;
    double *l1W = T.lam1.p, *l1G = l1W + 5 * N, *l1A = l1G + 15 * N;
    double *nW = T.tmp.p, *nG = nW + 5 * N, *nA = nG + 15 * N;
    std::vector<double> hp(2 * nbk);
    int it = 0;
    for (; it < max_iter; ++it) {
        // coarse chain: lam_r = R_1^T Rs_1
        if (nl > 1) {
            Level *L1 = c->lev[1];
            hipLaunchKernelGGL(k_prolong_t, B1(L1->n), dim3(256), 0, st, L1->n, L1->nfine, L1->c2f_ptr.p,
                               L1->c2f_idx.p, lW, T.cX[1]->p);
            for (int l = 1; l + 1 < nl; ++l) {
                Level *Lc = c->lev[l + 1];
                hipLaunchKernelGGL(k_prolong_t, B1(Lc->n), dim3(256), 0, st, Lc->n, Lc->nfine, Lc->c2f_ptr.p,
                                   Lc->c2f_idx.p, T.cX[l]->p, T.cX[l + 1]->p);
            }
            {
                Level *Lt = c->lev[nl - 1];
                hipLaunchKernelGGL(k_scale_dtv, B1(Lt->n), dim3(256), 0, st, Lt->n, T.cdt[nl - 1]->p, Lt->V.p,
                                   T.cX[nl - 1]->p, T.cRs[nl - 1]->p);
            }
            for (int l = nl - 2; l >= 1; --l) {
                Level *Lv = c->lev[l], *Lc = c->lev[l + 1];
                double *t = T.cD[l]->p;  // t = R_{l+1}^T Rs_{l+1}, then D_l
                hipLaunchKernelGGL(k_restrict_t, B1(Lv->n), dim3(256), 0, st, Lv->n, Lc->n, Lc->f2c.p, T.cRs[l + 1]->p,
                                   T.cRs[l]->p);
                hipLaunchKernelGGL(k_copy, B1(5 * Lv->n), dim3(256), 0, st, 5 * Lv->n, T.cX[l]->p, t);
                adj_vjp_kfvs(c, l, T.cW[l]->p, T.cRs[l]->p, t, true);
                hipLaunchKernelGGL(k_add_scaled_dtv, B1(Lv->n), dim3(256), 0, st, Lv->n, T.cdt[l]->p, Lv->V.p,
                                   T.cRs[l]->p, t, T.cRs[l]->p);
            }
            hipLaunchKernelGGL(k_restrict_t, B1(N), dim3(256), 0, st, N, L1->n, L1->f2c.p, T.cRs[1]->p, T.bR.p);
        } else {
            launch_fill(T.bR.p, 0.0, 5 * N, st);
        }
        // lam_1 = lam + dR^T lam_r
        hipLaunchKernelGGL(k_copy, B1(n21), dim3(256), 0, st, n21, T.lam.p, T.lam1.p);
        adj_vjp_residual(c, T.bR.p, nullptr, nullptr, l1W, l1G, l1A, true);
        // parameter cotangents: c_R = lam_r + (dt/V) lam_1,W; c_G = lam_1,G; c_alpha = lam_1,alpha
        hipLaunchKernelGGL(k_add_scaled_dtv, B1(N), dim3(256), 0, st, N, T.dt.p, c->vol.p, T.bR.p, l1W, T.cR.p);
        hipLaunchKernelGGL(k_scale_dtv, B1(N), dim3(256), 0, st, N, T.dt.p, c->vol.p, l1W, T.bR.p);
        // lam' = (lam_1,W, 0, 0) + dE^T((dt/V) lam_1,W, lam_1,G, lam_1,alpha) + dJ/dU
        hipLaunchKernelGGL(k_copy, B1(n21), dim3(256), 0, st, n21, T.jv.p, T.tmp.p);
        hipLaunchKernelGGL(k_axpy, B1(5 * N), dim3(256), 0, st, 5 * N, 1.0, l1W, nW);
        adj_vjp_residual(c, T.bR.p, l1G, l1A, nW, nG, nA, true);
        // convergence: |lam' - lam| / |lam'|
        hipLaunchKernelGGL(k_diff_part, dim3(nbk), dim3(256), 0, st, n21, T.tmp.p, T.lam.p, T.part.p);
        CGKS_HIP(hipMemcpyAsync(hp.data(), T.part.p, sizeof(double) * 2 * nbk, hipMemcpyDeviceToHost, st));
        std::swap(T.lam.p, T.tmp.p);
        lW = T.lam.p;
        nW = T.tmp.p;
        nG = nW + 5 * N;
        nA = nG + 15 * N;
        CGKS_HIP(hipStreamSynchronize(st));
        double d2 = 0.0, a2 = 0.0;
        for (int b = 0; b < nbk; ++b) {
            d2 += hp[2 * b];
            a2 += hp[2 * b + 1];
        }
        const double rel = a2 > 0.0 ? std::sqrt(d2 / a2) : 0.0;
        if (!std::isfinite(rel)) throw Error{CGKS_E_NONFINITE, "adjoint iteration produced a non-finite value"};
        if (hist) hist[it] = rel;
        if (rel <= tol) {
            ++it;
            break;
        }
    }
    // outputs
    const double *fW = T.lam.p;
    if (lamW) CGKS_HIP(hipMemcpyAsync(lamW, fW, sizeof(double) * 5 * N, hipMemcpyDeviceToDevice, st));
    if (lamG) CGKS_HIP(hipMemcpyAsync(lamG, fW + 5 * N, sizeof(double) * 15 * N, hipMemcpyDeviceToDevice, st));
    if (lamA) CGKS_HIP(hipMemcpyAsync(lamA, fW + 20 * N, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    if (cR) CGKS_HIP(hipMemcpyAsync(cR, T.cR.p, sizeof(double) * 5 * N, hipMemcpyDeviceToDevice, st));
    if (cG) CGKS_HIP(hipMemcpyAsync(cG, l1G, sizeof(double) * 15 * N, hipMemcpyDeviceToDevice, st));
    if (cA) CGKS_HIP(hipMemcpyAsync(cA, l1A, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    CGKS_HIP(hipStreamSynchronize(st));
    return it;
}

// ---------------------------------------------------------------- forward-mode JVP
// Directional derivative of the fine operator E(W, G, alpha) = (R, G_new, alpha_new) along
// (vW, vG, vA), by one pass of dual numbers (one tangent) through the reconstruction, the local
// steps, the Gauss-point physics (the moment-matrix form of the flux, as in the linearisation)
// and the cell sums.  It uses no recorded Jacobian, so it checks the vector-Jacobian products
// independently (their dot products must agree to rounding).
using D1 = Dual<1>;

template <int C> __device__ __forceinline__ void recon_jvp_comp(const ReconArgs &A, const double *vW, const double *vG,
                                                               const double *vA, int64_t i, double *cv, double *ct)
{
    const int64_t N = A.N;
    D1 x[6];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        x[c] = D1(A.W[c * N + i]);
        x[c].d[0] = vW[c * N + i];
    }
    x[5] = D1(A.alpha ? A.alpha[i] : 1.0);
    x[5].d[0] = (A.alpha && vA) ? vA[i] : 0.0;
    D1 nbw[6], nbg[6][3];
    for (int s = 0; s < 6; ++s) {
        const int nbv = A.slot_nb[s * N + i];
        const bool in = nbv >= 0;
        nbw[s] = D1(in ? A.W[C * N + nbv] : 0.0);
        nbw[s].d[0] = in ? vW[C * N + nbv] : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            nbg[s][d] = D1(in ? A.G[(3 * C + d) * N + nbv] : 0.0);
            nbg[s][d].d[0] = in ? vG[(3 * C + d) * N + nbv] : 0.0;
        }
    }
    D1 r[10];
    recon_generic<D1, C>(A, i, x, x[5], nbw, nbg, r);
#pragma unroll
    for (int o = 0; o < 10; ++o) {
        cv[i * 50 + 10 * C + o] = r[o].v;
        ct[i * 50 + 10 * C + o] = r[o].d[0];
    }
}

__global__ __launch_bounds__(320) void k_recon_jvp(ReconArgs A, const double *vW, const double *vG, const double *vA,
                                                   double *cv, double *ct)
{
    const int64_t i = (int64_t)blockIdx.x * OP_GROUP + (threadIdx.x & (OP_GROUP - 1));
    if (i >= A.N) return;
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: recon_jvp_comp<0>(A, vW, vG, vA, i, cv, ct); break;
    case 1: recon_jvp_comp<1>(A, vW, vG, vA, i, cv, ct); break;
    case 2: recon_jvp_comp<2>(A, vW, vG, vA, i, cv, ct); break;
    case 3: recon_jvp_comp<3>(A, vW, vG, vA, i, cv, ct); break;
    default: recon_jvp_comp<4>(A, vW, vG, vA, i, cv, ct); break;
    }
}

__global__ void k_dt_jvp(int64_t N, int64_t F, double gam, double cfl, double mu, int viscous, const double *W,
                         const double *vW, const int32_t *cf_ptr, const int32_t *cf_face, const double *favec,
                         const double *farea, const double *vol, double *dtv, double *dtt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    D1 w[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        w[c] = D1(W[c * N + i]);
        w[c].d[0] = vW[c * N + i];
    }
    const D1 dt = local_dt_t(i, F, gam, cfl, mu, viscous, w, cf_ptr, cf_face, favec, farea, vol[i]);
    dtv[i] = dt.v;
    dtt[i] = dt.d[0];
}

// one lane per Gauss-point slot: the 11 outputs and their tangents, [22][NS]
__global__ __launch_bounds__(64) void k_face_jvp(GpArgs A, const double *ct, const double *dtt, double *sv)
{
    const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t f = gp >> 2;
    const int k = (int)(gp & 3);
    if (f >= A.F || k >= A.fngp[f]) return;
    const int64_t F = A.F, N = A.N, NS = 4 * A.F;
    const int L = A.fl[f], R = A.fr[f];
    const double x[3] = {A.gpx[(3 * k) * F + f], A.gpx[(3 * k + 1) * F + f], A.gpx[(3 * k + 2) * F + f]};
    const double n[3] = {A.gpn[(3 * k) * F + f], A.gpn[(3 * k + 1) * F + f], A.gpn[(3 * k + 2) * F + f]};
    // the face step: the smaller of the two local steps (the left one on a tie)
    const bool left = R < 0 || A.dt[L] <= A.dt[R];
    D1 dtf(left ? A.dt[L] : A.dt[R]);
    dtf.d[0] = left ? dtt[L] : dtt[R];
    D1 WL[5], GL[15], WR[5], GR[15];
    auto eval = [&](int cell, const double dx[3], D1 w[5], D1 g[15]) {
        const D1 dxd[3] = {D1(dx[0]), D1(dx[1]), D1(dx[2])};
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            D1 r[10];
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                r[q] = D1(A.coef[cell * 50 + 10 * c + q]);
                r[q].d[0] = ct[cell * 50 + 10 * c + q];
            }
            poly_eval(r, dxd, w[c], &g[3 * c]);
        }
    };
    {
        const double dx[3] = {x[0] - A.cen[L], x[1] - A.cen[N + L], x[2] - A.cen[2 * N + L]};
        eval(L, dx, WL, GL);
    }
    if (R >= 0) {
        const double dx[3] = {x[0] - A.fshift[f] - A.cen[R], x[1] - A.fshift[F + f] - A.cen[N + R],
                              x[2] - A.fshift[2 * F + f] - A.cen[2 * N + R]};
        eval(R, dx, WR, GR);
    }
    D1 out[GP_OUT];
    const bool ok = gp_outputs(A, (int)f, R, n, WL, GL, WR, GR, dtf, out);
    if (!ok) atomicMin(A.bad, L);
#pragma unroll
    for (int o = 0; o < GP_OUT; ++o) {
        sv[(int64_t)o * NS + gp] = ok ? out[o].v : (o == 10 ? 1.0 : 0.0);
        sv[(int64_t)(GP_OUT + o) * NS + gp] = ok ? out[o].d[0] : 0.0;
    }
}

// per cell: R = -sum_faces s sum_k w_k S F, G_new = alpha_new S_gv / V with
// S_gv = sum_faces s sum_k w_k S W(dt_f) n, alpha_new = product over interior-face points
__global__ void k_gather_jvp(int64_t N, int64_t F, int64_t NS, const int32_t *cf_ptr, const int32_t *cf_face,
                             const int32_t *fr, const int32_t *fngp, const double *gpw, const double *gpn,
                             const double *vol, const double *sv, double *dR, double *dG, double *dA)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    D1 r[5], gs[15], al(1.0);
    for (int k = cf_ptr[i]; k < cf_ptr[i + 1]; ++k) {
        const int it = cf_face[k];
        const int f = it >> 1;
        const double s = (it & 1) ? -1.0 : 1.0;
        for (int q = 0; q < fngp[f]; ++q) {
            const int64_t gp = 4 * (int64_t)f + q;
            const double wS = gpw[(int64_t)q * F + f];
            D1 o[GP_OUT];
#pragma unroll
            for (int j = 0; j < GP_OUT; ++j) {
                o[j] = D1(sv[(int64_t)j * NS + gp]);
                o[j].d[0] = sv[(int64_t)(GP_OUT + j) * NS + gp];
            }
#pragma unroll
            for (int c = 0; c < 5; ++c) r[c] = r[c] - (s * wS) * o[c];
#pragma unroll
            for (int c = 0; c < 5; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) gs[3 * c + d] = gs[3 * c + d] + (s * wS * gpn[(int64_t)(3 * q + d) * F + f]) * o[5 + c];
            if (fr[f] >= 0) al = al * o[10];
        }
    }
    const double iv = 1.0 / vol[i];
#pragma unroll
    for (int c = 0; c < 5; ++c) dR[c * N + i] = r[c].d[0];
#pragma unroll
    for (int q = 0; q < 15; ++q) {
        const D1 g = al * gs[q] * D1(iv);
        if (dG) dG[q * N + i] = g.d[0];
    }
    if (dA) dA[i] = al.d[0];
}

void jvp_residual(cgks_ctx *c, const double *W, const double *G, const double *alpha, const double *vW,
                  const double *vG, const double *vA, double *dR, double *dG, double *dA)
{
    hipStream_t st = c->stream;
    const int64_t N = c->N, F = c->F, NS = 4 * F;
    DBuf<double> cv, ct, dtv, dtt, sv, bg;
    cv.alloc(50 * N);
    ct.alloc(50 * N);
    dtv.alloc(N);
    dtt.alloc(N);
    sv.alloc(2 * GP_OUT * NS);
    ReconArgs RA = recon_args(c, W, G, alpha);
    hipLaunchKernelGGL(k_recon_jvp, dim3(blocks_for(N, OP_GROUP)), dim3(5 * OP_GROUP), 0, st, RA, vW, vG, vA, cv.p,
                       ct.p);
    hipLaunchKernelGGL(k_dt_jvp, B1(N), dim3(256), 0, st, N, F, c->prm.gamma, c->prm.cfl, c->prm.mu, c->prm.viscous, W,
                       vW, c->cf_ptr.p, c->cf_face.p, c->favec.p, c->farea.p, c->vol.p, dtv.p, dtt.p);
    GpArgs A;
    A.N = N;
    A.F = F;
    A.NGP = c->NGP;
    A.cfg = cfg_of(c);
    A.coef = cv.p;
    A.dt = dtv.p;
    A.cen = c->cen.p;
    A.gpx = c->gpx.p;
    A.gpw = c->gpw.p;
    A.gpn = c->gpn.p;
    A.fshift = c->fshift.p;
    A.dtL = nullptr;
    A.fl = c->fl.p;
    A.fr = c->fr.p;
    A.ftag = c->ftag.p;
    A.fngp = c->fngp.p;
    A.gpoff = c->gpoff.p;
    A.bc = c->bc.p;
    A.Jf = nullptr;
    A.Jf32 = nullptr;
    A.agp = nullptr;
    A.bad = c->bad.p;
    hipLaunchKernelGGL(k_face_jvp, B1(NS, 64), dim3(64), 0, st, A, ct.p, dtt.p, sv.p);
    hipLaunchKernelGGL(k_gather_jvp, B1(N), dim3(256), 0, st, N, F, NS, c->cf_ptr.p, c->cf_face.p, c->fr.p, c->fngp.p,
                       c->gpw.p, c->gpn.p, c->vol.p, sv.p, dR, dG, dA);
    CGKS_HIP(hipGetLastError());
    CGKS_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- parameter sensitivities
// sum over blocks of a . b, one partial per block (fixed grid: the sum is deterministic)
__global__ __launch_bounds__(256) void k_dot_part(int64_t n, const double *a, const double *b, double *part)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v += a[i] * b[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Explicit dependence on the parameters at the fixed (linearised) state.  A parameter p_k moves the
// far-field states of the boundary tags and the mesh nodes along the directions given to
// cgks_set_param_directions; J = e . F_wall(tag) and E = (R, G_new, alpha_new) change with it at
// fixed (W, G, alpha) through the ghost states, the geometry, the reconstruction operators and the
// local steps.  Both are evaluated on a context rebuilt at p_k = +-h, +-2h (same cells, same
// internal order) and differentiated by the fourth-order central difference
// f' = (8 (f(h) - f(-h)) - (f(2h) - f(-2h))) / (12 h); with the adjoint's cotangents c on E,
// dJ/dp_k = dJ/dp_k|_U + c . dE/dp_k|_U.
void adj_param_derivatives(cgks_ctx *c, int32_t tag, const double e[3], double *out)
{
    AdjTape &T = tape(c);
    hipStream_t st = c->stream;
    const int64_t N = c->N;
    const auto &H = c->hmesh;
    const double *cRp = T.cR.p, *cGp = T.lam1.p + 5 * N, *cAp = T.lam1.p + 20 * N;
    const int nbk = 256;
    DBuf<double> part, R, Gn, an, Fw;
    part.alloc(3 * nbk);
    R.alloc(5 * N);
    Gn.alloc(15 * N);
    an.alloc(N);
    Fw.alloc(3);
    std::vector<double> hp(3 * nbk);
    const double h = c->param_step;
    const double steps[4] = {-2.0 * h, -h, h, 2.0 * h};
    for (int k = 0; k < c->n_params; ++k) {
        double fE[4], fJ[4];
        for (int q = 0; q < 4; ++q) {
            const double sk = steps[q];
            std::unique_ptr<cgks_ctx> X(new cgks_ctx());
            X->prm = c->prm;
            X->prm.cell_order = 0;
            X->stream = st;
            X->device = c->device;
            X->gpu_cus = c->gpu_cus;
            X->bc_host = c->bc_host;
            X->tags_set = c->tags_set;
            for (int t = 0; t < 64; ++t)
                for (int v = 0; v < 5; ++v) X->bc_host.prim[t][v] += sk * c->pdir_prim[((size_t)k * 64 + t) * 5 + v];
            X->bc.alloc(1);
            CGKS_HIP(hipMemcpyAsync(X->bc.p, &X->bc_host, sizeof(BcTable), hipMemcpyHostToDevice, st));
            std::vector<double> xyz = H.xyz;
            if (!c->pdir_xyz.empty()) {
                const double *d = c->pdir_xyz.data() + (size_t)k * 3 * H.n_nodes;
                for (size_t j = 0; j < xyz.size(); ++j) xyz[j] += sk * d[j];
            }
            mesh_build(X.get(), H.n_nodes, xyz.data(), N, H.ct.data(), H.cp.data(), H.cn.data(), H.n_bf,
                       H.bp.empty() ? nullptr : H.bp.data(), H.bn.empty() ? nullptr : H.bn.data(),
                       H.bt.empty() ? nullptr : H.bt.data(), H.canon.empty() ? nullptr : H.canon.data());
            if (X->F != c->F) throw Error{CGKS_E_MESH, "a parameter step changed the mesh topology"};
            launch_local_dt_recon(X.get(), T.W.p, T.G.p, T.al.p, X->dtc.p, X->coef.p);
            launch_face(X.get(), MODE_RES, X->coef.p, X->dtc.p, -1.0, false);
            launch_gather_res(X.get(), R.p, Gn.p, an.p, MODE_RES);
            launch_face(X.get(), MODE_RESONLY, X->coef.p, X->dtc.p, -1.0, false);
            launch_wall_force(X.get(), tag, Fw.p);
            hipLaunchKernelGGL(k_dot_part, dim3(nbk), dim3(256), 0, st, 5 * N, cRp, R.p, part.p);
            hipLaunchKernelGGL(k_dot_part, dim3(nbk), dim3(256), 0, st, 15 * N, cGp, Gn.p, part.p + nbk);
            hipLaunchKernelGGL(k_dot_part, dim3(nbk), dim3(256), 0, st, N, cAp, an.p, part.p + 2 * nbk);
            CGKS_HIP(hipGetLastError());
            double hF[3];
            CGKS_HIP(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * 3 * nbk, hipMemcpyDeviceToHost, st));
            CGKS_HIP(hipMemcpyAsync(hF, Fw.p, sizeof(hF), hipMemcpyDeviceToHost, st));
            CGKS_HIP(hipStreamSynchronize(st));
            int32_t hb = 0;
            CGKS_HIP(hipMemcpy(&hb, X->bad.p, sizeof(int32_t), hipMemcpyDeviceToHost));
            if (hb != INT32_MAX)
                throw Error{CGKS_E_PHYS, "non-physical Gauss-point state at a parameter step, cell " +
                                             std::to_string(c->caller_cell(hb))};
            double acc = 0.0;
            for (int b = 0; b < 3 * nbk; ++b) acc += hp[b];
            fE[q] = acc;
            fJ[q] = e[0] * hF[0] + e[1] * hF[1] + e[2] * hF[2];
        }
        const double dE = (8.0 * (fE[2] - fE[1]) - (fE[3] - fE[0])) / (12.0 * h);
        const double dJ = (8.0 * (fJ[2] - fJ[1]) - (fJ[3] - fJ[0])) / (12.0 * h);
        out[k] = dJ + dE;
    }
}

}  // namespace cgks
