// Device-side gas-kinetic physics for CDNA4 (gfx950), templated on the
// floating-point type so the flux can run in FP64 or FP32.
//
// Paper: BGK model and K = (5 - 3 gamma)/(gamma - 1) (Sec. 2.1); micro-slopes
// from the moment equations and compatibility (Sec. 2.3, Eqs. co, co-moment);
// interface equilibrium from half-space moments (Eq. compatibility2); collision
// times with the pressure-jump term; time-dependent interface distribution
// (Eq. 2nd-flux); interface conservative values (Sec. 2.4).
//
// Moments are tabulated per side as one-dimensional recursions and combined by
// compile-time-indexed helpers, so every table entry stays in registers.
// Micro-slopes use the closed-form inverse of the 5x5 moment matrix, derived in
// peculiar velocity c = u - U where the matrix is nearly diagonal.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

// Host-and-device so the same source can be instantiated with a counting scalar
// on the host to tally the arithmetic per Gauss point.
#ifndef CGKS_HD
#define CGKS_HD __host__ __device__ __forceinline__
#endif

namespace cgks {

template <class T> struct Fp;
template <> struct Fp<double> {
    CGKS_HD static double erfc_(double x) { return ::erfc(x); }
    CGKS_HD static double exp_(double x) { return ::exp(x); }
    CGKS_HD static double expm1_(double x) { return ::expm1(x); }
    CGKS_HD static double sqrt_(double x) { return ::sqrt(x); }
};
template <> struct Fp<float> {
    CGKS_HD static float erfc_(float x) { return ::erfcf(x); }
    CGKS_HD static float exp_(float x) { return ::expf(x); }
    CGKS_HD static float expm1_(float x) { return ::expm1f(x); }
    CGKS_HD static float sqrt_(float x) { return ::sqrtf(x); }
};

CGKS_HD double abs_(double x) { return fabs(x); }
CGKS_HD float abs_(float x) { return fabsf(x); }
CGKS_HD double sign_(double x) { return copysign(1.0, x); }
CGKS_HD float sign_(float x) { return copysignf(1.0f, x); }

// 1/sqrt(pi)
#define CGKS_RSQRT_PI 0.56418958354775628694807945156077

template <class T> struct Side {
    T rho, U, V, W, lam;
};

template <class T> CGKS_HD Side<T> side_of(const T w[5], T gam)
{
    Side<T> s;
    s.rho = w[0];
    const T ir = T(1) / w[0];
    s.U = w[1] * ir;
    s.V = w[2] * ir;
    s.W = w[3] * ir;
    const T p = (gam - T(1)) * (w[4] - T(0.5) * w[0] * (s.U * s.U + s.V * s.V + s.W * s.W));
    s.lam = T(0.5) * w[0] / p;
    return s;
}

// Moment tables of the normalised Maxwellian: <u^n>, <v^n>, <w^n>, n = 0..6; <xi^0>, <xi^2>, <xi^4>.
template <class T> struct Tab {
    T u[7], v[7], w[7], x[3];
};

template <class T> CGKS_HD void recur(T *m, T U, T h)
{
    // m[n+2] = U m[n+1] + (n+1) h m[n], h = 1/(2 lambda)
#pragma unroll
    for (int n = 0; n < 5; ++n) m[n + 2] = U * m[n + 1] + T(n + 1) * h * m[n];
}

template <class T> CGKS_HD void tab_vw(Tab<T> &t, const Side<T> &s, T K)
{
    const T h = T(0.5) / s.lam;
    t.v[0] = T(1);
    t.v[1] = s.V;
    recur(t.v, s.V, h);
    t.w[0] = T(1);
    t.w[1] = s.W;
    recur(t.w, s.W, h);
    t.x[0] = T(1);
    t.x[1] = K * h;
    t.x[2] = K * (K + T(2)) * h * h;
}

template <class T> CGKS_HD void tab_u_full(Tab<T> &t, const Side<T> &s)
{
    t.u[0] = T(1);
    t.u[1] = s.U;
    recur(t.u, s.U, T(0.5) / s.lam);
}

// half space: sgn = +1 for u > 0, -1 for u < 0
template <class T> CGKS_HD void tab_u_half(Tab<T> &t, const Side<T> &s, T sgn)
{
    const T sl = Fp<T>::sqrt_(s.lam);
    t.u[0] = T(0.5) * Fp<T>::erfc_(-sgn * sl * s.U);
    t.u[1] = s.U * t.u[0] + sgn * T(0.5) * Fp<T>::exp_(-s.lam * s.U * s.U) * T(CGKS_RSQRT_PI) / sl;
    recur(t.u, s.U, T(0.5) / s.lam);
}

// <u^n v^m w^k psi_a>, a = 0..4
template <int n, int m, int k, class T> CGKS_HD void mpsi(const Tab<T> &t, T o[5])
{
    const T vw = t.v[m] * t.w[k];
    const T uvw = t.u[n] * vw;
    o[0] = uvw;
    o[1] = t.u[n + 1] * vw;
    o[2] = t.u[n] * t.v[m + 1] * t.w[k];
    o[3] = t.u[n] * t.v[m] * t.w[k + 1];
    o[4] = T(0.5) * (t.u[n + 2] * vw + t.u[n] * (t.v[m + 2] * t.w[k] + t.v[m] * t.w[k + 2]) + uvw * t.x[1]);
}

// <xi^2 u^n v^m w^k psi_a>
template <int n, int m, int k, class T> CGKS_HD void mpsi_x2(const Tab<T> &t, T o[5])
{
    const T vw = t.v[m] * t.w[k];
    const T uvw = t.u[n] * vw;
    o[0] = t.x[1] * uvw;
    o[1] = t.x[1] * t.u[n + 1] * vw;
    o[2] = t.x[1] * t.u[n] * t.v[m + 1] * t.w[k];
    o[3] = t.x[1] * t.u[n] * t.v[m] * t.w[k + 1];
    o[4] = T(0.5) * (t.x[1] * (t.u[n + 2] * vw + t.u[n] * (t.v[m + 2] * t.w[k] + t.v[m] * t.w[k + 2])) + uvw * t.x[2]);
}

// acc += s * <a u^n v^m w^k psi>, a = a0 + a1 u + a2 v + a3 w + a4 (u^2+v^2+w^2+xi^2)/2
template <int n, int m, int k, class T> CGKS_HD void macc(const Tab<T> &t, const T a[5], T s, T acc[5])
{
    T q[5], r[5];
    mpsi<n, m, k>(t, q);
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] = a[0] * q[i];
    mpsi<n + 1, m, k>(t, q);
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] += a[1] * q[i];
    mpsi<n, m + 1, k>(t, q);
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] += a[2] * q[i];
    mpsi<n, m, k + 1>(t, q);
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] += a[3] * q[i];
    T e[5];
    mpsi<n + 2, m, k>(t, e);
    mpsi<n, m + 2, k>(t, q);
#pragma unroll
    for (int i = 0; i < 5; ++i) e[i] += q[i];
    mpsi<n, m, k + 2>(t, q);
#pragma unroll
    for (int i = 0; i < 5; ++i) e[i] += q[i];
    mpsi_x2<n, m, k>(t, q);
    const T h4 = T(0.5) * a[4];
#pragma unroll
    for (int i = 0; i < 5; ++i) acc[i] += s * (r[i] + h4 * (e[i] + q[i]));
}

// acc += s * <(u a_x + v a_y + w a_z) u^n psi>   (n = 0: value moment, n = 1: flux moment)
template <int n, class T> CGKS_HD void macc_transport(const Tab<T> &t, const T a[3][5], T s, T acc[5])
{
    macc<n + 1, 0, 0>(t, a[0], s, acc);
    macc<n, 1, 0>(t, a[1], s, acc);
    macc<n, 0, 1>(t, a[2], s, acc);
}

// Solve M a = b for a micro-slope, M = <psi psi^T> of the normalised Maxwellian (closed form).
template <class T> CGKS_HD void slope_solve(const Side<T> &s, T K, const T b[5], T a[5])
{
    const T q2 = s.U * s.U + s.V * s.V + s.W * s.W;
    const T e = q2 + (K + T(3)) / (T(2) * s.lam);
    const T R1 = b[1] - s.U * b[0];
    const T R2 = b[2] - s.V * b[0];
    const T R3 = b[3] - s.W * b[0];
    const T R4 = T(2) * b[4] - e * b[0];
    a[4] = T(4) * s.lam * s.lam / (K + T(3)) * (R4 - T(2) * (s.U * R1 + s.V * R2 + s.W * R3));
    a[1] = T(2) * s.lam * R1 - s.U * a[4];
    a[2] = T(2) * s.lam * R2 - s.V * a[4];
    a[3] = T(2) * s.lam * R3 - s.W * a[4];
    a[0] = b[0] - s.U * a[1] - s.V * a[2] - s.W * a[3] - T(0.5) * a[4] * e;
}

// Space slopes a_j from local-frame gradients g[j][c] of conservative variables, and the time slope A.
template <class T>
CGKS_HD void slopes(const Side<T> &s, const Tab<T> &full, T K, const T g[3][5], T a[3][5], T A[5])
{
    const T ir = T(1) / s.rho;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T b[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) b[c] = g[j][c] * ir;
        slope_solve(s, K, b, a[j]);
    }
    T b[5] = {T(0), T(0), T(0), T(0), T(0)};
    macc_transport<0>(full, a, T(-1), b);
    slope_solve(s, K, b, A);
}

struct GksCfg {
    double gamma, K, mu, prandtl, eps_tau, c_tau;
    int viscous;
};

// Moment vectors of one Gauss point, local frame (normal = x).
template <class T> struct GksMoments {
    T Mc[3][5];  // rho_c <u psi {1, a_c.u, A_c}>
    T Mk[3][5];  // kinetic: rho_l <u psi {1, a_l.u, A_l}>_{u>0} + rho_r <...>_{u<0}
    T Vc[3][5];  // rho_c <psi {1, a_c.u, A_c}>
    T Vk[3][5];
    T Uc[3];     // velocity of g^c
    T pl, pr, pc;
};

template <class T>
CGKS_HD bool gks_moments(const T wl[5], const T gl[3][5], const T wr[5], const T gr[3][5], T gam, T K,
                                            GksMoments<T> &o)
{
    const Side<T> sl = side_of(wl, gam), sr = side_of(wr, gam);
    if (!(sl.rho > T(0) && sr.rho > T(0) && sl.lam > T(0) && sr.lam > T(0))) return false;
    T Wc[5] = {T(0), T(0), T(0), T(0), T(0)};
    T dWc[3][5];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 5; ++c) dWc[j][c] = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 5; ++c) o.Mk[i][c] = o.Vk[i][c] = T(0);
    // two sides, processed one after the other to bound register live ranges
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const Side<T> &s = side == 0 ? sl : sr;
        const T(*g)[5] = side == 0 ? gl : gr;
        Tab<T> t;
        tab_vw(t, s, K);
        tab_u_full(t, s);
        T a[3][5], A[5];
        slopes(s, t, K, g, a, A);
        tab_u_half(t, s, side == 0 ? T(1) : T(-1));
        const T rho = s.rho;
        T q[5];
        mpsi<0, 0, 0>(t, q);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            Wc[c] += rho * q[c];
            o.Vk[0][c] += rho * q[c];
        }
        mpsi<1, 0, 0>(t, q);
#pragma unroll
        for (int c = 0; c < 5; ++c) o.Mk[0][c] += rho * q[c];
#pragma unroll
        for (int j = 0; j < 3; ++j) macc<0, 0, 0>(t, a[j], rho, dWc[j]);
        macc_transport<1>(t, a, rho, o.Mk[1]);
        macc_transport<0>(t, a, rho, o.Vk[1]);
        macc<1, 0, 0>(t, A, rho, o.Mk[2]);
        macc<0, 0, 0>(t, A, rho, o.Vk[2]);
    }
    const Side<T> sc = side_of(Wc, gam);
    if (!(sc.rho > T(0) && sc.lam > T(0))) return false;
    {
        Tab<T> t;
        tab_vw(t, sc, K);
        tab_u_full(t, sc);
        T a[3][5], A[5];
        slopes(sc, t, K, dWc, a, A);
        const T rho = sc.rho;
        T q[5];
        mpsi<1, 0, 0>(t, q);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            o.Mc[0][c] = rho * q[c];
            o.Mc[1][c] = o.Mc[2][c] = o.Vc[1][c] = o.Vc[2][c] = T(0);
            o.Vc[0][c] = Wc[c];
        }
        macc_transport<1>(t, a, rho, o.Mc[1]);
        macc<1, 0, 0>(t, A, rho, o.Mc[2]);
        macc_transport<0>(t, a, rho, o.Vc[1]);
        macc<0, 0, 0>(t, A, rho, o.Vc[2]);
    }
    o.Uc[0] = sc.U;
    o.Uc[1] = sc.V;
    o.Uc[2] = sc.W;
    o.pl = sl.rho / (T(2) * sl.lam);
    o.pr = sr.rho / (T(2) * sr.lam);
    o.pc = sc.rho / (T(2) * sc.lam);
    return true;
}

// Time coefficients of Eq. 2nd-flux integrated over [0, T] (first six) and at time t (last six).
template <class T> struct TimeCoef {
    T c1, c2, c3, e, k1, k2;
};

template <class T> CGKS_HD TimeCoef<T> coef_integrated(T Tt, T tau, T taun)
{
    const T x = Tt / taun;
    const T E = Fp<T>::exp_(-x);
    const T omE = -Fp<T>::expm1_(-x);
    TimeCoef<T> c;
    const T Ie = taun * omE;
    const T Ite = taun * taun * omE - taun * Tt * E;
    c.c1 = Tt - taun * omE;
    c.c2 = Ite + tau * Ie - tau * Tt;
    c.c3 = T(0.5) * Tt * Tt - tau * Tt + tau * Ie;
    c.e = Ie;
    c.k1 = tau * Ie + Ite;
    c.k2 = tau * Ie;
    return c;
}

template <class T> CGKS_HD TimeCoef<T> coef_at(T t, T tau, T taun)
{
    const T e = Fp<T>::exp_(-t / taun);
    TimeCoef<T> c;
    c.c1 = -Fp<T>::expm1_(-t / taun);
    c.c2 = (t + tau) * e - tau;
    c.c3 = t - tau + tau * e;
    c.e = e;
    c.k1 = (tau + t) * e;
    c.k2 = tau * e;
    return c;
}

template <class T> CGKS_HD void combine(const TimeCoef<T> &c, const T Mc[3][5], const T Mk[3][5], T out[5])
{
#pragma unroll
    for (int i = 0; i < 5; ++i)
        out[i] = c.c1 * Mc[0][i] + c.c2 * Mc[1][i] + c.c3 * Mc[2][i] + c.e * Mk[0][i] - c.k1 * Mk[1][i] - c.k2 * Mk[2][i];
}

// Heat flux (relative to the g^c velocity) of time-integrated flux F and conserved integral Q.
template <class T> CGKS_HD T heat_flux(const T F[5], const T Q[5], const T U[3])
{
    const T u2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    return F[4] - (U[0] * F[1] + U[1] * F[2] + U[2] * F[3]) + T(0.5) * u2 * F[0] - U[0] * Q[4] +
           U[0] * (U[0] * Q[1] + U[1] * Q[2] + U[2] * Q[3]) - T(0.5) * u2 * U[0] * Q[0];
}

// Collision times: tau (outside the exponentials) and tau_n.
template <class T> CGKS_HD void collision_times(const GksMoments<T> &m, T dt, const GksCfg &cfg, T &tau, T &taun)
{
    const T jump = abs_((m.pl - m.pr) / (m.pl + m.pr));
    if (cfg.viscous) {
        tau = T(cfg.mu) / m.pc;
        taun = tau + T(cfg.c_tau) * jump * dt;
    } else {
        tau = T(0);
        taun = T(cfg.eps_tau) * dt + T(cfg.c_tau) * jump * dt;
    }
}

// Time-integrated flux over [0, Tt] with the Prandtl correction.
template <class T>
CGKS_HD void flux_integrated(const GksMoments<T> &m, T Tt, T tau, T taun, const GksCfg &cfg, T F[5])
{
    const TimeCoef<T> c = coef_integrated(Tt, tau, taun);
    combine(c, m.Mc, m.Mk, F);
    if (cfg.viscous && cfg.prandtl != 1.0) {
        T Q[5];
        combine(c, m.Vc, m.Vk, Q);
        F[4] += (T(1) / T(cfg.prandtl) - T(1)) * heat_flux(F, Q, m.Uc);
    }
}

template <class T> CGKS_HD void value_at(const GksMoments<T> &m, T t, T tau, T taun, T Wt[5])
{
    const TimeCoef<T> c = coef_at(t, tau, taun);
    combine(c, m.Vc, m.Vk, Wt);
}

// ---------------------------------------------------------------- frames
// Orthonormal basis completing a unit normal (Duff et al. 2017, branchless).
template <class T> CGKS_HD void onb(const T n[3], T t1[3], T t2[3])
{
    const T s = sign_(n[2]);
    const T a = T(-1) / (s + n[2]);
    const T b = n[0] * n[1] * a;
    t1[0] = T(1) + s * n[0] * n[0] * a;
    t1[1] = s * b;
    t1[2] = -s * n[0];
    t2[0] = b;
    t2[1] = s + n[1] * n[1] * a;
    t2[2] = -n[1];
}

// ---------------------------------------------------------------- per-point helpers
// value and gradient of R(x) = r0 + r.dx + quadratic terms (order 1, x, y, z, xx, yy, zz, xy, yz, xz)
template <class S> CGKS_HD void poly_eval(const S r[10], const S dx[3], S &w, S g[3])
{
    const S x = dx[0], y = dx[1], z = dx[2];
    w = r[0] + r[1] * x + r[2] * y + r[3] * z + r[4] * x * x + r[5] * y * y + r[6] * z * z + r[7] * x * y + r[8] * y * z +
        r[9] * x * z;
    g[0] = r[1] + S(2) * r[4] * x + r[7] * y + r[9] * z;
    g[1] = r[2] + S(2) * r[5] * y + r[7] * x + r[8] * z;
    g[2] = r[3] + S(2) * r[6] * z + r[8] * y + r[9] * x;
}

// conservative state and gradients G[3c+d] into the frame (n, t1, t2): wl[c'], gl[j][c']
template <class S, class T>
CGKS_HD void to_local(const S w[5], const S g[15], const S n[3], const S t1[3], const S t2[3], T wl[5], T gl[3][5])
{
    wl[0] = T(w[0]);
    wl[1] = T(w[1] * n[0] + w[2] * n[1] + w[3] * n[2]);
    wl[2] = T(w[1] * t1[0] + w[2] * t1[1] + w[3] * t1[2]);
    wl[3] = T(w[1] * t2[0] + w[2] * t2[1] + w[3] * t2[2]);
    wl[4] = T(w[4]);
    const S *E[3] = {n, t1, t2};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        S D[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) D[c] = g[3 * c] * E[j][0] + g[3 * c + 1] * E[j][1] + g[3 * c + 2] * E[j][2];
        gl[j][0] = T(D[0]);
        gl[j][1] = T(D[1] * n[0] + D[2] * n[1] + D[3] * n[2]);
        gl[j][2] = T(D[1] * t1[0] + D[2] * t1[1] + D[3] * t1[2]);
        gl[j][3] = T(D[1] * t2[0] + D[2] * t2[1] + D[3] * t2[2]);
        gl[j][4] = T(D[4]);
    }
}

template <class T, class S>
CGKS_HD void to_global(const T l[5], const S n[3], const S t1[3], const S t2[3], S o[5])
{
    o[0] = S(l[0]);
#pragma unroll
    for (int d = 0; d < 3; ++d) o[1 + d] = S(l[1]) * n[d] + S(l[2]) * t1[d] + S(l[3]) * t2[d];
    o[4] = S(l[4]);
}

// gradient compression factor of one Gauss point from the two local-frame states (Sec. 3.3):
// 1/(1+A^2), A = |dp|/p_l + |dp|/p_r + (Ma_n,l - Ma_n,r)^2 + (Ma_t,l - Ma_t,r)^2
template <class T, class S>
CGKS_HD S cf_factor(const T wl[5], const T wr[5], S pl, S pr, S gam)
{
    const S rl = S(wl[0]), rr = S(wr[0]);
    const S cl = Fp<S>::sqrt_(gam * pl / rl), cr = Fp<S>::sqrt_(gam * pr / rr);
    const S unl = S(wl[1]) / rl, unr = S(wr[1]) / rr;
    const S vtl = Fp<S>::sqrt_(S(wl[2]) * S(wl[2]) + S(wl[3]) * S(wl[3])) / rl;
    const S vtr = Fp<S>::sqrt_(S(wr[2]) * S(wr[2]) + S(wr[3]) * S(wr[3])) / rr;
    const S dp = abs_(pl - pr);
    const S dmn = unl / cl - unr / cr, dmt = vtl / cl - vtr / cr;
    const S A = dp / pl + dp / pr + dmn * dmn + dmt * dmt;
    return S(1) / (S(1) + A * A);
}

}  // namespace cgks
