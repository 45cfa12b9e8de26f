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
// peculiar velocity c = u - U where the matrix is nearly diagonal.  Full-space
// moments that equal Euler fluxes or their Jacobians applied to a vector are
// formed in that closed form, and in the steady modes the time coefficients are
// applied while the moments accumulate.
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
// div_ and rsqrt_: correctly rounded in FP64; in FP32 the hardware reciprocal and reciprocal square
// root (1 ulp, one instruction each, against about ten for an IEEE division), well inside the
// FP32 flux's error budget.
template <> struct Fp<double> {
    CGKS_HD static double erfc_(double x) { return ::erfc(x); }
    CGKS_HD static double exp_(double x) { return ::exp(x); }
    CGKS_HD static double expm1_(double x) { return ::expm1(x); }
    CGKS_HD static double sqrt_(double x) { return ::sqrt(x); }
#ifdef __HIP_DEVICE_COMPILE__
    // hardware reciprocal, two Newton steps and one residual correction of the quotient
    CGKS_HD static double div_(double a, double b)
    {
        double r = __builtin_amdgcn_rcp(b);
        r = fma(fma(-b, r, 1.0), r, r);
        r = fma(fma(-b, r, 1.0), r, r);
        const double q = a * r;
        return fma(fma(-b, q, a), r, q);
    }
#else
    CGKS_HD static double div_(double a, double b) { return a / b; }
#endif
    CGKS_HD static double rsqrt_(double x) { return div_(1.0, ::sqrt(x)); }
};
template <> struct Fp<float> {
    CGKS_HD static float erfc_(float x) { return ::erfcf(x); }
    CGKS_HD static float exp_(float x) { return ::expf(x); }
    CGKS_HD static float expm1_(float x) { return ::expm1f(x); }
    CGKS_HD static float sqrt_(float x) { return ::sqrtf(x); }
#ifdef __HIP_DEVICE_COMPILE__
    CGKS_HD static float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    CGKS_HD static float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
#else
    CGKS_HD static float div_(float a, float b) { return a / b; }
    CGKS_HD static float rsqrt_(float x) { return 1.0f / ::sqrtf(x); }
#endif
};

CGKS_HD double abs_(double x) { return fabs(x); }
CGKS_HD float abs_(float x) { return fabsf(x); }
CGKS_HD double sign_(double x) { return copysign(1.0, x); }
CGKS_HD float sign_(float x) { return copysignf(1.0f, x); }
// x^e for a constant exponent
CGKS_HD double powc_(double x, double e) { return ::pow(x, e); }

// 1/sqrt(pi)
#define CGKS_RSQRT_PI 0.56418958354775628694807945156077

template <class T> struct Side {
    T rho, U, V, W, lam;
    T ir;  // 1/rho
    T p;   // pressure
    T h;   // 1/(2 lambda) = p/rho
};

// Primitive quantities of a conservative state.  rho p = (gamma - 1)(rho E - |m|^2/2) needs no
// division, and the one reciprocal 1/(rho^2 p) yields both 1/rho and lambda = rho/(2p).
template <class T> CGKS_HD Side<T> side_of(const T w[5], T gam)
{
    Side<T> s;
    s.rho = w[0];
    const T rp = (gam - T(1)) * (w[4] * w[0] - T(0.5) * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]));
    const T d = Fp<T>::div_(T(1), w[0] * rp);
    s.ir = rp * d;
    s.U = w[1] * s.ir;
    s.V = w[2] * s.ir;
    s.W = w[3] * s.ir;
    s.p = rp * s.ir;
    s.h = s.p * s.ir;
    s.lam = T(0.5) * (w[0] * w[0]) * w[0] * d;
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
    const T h = s.h;
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
    recur(t.u, s.U, s.h);
}

// half space: sgn = +1 for u > 0, -1 for u < 0
template <class T> CGKS_HD void tab_u_half(Tab<T> &t, const Side<T> &s, T sgn)
{
    const T isl = Fp<T>::sqrt_(T(2) * s.h);  // 1/sqrt(lambda)
    const T sl = s.lam * isl;                // sqrt(lambda)
    t.u[0] = T(0.5) * Fp<T>::erfc_(-sgn * sl * s.U);
    t.u[1] = s.U * t.u[0] + sgn * T(0.5) * Fp<T>::exp_(-s.lam * s.U * s.U) * T(CGKS_RSQRT_PI) * isl;
    recur(t.u, s.U, s.h);
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

// Constants of the closed-form inverse for one Maxwellian: e = |U|^2 + (K + 3)/(2 lambda) and
// c4 = 4 lambda^2/(K + 3), given iK3 = 1/(K + 3).
template <class T> struct SlopeK {
    T e, c4;
};
template <class T> CGKS_HD SlopeK<T> slope_k(const Side<T> &s, T K, T iK3)
{
    SlopeK<T> k;
    k.e = s.U * s.U + s.V * s.V + s.W * s.W + (K + T(3)) * s.h;
    k.c4 = T(4) * s.lam * s.lam * iK3;
    return k;
}

// Solve M a = b for a micro-slope, M = <psi psi^T> of the normalised Maxwellian (closed form).
template <class T> CGKS_HD void slope_solve(const Side<T> &s, const SlopeK<T> &k, const T b[5], T a[5])
{
    const T e = k.e;
    const T R1 = b[1] - s.U * b[0];
    const T R2 = b[2] - s.V * b[0];
    const T R3 = b[3] - s.W * b[0];
    const T R4 = T(2) * b[4] - e * b[0];
    a[4] = k.c4 * (R4 - T(2) * (s.U * R1 + s.V * R2 + s.W * R3));
    a[1] = T(2) * s.lam * R1 - s.U * a[4];
    a[2] = T(2) * s.lam * R2 - s.V * a[4];
    a[3] = T(2) * s.lam * R3 - s.W * a[4];
    a[0] = b[0] - s.U * a[1] - s.V * a[2] - s.W * a[3] - T(0.5) * a[4] * e;
}

// ---------------------------------------------------------------- moment matrices
// Symmetric 5x5 matrix m_ab = <w psi_a psi_b> for the weight w = u^A v^B w^C, packed as
// (00 01 02 03 04 11 12 13 14 22 23 24 33 34 44).  psi_4 = (u^2 + v^2 + w^2 + xi^2)/2.
template <int A, int B, int C, class T> CGKS_HD void mmat(const Tab<T> &t, T m[15])
{
#define CGKS_P(i, j, k) (t.u[i] * t.v[j] * t.w[k])
    const T x1 = t.x[1];
    const T p000 = CGKS_P(A, B, C);
    const T p200 = CGKS_P(A + 2, B, C), p020 = CGKS_P(A, B + 2, C), p002 = CGKS_P(A, B, C + 2);
    const T p100 = CGKS_P(A + 1, B, C), p010 = CGKS_P(A, B + 1, C), p001 = CGKS_P(A, B, C + 1);
    m[0] = p000;
    m[1] = p100;
    m[2] = p010;
    m[3] = p001;
    m[4] = T(0.5) * (p200 + p020 + p002 + p000 * x1);
    m[5] = p200;
    m[6] = CGKS_P(A + 1, B + 1, C);
    m[7] = CGKS_P(A + 1, B, C + 1);
    m[8] = T(0.5) * (CGKS_P(A + 3, B, C) + CGKS_P(A + 1, B + 2, C) + CGKS_P(A + 1, B, C + 2) + p100 * x1);
    m[9] = p020;
    m[10] = CGKS_P(A, B + 1, C + 1);
    m[11] = T(0.5) * (CGKS_P(A + 2, B + 1, C) + CGKS_P(A, B + 3, C) + CGKS_P(A, B + 1, C + 2) + p010 * x1);
    m[12] = p002;
    m[13] = T(0.5) * (CGKS_P(A + 2, B, C + 1) + CGKS_P(A, B + 2, C + 1) + CGKS_P(A, B, C + 3) + p001 * x1);
    m[14] = T(0.25) * (CGKS_P(A + 4, B, C) + CGKS_P(A, B + 4, C) + CGKS_P(A, B, C + 4) +
                       T(2) * (CGKS_P(A + 2, B + 2, C) + CGKS_P(A + 2, B, C + 2) + CGKS_P(A, B + 2, C + 2)) +
                       T(2) * (p200 + p020 + p002) * x1 + p000 * t.x[2]);
#undef CGKS_P
}

// y += s * m x for a packed symmetric matrix
template <class T> CGKS_HD void msym_acc(const T m[15], const T x[5], T s, T y[5])
{
    y[0] += s * (m[0] * x[0] + m[1] * x[1] + m[2] * x[2] + m[3] * x[3] + m[4] * x[4]);
    y[1] += s * (m[1] * x[0] + m[5] * x[1] + m[6] * x[2] + m[7] * x[3] + m[8] * x[4]);
    y[2] += s * (m[2] * x[0] + m[6] * x[1] + m[9] * x[2] + m[10] * x[3] + m[11] * x[4]);
    y[3] += s * (m[3] * x[0] + m[7] * x[1] + m[10] * x[2] + m[12] * x[3] + m[13] * x[4]);
    y[4] += s * (m[4] * x[0] + m[8] * x[1] + m[11] * x[2] + m[13] * x[3] + m[14] * x[4]);
}

// first column of m (the moments <w psi_a>), scaled
template <class T> CGKS_HD void mcol0_acc(const T m[15], T s, T y[5])
{
    y[0] += s * m[0];
    y[1] += s * m[1];
    y[2] += s * m[2];
    y[3] += s * m[3];
    y[4] += s * m[4];
}

// The full-space Maxwellian family g = exp(theta . psi) has the Euler fluxes as its moments
// rho <u_j psi> = F_j(W) (K internal degrees of freedom: gamma - 1 = 2/(K + 3)).  A change of
// theta along a vector b moves g by g (b . psi), so rho <u_j psi psi^T> b = A_j(W) rho <psi psi^T> b
// with A_j = dF_j/dW, the Euler flux Jacobian.  Two uses: the transport moment of the
// compatibility condition, Eq. (co), rho sum_j <u_j psi psi^T> a_j = sum_j A_j dW_j (the micro-slopes
// are fixed by rho <psi psi^T> a_j = dW_j), and the interface Maxwellian's flux and time-slope
// moments rho <u psi> = F_x and rho <u psi psi^T> A = A_x (rho <psi psi^T> A).  Both are formed here
// from the closed forms instead of from moment matrices.
template <class T> struct EulerLin {
    T U[3], q2h, Ep, gm1, ir;  // velocity, |U|^2/2, E + p, gamma - 1, 1/rho
};
template <class T> CGKS_HD EulerLin<T> euler_lin(const Side<T> &s, T K, T iK3)
{
    EulerLin<T> e;
    e.U[0] = s.U;
    e.U[1] = s.V;
    e.U[2] = s.W;
    e.q2h = T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
    e.Ep = s.p * (T(0.5) * K + T(2.5)) + s.rho * e.q2h;
    e.gm1 = T(2) * iK3;
    e.ir = s.ir;
    return e;
}
// r += A_j(W) d
template <class T> CGKS_HD void euler_jvp_acc(const EulerLin<T> &e, int j, const T d[5], T r[5])
{
    const T dp = e.gm1 * (d[4] - (e.U[0] * d[1] + e.U[1] * d[2] + e.U[2] * d[3]) + e.q2h * d[0]);
    const T rdu = d[1 + j] - e.U[j] * d[0];  // rho du_j
    r[0] += d[1 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i) r[1 + i] += d[1 + i] * e.U[j] + e.U[i] * rdu + (i == j ? dp : T(0));
    r[4] += (d[4] + dp) * e.U[j] + e.Ep * rdu * e.ir;
}
// rho tr = sum_j A_j(W) dW_j
template <class T> CGKS_HD void euler_divergence(const EulerLin<T> &e, const T g[3][5], T r[5])
{
#pragma unroll
    for (int c = 0; c < 5; ++c) r[c] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) euler_jvp_acc(e, j, g[j], r);
}

// The interface Maxwellian's second-order transport term sum_j rho <u u_j psi psi^T> a_j, by the
// same argument: it is sum_j dQ_j/dW dW_j with Q_j(W) = rho <u u_j psi> (x = u the normal),
//   Q_j = (rho U_x U_j + p d_xj,  rho U_x U_j U_i + p (U_x d_ij + U_j d_xi + U_i d_xj),
//          rho U_x U_j (|U|^2 + (K + 7) th) / 2 + p d_xj (|U|^2 + (K + 5) th) / 2),  th = p / rho,
// the Maxwellian's third and fourth velocity moments.  Formed in closed form, this leaves the
// interface Maxwellian without slopes, tables or moment matrices.
template <class T>
CGKS_HD void second_transport(const EulerLin<T> &e, const Side<T> &s, T K, const T g[3][5], T out[5])
{
    const T *U = e.U;
    const T th = s.p * s.ir;
    const T A = T(2) * e.q2h + (K + T(7)) * th;   // |U|^2 + (K + 7) th
    const T Bc = T(2) * e.q2h + (K + T(5)) * th;  // |U|^2 + (K + 5) th
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T *d = g[j];
        T rdu[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) rdu[i] = d[1 + i] - U[i] * d[0];  // rho dU_i
        const T dp = e.gm1 * (d[4] - (U[0] * d[1] + U[1] * d[2] + U[2] * d[3]) + e.q2h * d[0]);
        const T udu = U[0] * rdu[0] + U[1] * rdu[1] + U[2] * rdu[2];  // rho U.dU
        const T dth = dp - th * d[0];                                  // rho d(th)
        const T dmu = d[1] * U[j] + U[0] * rdu[j];                     // d(rho U_x U_j)
        out[0] += dmu + (j == 0 ? dp : T(0));
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T v = d[1] * U[j] * U[i] + U[0] * (rdu[j] * U[i] + U[j] * rdu[i]);
            if (i == j) v += dp * U[0] + th * rdu[0];
            if (i == 0) v += dp * U[j] + th * rdu[j];
            if (j == 0) v += dp * U[i] + th * rdu[i];
            out[1 + i] += v;
        }
        T v4 = T(0.5) * dmu * A + U[0] * U[j] * (udu + T(0.5) * (K + T(7)) * dth);
        if (j == 0) v4 += T(0.5) * dp * Bc + th * (udu + T(0.5) * (K + T(5)) * dth);
        out[4] += v4;
    }
}

// Space slopes a_j from local-frame gradients g[j][c].
template <class T> CGKS_HD void space_slopes(const Side<T> &s, const SlopeK<T> &k, const T g[3][5], T a[3][5])
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T b[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) b[c] = g[j][c] * s.ir;
        slope_solve(s, k, b, a[j]);
    }
}

// Space slopes a_j and the time slope A of a side Maxwellian: M A = -tr with
// tr = sum_j <u_j a_j psi> from its closed form.
template <class T>
CGKS_HD void slopes(const Side<T> &s, T K, T iK3, const T g[3][5], T a[3][5], T A[5])
{
    const SlopeK<T> k = slope_k(s, K, iK3);
    space_slopes(s, k, g, a);
    T r[5];
    euler_divergence(euler_lin(s, K, iK3), g, r);
    T b[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) b[c] = -r[c] * s.ir;
    slope_solve(s, k, b, A);
}

// Interface Maxwellian (local frame), all in closed form: rho tr = sum_j A_j dW_j (= -rho <A psi>),
// its Euler flux F_x(W) = rho <u psi>, A_x (rho tr) = -rho <u psi psi^T> A, and
// sum_j rho <u u_j psi psi^T> a_j.
template <class T>
CGKS_HD void center_terms(const Side<T> &s, const T W[5], T K, T iK3, const T g[3][5], T rtr[5], T fx[5], T jt[5],
                          T q2[5])
{
    const EulerLin<T> e = euler_lin(s, K, iK3);
    euler_divergence(e, g, rtr);
    fx[0] = W[1];
    fx[1] = W[1] * s.U + s.p;
    fx[2] = W[1] * s.V;
    fx[3] = W[1] * s.W;
    fx[4] = e.Ep * s.U;
#pragma unroll
    for (int c = 0; c < 5; ++c) jt[c] = T(0);
    euler_jvp_acc(e, 0, rtr, jt);
    second_transport(e, s, K, g, q2);
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

// VAL = false skips the moments that only the interface value W(t) and the Prandtl
// correction need (a uniform branch).
template <class T>
CGKS_HD bool gks_moments(const T wl[5], const T gl[3][5], const T wr[5], const T gr[3][5], T gam, T K,
                         GksMoments<T> &o, bool VAL = true)
{
    const Side<T> sl = side_of(wl, gam), sr = side_of(wr, gam);
    if (!(sl.rho > T(0) && sr.rho > T(0) && sl.lam > T(0) && sr.lam > T(0))) return false;
    const T iK3 = T(1) / (K + T(3));
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
    // two sides, one after the other to bound register live ranges
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const Side<T> &s = side == 0 ? sl : sr;
        const T(*g)[5] = side == 0 ? gl : gr;
        Tab<T> t;
        tab_vw(t, s, K);
        T a[3][5], A[5];
        slopes(s, K, iK3, g, a, A);
        tab_u_half(t, s, side == 0 ? T(1) : T(-1));
        const T rho = s.rho;
        T m[15];
        mmat<0, 0, 0>(t, m);  // <psi psi>_half
        mcol0_acc(m, rho, Wc);
        mcol0_acc(m, rho, o.Vk[0]);
#pragma unroll
        for (int j = 0; j < 3; ++j) msym_acc(m, a[j], rho, dWc[j]);
        if (VAL) msym_acc(m, A, rho, o.Vk[2]);
        mmat<1, 0, 0>(t, m);  // <u psi psi>_half
        mcol0_acc(m, rho, o.Mk[0]);
        msym_acc(m, A, rho, o.Mk[2]);
        if (VAL) {
            msym_acc(m, a[0], rho, o.Vk[1]);
            mmat<0, 1, 0>(t, m);
            msym_acc(m, a[1], rho, o.Vk[1]);
            mmat<0, 0, 1>(t, m);
            msym_acc(m, a[2], rho, o.Vk[1]);
        }
        mmat<2, 0, 0>(t, m);
        msym_acc(m, a[0], rho, o.Mk[1]);
        mmat<1, 1, 0>(t, m);
        msym_acc(m, a[1], rho, o.Mk[1]);
        mmat<1, 0, 1>(t, m);
        msym_acc(m, a[2], rho, o.Mk[1]);
    }
    const Side<T> sc = side_of(Wc, gam);
    if (!(sc.rho > T(0) && sc.lam > T(0))) return false;
    {
        T rtr[5], fx[5], jt[5], q2[5];
        center_terms(sc, Wc, K, iK3, dWc, rtr, fx, jt, q2);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            o.Vc[0][c] = Wc[c];
            o.Vc[1][c] = rtr[c];   // rho_c <(a_c.u) psi>
            o.Vc[2][c] = -rtr[c];  // compatibility: <A_c psi> = -<(a_c.u) psi>
            o.Mc[0][c] = fx[c];    // rho_c <u psi>
            o.Mc[1][c] = q2[c];    // rho_c <u (a_c.u) psi>
            o.Mc[2][c] = -jt[c];   // rho_c <u A_c psi>
        }
    }
    o.Uc[0] = sc.U;
    o.Uc[1] = sc.V;
    o.Uc[2] = sc.W;
    o.pl = sl.p;
    o.pr = sr.p;
    o.pc = sc.p;
    return true;
}

// Time coefficients of Eq. 2nd-flux integrated over [0, T] (first six) and at time t (last six).
template <class T> struct TimeCoef {
    T c1, c2, c3, e, k1, k2;
};

template <class T> CGKS_HD TimeCoef<T> coef_integrated(T Tt, T tau, T taun)
{
    const T x = Fp<T>::div_(Tt, taun);
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
    const T x = Fp<T>::div_(t, taun);
    const T e = Fp<T>::exp_(-x);
    TimeCoef<T> c;
    c.c1 = -Fp<T>::expm1_(-x);
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

// Tangential transport over a half space in u: with m = <h(u) psi psi^T>_half for a weight h(u),
// out = <h v psi psi^T>_half a1 + <h w psi psi^T>_half a2.  The half space restricts u only, so
// the v and w integrals are Gaussian with means V, W and variance th = p/rho, and Stein's
// identity <v f> = V <f> + th <df/dv> (dpsi/dv = e_v + v e_E) reduces both terms to the products
// y1 = m a1, y2 = m a2 (returned) and the columns <h psi>, <h v psi>, <h w psi> of m.
template <class T>
CGKS_HD void tangential_transport(const T m[15], const T a1[5], const T a2[5], T V, T W, T th, T y1[5], T y2[5],
                                  T out[5])
{
#pragma unroll
    for (int c = 0; c < 5; ++c) y1[c] = y2[c] = T(0);
    msym_acc(m, a1, T(1), y1);
    msym_acc(m, a2, T(1), y2);
    const T c0[5] = {m[0], m[1], m[2], m[3], m[4]};     // <h psi>
    const T c2[5] = {m[2], m[6], m[9], m[10], m[11]};   // <h v psi>
    const T c3[5] = {m[3], m[7], m[10], m[12], m[13]};  // <h w psi>
#pragma unroll
    for (int c = 0; c < 5; ++c)
        out[c] = V * y1[c] + W * y2[c] + th * ((a1[2] + a2[3]) * c0[c] + a1[4] * c2[c] + a2[4] * c3[c]);
    out[2] += th * y1[0];
    out[3] += th * y2[0];
    out[4] += th * (y1[2] + y2[3]);
}

// The parts of tangential_transport that are not m (V a1 + W a2): th ((a1_v + a2_w) <h psi> +
// a1_E <h v psi> + a2_E <h w psi>) and the e_v, e_w, e_E terms from rows 0, 2 and 3 of m times
// a1, a2.  A caller that folds m (V a1 + W a2) into another product with m adds these.
template <class T>
CGKS_HD void tangential_rest(const T m[15], const T a1[5], const T a2[5], T th, T s, T out[5])
{
    const T r10 = m[0] * a1[0] + m[1] * a1[1] + m[2] * a1[2] + m[3] * a1[3] + m[4] * a1[4];     // (m a1)_0
    const T r12 = m[2] * a1[0] + m[6] * a1[1] + m[9] * a1[2] + m[10] * a1[3] + m[11] * a1[4];   // (m a1)_v
    const T r20 = m[0] * a2[0] + m[1] * a2[1] + m[2] * a2[2] + m[3] * a2[3] + m[4] * a2[4];     // (m a2)_0
    const T r23 = m[3] * a2[0] + m[7] * a2[1] + m[10] * a2[2] + m[12] * a2[3] + m[13] * a2[4];  // (m a2)_w
    const T c0[5] = {m[0], m[1], m[2], m[3], m[4]};
    const T c2[5] = {m[2], m[6], m[9], m[10], m[11]};
    const T c3[5] = {m[3], m[7], m[10], m[12], m[13]};
    const T st = s * th;
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] += st * ((a1[2] + a2[3]) * c0[c] + a1[4] * c2[c] + a2[4] * c3[c]);
    out[2] += st * r10;
    out[3] += st * r20;
    out[4] += st * (r12 + r23);
}

// Normal transport over a half space in u: <u^2 psi psi^T>_half a from mu = <u psi psi^T>_half,
// y0 = <psi psi^T>_half a and yu = mu a.  Integrating by parts in u, (u - U) g = -th dg/du, so
// <u f>_half = U <f>_half + th <df/du>_half plus a boundary term th f(0) g(0) that vanishes here
// because f = u psi (psi.a) has the factor u; with dpsi/du = e_u + u e_E that leaves y0, yu and
// the columns <u psi>, <u^2 psi> of mu.
template <class T>
CGKS_HD void normal_transport(const T mu[15], const T y0[5], const T yu[5], const T a[5], T U, T th, T out[5])
{
    const T c0[5] = {mu[0], mu[1], mu[2], mu[3], mu[4]};  // <u psi>
    const T c1[5] = {mu[1], mu[5], mu[6], mu[7], mu[8]};  // <u^2 psi>
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = U * yu[c] + th * (y0[c] + a[1] * c0[c] + a[4] * c1[c]);
    out[1] += th * yu[0];
    out[4] += th * yu[1];
}

// Flux over [0, dt] and interface value at dt of one Gauss point with the time coefficients
// applied while the moments accumulate: the same sums as gks_moments + flux_integrated + value_at
// without keeping the twelve moment vectors for a final combination.
//  - Inviscid (VISC = false): tau = 0 and tau_n depends only on the two side pressures, so the
//    coefficients are known before the moment loops.
//  - Viscous (VISC = true): tau = mu/p_c needs the interface state first, so W_c is formed in a
//    first pass over the two half-space Maxwellians (zeroth moments only); the flux moments are
//    then folded as in the inviscid case.  The value moments rho <psi {1, a.u, A}> of the two
//    sides are kept (15 values) because the interface value (coefficients at dt) and the Prandtl
//    correction (coefficients integrated over [0, dt]) each combine them with their own set.
// VAL = false skips the interface value.
template <class T, bool VAL, bool VISC>
CGKS_HD bool gks_flux_folded(const T wl[5], const T gl[3][5], const T wr[5], const T gr[3][5], T gam, T K, T dt,
                             const GksCfg &cfg, T F[5], T Wt[5], T &pl, T &pr)
{
    const Side<T> sl = side_of(wl, gam), sr = side_of(wr, gam);
    if (!(sl.rho > T(0) && sr.rho > T(0) && sl.lam > T(0) && sr.lam > T(0))) return false;
    pl = sl.p;
    pr = sr.p;
    const T jump = abs_(Fp<T>::div_(pl - pr, pl + pr));
    T Wc[5] = {T(0), T(0), T(0), T(0), T(0)};
    T tau = T(0), taun;
    if (VISC) {
        // W_c = rho_l <psi>_{u>0} + rho_r <psi>_{u<0}, Eq. (compatibility2)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const Side<T> &s = side == 0 ? sl : sr;
            Tab<T> t;
            tab_vw(t, s, K);
            tab_u_half(t, s, side == 0 ? T(1) : T(-1));
            T q[5];
            mpsi<0, 0, 0>(t, q);
#pragma unroll
            for (int c = 0; c < 5; ++c) Wc[c] += s.rho * q[c];
        }
        const Side<T> s0 = side_of(Wc, gam);
        if (!(s0.rho > T(0) && s0.lam > T(0))) return false;
        tau = Fp<T>::div_(T(cfg.mu), s0.p);
        taun = tau + T(cfg.c_tau) * jump * dt;
    } else {
        taun = T(cfg.eps_tau) * dt + T(cfg.c_tau) * jump * dt;
    }
    const TimeCoef<T> cf = coef_integrated(dt, tau, taun);
    TimeCoef<T> cw;
    if (VAL) cw = coef_at(dt, tau, taun);
    const T iK3 = Fp<T>::div_(T(1), K + T(3));
    T dWc[3][5];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 5; ++c) dWc[j][c] = T(0);
    T Vk[3][5];  // viscous: rho <psi {-, a.u, A}>_half summed over the sides (Vk[0] is W_c)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        F[c] = Wt[c] = T(0);
        Vk[1][c] = Vk[2][c] = T(0);
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const Side<T> &s = side == 0 ? sl : sr;
        const T(*g)[5] = side == 0 ? gl : gr;
        Tab<T> t;
        tab_vw(t, s, K);
        T a[3][5], A[5];
        slopes(s, K, iK3, g, a, A);
        tab_u_half(t, s, side == 0 ? T(1) : T(-1));
        const T rho = s.rho;
        T m[15];
        mmat<0, 0, 0>(t, m);  // <psi psi>_half
        if (!VISC) mcol0_acc(m, rho, Wc);
        // value modes keep <psi psi^T>_half a_0 for the normal transport below; the residual-only
        // mode forms that term from <u^2 psi psi^T>_half instead (fewer live registers)
        T y0[5] = {T(0), T(0), T(0), T(0), T(0)};
        if (VISC || VAL) {
            msym_acc(m, a[0], T(1), y0);
#pragma unroll
            for (int c = 0; c < 5; ++c) dWc[0][c] += rho * y0[c];
        } else {
            msym_acc(m, a[0], rho, dWc[0]);
        }
        T tv[5];  // <v psi psi^T>_half a_1 + <w psi psi^T>_half a_2
        if (VISC || VAL) {
            T y1[5], y2[5];
            tangential_transport(m, a[1], a[2], s.V, s.W, s.h, y1, y2, tv);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                dWc[1][c] += rho * y1[c];
                dWc[2][c] += rho * y2[c];
            }
        } else {
            msym_acc(m, a[1], rho, dWc[1]);
            msym_acc(m, a[2], rho, dWc[2]);
        }
        if (VISC) {
            msym_acc(m, A, rho, Vk[2]);
        } else if (VAL) {
            mcol0_acc(m, cw.e * rho, Wt);
            msym_acc(m, A, -cw.k2 * rho, Wt);
        }
        mmat<1, 0, 0>(t, m);  // <u psi psi>_half
        mcol0_acc(m, cf.e * rho, F);
        const T sk = -cf.k1 * rho;
        {
            // F += <u psi psi^T>_half (-k2 rho A - k1 rho (V a_1 + W a_2)) in one product, then the
            // rest of the tangential transport <u v psi psi^T>_half a_1 + <u w psi psi^T>_half a_2
            T b[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) b[c] = -cf.k2 * rho * A[c] + sk * (s.V * a[1][c] + s.W * a[2][c]);
            msym_acc(m, b, T(1), F);
            tangential_rest(m, a[1], a[2], s.h, sk, F);
        }
        T yu[5] = {T(0), T(0), T(0), T(0), T(0)};  // <u psi psi^T>_half a_0
        if (VISC || VAL) {
            msym_acc(m, a[0], T(1), yu);
            const T sv = VISC ? rho : -cw.k1 * rho;
            T *dst = VISC ? Vk[1] : Wt;
#pragma unroll
            for (int c = 0; c < 5; ++c) dst[c] += sv * (yu[c] + tv[c]);
        }
        if (VISC || VAL) {
            // <u^2 psi psi^T>_half a_0
            T tn[5];
            normal_transport(m, y0, yu, a[0], s.U, s.h, tn);
#pragma unroll
            for (int c = 0; c < 5; ++c) F[c] += sk * tn[c];
        } else {
            mmat<2, 0, 0>(t, m);
            msym_acc(m, a[0], -cf.k1 * rho, F);
        }
    }
    const Side<T> sc = side_of(Wc, gam);
    if (!(sc.rho > T(0) && sc.lam > T(0))) return false;
    T Q[5];  // viscous: time-integrated conserved variables for the Prandtl correction
    {
        // interface Maxwellian in closed form (see center_terms), each term entering as formed
        const EulerLin<T> e = euler_lin(sc, K, iK3);
        T rtr[5];
        euler_divergence(e, dWc, rtr);
        // rho_c <psi {1, a_c.u, A_c}> = {W_c, rho tr, -rho tr}
        if (VISC) {
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                const T vc = (cf.c2 - cf.c3) * rtr[c] + cf.c1 * Wc[c];
                Q[c] = vc + cf.e * Wc[c] - cf.k1 * Vk[1][c] - cf.k2 * Vk[2][c];
                if (VAL)
                    Wt[c] = cw.c1 * Wc[c] + (cw.c2 - cw.c3) * rtr[c] + cw.e * Wc[c] - cw.k1 * Vk[1][c] -
                            cw.k2 * Vk[2][c];
            }
        } else if (VAL) {
#pragma unroll
            for (int c = 0; c < 5; ++c) Wt[c] += cw.c1 * Wc[c] + (cw.c2 - cw.c3) * rtr[c];
        }
        // rho_c <u psi {1, a_c.u, A_c}> = {F_x(W_c), sum_j dQ_j dW_j, -A_x rho tr}
        F[0] += cf.c1 * Wc[1];
        F[1] += cf.c1 * (Wc[1] * sc.U + sc.p);
        F[2] += cf.c1 * (Wc[1] * sc.V);
        F[3] += cf.c1 * (Wc[1] * sc.W);
        F[4] += cf.c1 * (e.Ep * sc.U);
        T t5[5] = {T(0), T(0), T(0), T(0), T(0)};
        euler_jvp_acc(e, 0, rtr, t5);
#pragma unroll
        for (int c = 0; c < 5; ++c) F[c] -= cf.c3 * t5[c];
        second_transport(e, sc, K, dWc, t5);
#pragma unroll
        for (int c = 0; c < 5; ++c) F[c] += cf.c2 * t5[c];
    }
    if (VISC && cfg.prandtl != 1.0) {
        const T Uc[3] = {sc.U, sc.V, sc.W};
        F[4] += (Fp<T>::div_(T(1), T(cfg.prandtl)) - T(1)) * heat_flux(F, Q, Uc);
    }
    return true;
}

// First-order kinetic flux vector splitting in the face frame (coarse levels, Sec. 4.2):
// F = rho_l <u psi>_{u>0} + rho_r <u psi>_{u<0}.
template <class T> CGKS_HD void kfvs_local(const T wl[5], const T wr[5], T gam, T K, T F[5])
{
    const Side<T> sl = side_of(wl, gam), sr = side_of(wr, gam);
    Tab<T> t;
    T q[5];
    tab_vw(t, sl, K);
    tab_u_half(t, sl, T(1));
    mpsi<1, 0, 0>(t, q);
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] = sl.rho * q[c];
    tab_vw(t, sr, K);
    tab_u_half(t, sr, T(-1));
    mpsi<1, 0, 0>(t, q);
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] += sr.rho * q[c];
}

// ---------------------------------------------------------------- frames
// Orthonormal basis completing a unit normal (Duff et al. 2017, branchless).
template <class T> CGKS_HD void onb(const T n[3], T t1[3], T t2[3])
{
    const T s = sign_(n[2]);
    const T a = Fp<T>::div_(T(-1), s + n[2]);
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
template <class S, class T, class Gm>
CGKS_HD void to_local(const S w[5], const S g[15], const Gm n[3], const Gm t1[3], const Gm t2[3], T wl[5], T gl[3][5])
{
    wl[0] = T(w[0]);
    wl[1] = T(w[1] * n[0] + w[2] * n[1] + w[3] * n[2]);
    wl[2] = T(w[1] * t1[0] + w[2] * t1[1] + w[3] * t1[2]);
    wl[3] = T(w[1] * t2[0] + w[2] * t2[1] + w[3] * t2[2]);
    wl[4] = T(w[4]);
    const Gm *E[3] = {n, t1, t2};
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

template <class T, class S, class Gm>
CGKS_HD void to_global(const T l[5], const Gm n[3], const Gm t1[3], const Gm t2[3], S o[5])
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
    // a Mach number is |m|/(rho c) with rho c = sqrt(gamma p rho); |dp|/p_l + |dp|/p_r = |dp| (p_l + p_r)/(p_l p_r)
    const S il = Fp<S>::rsqrt_(gam * pl * S(wl[0])), ir = Fp<S>::rsqrt_(gam * pr * S(wr[0]));
    const S mtl = Fp<S>::sqrt_(S(wl[2]) * S(wl[2]) + S(wl[3]) * S(wl[3]));
    const S mtr = Fp<S>::sqrt_(S(wr[2]) * S(wr[2]) + S(wr[3]) * S(wr[3]));
    const S dmn = S(wl[1]) * il - S(wr[1]) * ir, dmt = mtl * il - mtr * ir;
    const S A = Fp<S>::div_(abs_(pl - pr) * (pl + pr), pl * pr) + dmn * dmn + dmt * dmt;
    return Fp<S>::div_(S(1), S(1) + A * A);
}

}  // namespace cgks
