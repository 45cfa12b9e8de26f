// Forward-mode dual numbers with K tangent directions, host and device.
//
// The flux, reconstruction and time-step code is templated on its scalar type;
// instantiated with Dual<K> it carries K directional derivatives alongside each
// value, which is how the adjoint builds its local Jacobians exactly (no finite
// differences).  Non-smooth points take one-sided derivatives: |x| and sign use
// the sign of the value (+ at 0); sqrt has zero derivative at 0.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "gks_device.hpp"

namespace cgks {

template <int K> struct Dual {
    double v;
    double d[K];
    CGKS_HD Dual() : v(0.0)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
    CGKS_HD Dual(double x) : v(x)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
    CGKS_HD explicit operator double() const { return v; }
};

#define CGKS_DUAL_LOOP(body)                                                                                           \
    _Pragma("unroll") for (int k = 0; k < K; ++k) body

template <int K> CGKS_HD Dual<K> operator+(const Dual<K> &a, const Dual<K> &b)
{
    Dual<K> r;
    r.v = a.v + b.v;
    CGKS_DUAL_LOOP(r.d[k] = a.d[k] + b.d[k];)
    return r;
}
template <int K> CGKS_HD Dual<K> operator-(const Dual<K> &a, const Dual<K> &b)
{
    Dual<K> r;
    r.v = a.v - b.v;
    CGKS_DUAL_LOOP(r.d[k] = a.d[k] - b.d[k];)
    return r;
}
template <int K> CGKS_HD Dual<K> operator-(const Dual<K> &a)
{
    Dual<K> r;
    r.v = -a.v;
    CGKS_DUAL_LOOP(r.d[k] = -a.d[k];)
    return r;
}
template <int K> CGKS_HD Dual<K> operator*(const Dual<K> &a, const Dual<K> &b)
{
    Dual<K> r;
    r.v = a.v * b.v;
    CGKS_DUAL_LOOP(r.d[k] = a.d[k] * b.v + a.v * b.d[k];)
    return r;
}
template <int K> CGKS_HD Dual<K> operator/(const Dual<K> &a, const Dual<K> &b)
{
    Dual<K> r;
    const double ib = 1.0 / b.v;
    r.v = a.v * ib;
    CGKS_DUAL_LOOP(r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;)
    return r;
}
template <int K> CGKS_HD Dual<K> operator+(const Dual<K> &a, double b) { return a + Dual<K>(b); }
template <int K> CGKS_HD Dual<K> operator+(double a, const Dual<K> &b) { return Dual<K>(a) + b; }
template <int K> CGKS_HD Dual<K> operator-(const Dual<K> &a, double b) { return a - Dual<K>(b); }
template <int K> CGKS_HD Dual<K> operator-(double a, const Dual<K> &b) { return Dual<K>(a) - b; }
template <int K> CGKS_HD Dual<K> operator*(const Dual<K> &a, double b)
{
    Dual<K> r;
    r.v = a.v * b;
    CGKS_DUAL_LOOP(r.d[k] = a.d[k] * b;)
    return r;
}
template <int K> CGKS_HD Dual<K> operator*(double a, const Dual<K> &b) { return b * a; }
template <int K> CGKS_HD Dual<K> operator/(const Dual<K> &a, double b) { return a * (1.0 / b); }
template <int K> CGKS_HD Dual<K> operator/(double a, const Dual<K> &b) { return Dual<K>(a) / b; }
template <int K> CGKS_HD Dual<K> &operator+=(Dual<K> &a, const Dual<K> &b) { return a = a + b; }
template <int K> CGKS_HD Dual<K> &operator-=(Dual<K> &a, const Dual<K> &b) { return a = a - b; }
template <int K> CGKS_HD Dual<K> &operator*=(Dual<K> &a, const Dual<K> &b) { return a = a * b; }
template <int K> CGKS_HD Dual<K> &operator/=(Dual<K> &a, const Dual<K> &b) { return a = a / b; }
template <int K> CGKS_HD bool operator<(const Dual<K> &a, const Dual<K> &b) { return a.v < b.v; }
template <int K> CGKS_HD bool operator>(const Dual<K> &a, const Dual<K> &b) { return a.v > b.v; }
template <int K> CGKS_HD bool operator<=(const Dual<K> &a, const Dual<K> &b) { return a.v <= b.v; }
template <int K> CGKS_HD bool operator>=(const Dual<K> &a, const Dual<K> &b) { return a.v >= b.v; }
template <int K> CGKS_HD bool operator<(const Dual<K> &a, double b) { return a.v < b; }
template <int K> CGKS_HD bool operator>(const Dual<K> &a, double b) { return a.v > b; }
template <int K> CGKS_HD bool operator>=(const Dual<K> &a, double b) { return a.v >= b; }
template <int K> CGKS_HD bool operator<=(const Dual<K> &a, double b) { return a.v <= b; }

// derivative-scaled copy: value f, derivative fp * a.d
template <int K> CGKS_HD Dual<K> chain(const Dual<K> &a, double f, double fp)
{
    Dual<K> r;
    r.v = f;
    CGKS_DUAL_LOOP(r.d[k] = fp * a.d[k];)
    return r;
}

template <int K> CGKS_HD Dual<K> abs_(const Dual<K> &a) { return chain(a, fabs(a.v), copysign(1.0, a.v)); }
template <int K> CGKS_HD Dual<K> sign_(const Dual<K> &a) { return Dual<K>(copysign(1.0, a.v)); }

template <int K> struct Fp<Dual<K>> {
    CGKS_HD static Dual<K> erfc_(const Dual<K> &x)
    {
        return chain(x, ::erfc(x.v), -2.0 * CGKS_RSQRT_PI * ::exp(-x.v * x.v));
    }
    CGKS_HD static Dual<K> exp_(const Dual<K> &x)
    {
        const double e = ::exp(x.v);
        return chain(x, e, e);
    }
    CGKS_HD static Dual<K> expm1_(const Dual<K> &x) { return chain(x, ::expm1(x.v), ::exp(x.v)); }
    CGKS_HD static Dual<K> sqrt_(const Dual<K> &x)
    {
        const double s = ::sqrt(x.v);
        return chain(x, s, s > 0.0 ? 0.5 / s : 0.0);
    }
    CGKS_HD static Dual<K> div_(const Dual<K> &a, const Dual<K> &b) { return a / b; }
    CGKS_HD static Dual<K> rsqrt_(const Dual<K> &x) { return Dual<K>(1.0) / sqrt_(x); }
};

// x^e for a constant exponent
template <int K> CGKS_HD Dual<K> powc_(const Dual<K> &x, double e)
{
    const double p = ::pow(x.v, e);
    return chain(x, p, x.v != 0.0 ? e * p / x.v : 0.0);
}

#undef CGKS_DUAL_LOOP

}  // namespace cgks
