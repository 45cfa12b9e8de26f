// Algorithmic operation count of one face Gauss point of the fine flux kernel.
//
// The per-point physics in gks_device.hpp is host-and-device; here it is
// instantiated on the host with a scalar that counts every add, multiply,
// divide and transcendental call, following the exact sequence the face kernel
// executes in its steady mode with the gradient update (FP64): polynomial
// evaluation on both sides, rotation to the face frame, moments and micro-slopes
// of the three Maxwellians with the time coefficients of the flux and of the
// interface value applied as they accumulate, compression factor, rotation back
// and the weighted contribution.  Argument 1: Gauss points of the face (3 or 4);
// argument 2: "inviscid" (default) or "viscous" (Navier-Stokes path: a first
// pass for the interface state, tau = mu/p_c, and the Prandtl-number correction
// of the heat flux).  A fused multiply-add counts as two operations, matching
// the convention of the FP64 peak.
#include <cstdio>
#include <cstring>

#include "gks_device.hpp"

namespace cgks {
struct Tally {
    long add = 0, mul = 0, div = 0, trans = 0, cmp = 0;
};
static Tally g;

struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
    explicit operator double() const { return v; }
};
inline Cnt operator+(Cnt a, Cnt b) { ++g.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g.add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g.div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt &operator+=(Cnt &a, Cnt b) { a = a + b; return a; }
inline Cnt &operator-=(Cnt &a, Cnt b) { a = a - b; return a; }
inline Cnt &operator*=(Cnt &a, Cnt b) { a = a * b; return a; }
inline bool operator>(Cnt a, Cnt b) { ++g.cmp; return a.v > b.v; }
inline bool operator<(Cnt a, Cnt b) { ++g.cmp; return a.v < b.v; }
inline Cnt abs_(Cnt a) { return Cnt(a.v < 0 ? -a.v : a.v); }
inline Cnt sign_(Cnt a) { return Cnt(a.v < 0 ? -1.0 : 1.0); }
template <> struct Fp<Cnt> {
    static Cnt erfc_(Cnt x) { ++g.trans; return Cnt(::erfc(x.v)); }
    static Cnt exp_(Cnt x) { ++g.trans; return Cnt(::exp(x.v)); }
    static Cnt expm1_(Cnt x) { ++g.trans; return Cnt(::expm1(x.v)); }
    static Cnt sqrt_(Cnt x) { ++g.trans; return Cnt(::sqrt(x.v)); }
    static Cnt div_(Cnt a, Cnt b) { return a / b; }
    static Cnt rsqrt_(Cnt x) { return Cnt(1.0) / sqrt_(x); }
};
}  // namespace cgks

using namespace cgks;

int main(int argc, char **argv)
{
    const int ngp = argc > 1 ? atoi(argv[1]) : 4;  // Gauss points of the face (3 or 4) for the face-sum share
    const bool visc = argc > 2 && std::strcmp(argv[2], "viscous") == 0;
    // a smooth, non-degenerate state on both sides
    Cnt coefL[50], coefR[50];
    for (int c = 0; c < 5; ++c)
        for (int k = 0; k < 10; ++k) {
            const double base[5] = {1.0, 0.5, 0.1, -0.05, 2.0};
            coefL[10 * c + k] = k == 0 ? base[c] : 0.01 * (k + c);
            coefR[10 * c + k] = k == 0 ? base[c] * 1.01 : 0.012 * (k + c);
        }
    Cnt x[3] = {0.3, 0.2, 0.1}, cenL[3] = {0.25, 0.2, 0.1}, cenR[3] = {0.35, 0.21, 0.1}, sh[3] = {0, 0, 0};
    Cnt n[3] = {1.0, 0.0, 0.0};
    Cnt wS = 0.01, dtf = 0.002;
    const double gam = 1.4;
    GksCfg cfg{gam, (5.0 - 3.0 * gam) / (gam - 1.0), visc ? 2e-3 : 0.0, visc ? 0.72 : 1.0, 0.01, 1.0, visc ? 1 : 0};
    g = Tally();
    // polynomial evaluation, both sides
    Cnt WL[5], GL[15], WR[5], GR[15];
    {
        Cnt dx[3] = {x[0] - cenL[0], x[1] - cenL[1], x[2] - cenL[2]};
        for (int c = 0; c < 5; ++c) poly_eval(&coefL[10 * c], dx, WL[c], &GL[3 * c]);
        Cnt dxr[3] = {x[0] - sh[0] - cenR[0], x[1] - sh[1] - cenR[1], x[2] - sh[2] - cenR[2]};
        for (int c = 0; c < 5; ++c) poly_eval(&coefR[10 * c], dxr, WR[c], &GR[3 * c]);
    }
    const Tally t_eval = g;
    Cnt t1[3], t2[3];
    onb(n, t1, t2);
    Cnt wl[5], wr[5], gl[3][5], gr[3][5];
    to_local(WL, GL, n, t1, t2, wl, gl);
    to_local(WR, GR, n, t1, t2, wr, gr);
    const Tally t_rot = g;
    // the steady path of the kernel: moments with the time coefficients folded in
    Cnt Fl[5], Fg[5], Wt[5], pl, pr;
    if (visc) gks_flux_folded<Cnt, true, true>(wl, gl, wr, gr, Cnt(gam), Cnt(cfg.K), dtf, cfg, Fl, Wt, pl, pr);
    else gks_flux_folded<Cnt, true, false>(wl, gl, wr, gr, Cnt(gam), Cnt(cfg.K), dtf, cfg, Fl, Wt, pl, pr);
    const Tally t_mom = g;
    to_global(Fl, n, t1, t2, Fg);
    const Cnt s = wS / dtf;
    Cnt acc[21];
    for (int q = 0; q < 5; ++q) acc[q] = s * Fg[q];
    Cnt Wg[5];
    to_global(Wt, n, t1, t2, Wg);
    for (int q = 0; q < 5; ++q)
        for (int d = 0; d < 3; ++d) acc[5 + 3 * q + d] = wS * Wg[q] * n[d];
    Cnt al = cf_factor(wl, wr, pl, pr, Cnt(gam));
    (void)al;
    const Tally t_all = g;
    // face sum of 20 weighted values and the product of 1 factor over the face's points, per point
    const double face_ops = 21.0 * (ngp - 1) / ngp;
    const double flops = 2.0 * 0 + t_all.add + t_all.mul + t_all.div + t_all.trans + face_ops;
    printf("{\"add\": %ld, \"mul\": %ld, \"div\": %ld, \"trans\": %ld, \"cmp\": %ld, \"face_sum_per_point\": %.4f, "
           "\"eval\": %ld, \"rotate\": %ld, \"moments\": %ld, \"flops_per_point\": %.4f}\n",
           t_all.add, t_all.mul, t_all.div, t_all.trans, t_all.cmp, face_ops,
           t_eval.add + t_eval.mul + t_eval.div + t_eval.trans,
           t_rot.add + t_rot.mul + t_rot.div + t_rot.trans - (t_eval.add + t_eval.mul + t_eval.div + t_eval.trans),
           t_mom.add + t_mom.mul + t_mom.div + t_mom.trans - (t_rot.add + t_rot.mul + t_rot.div + t_rot.trans), flops);
    return 0;
}
