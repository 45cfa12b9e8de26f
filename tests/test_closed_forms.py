"""Host check of the closed forms in the face-flux physics (gks_device.hpp).

The flux kernels replace several moment-matrix products by exact identities of Maxwellian moments
(Euler fluxes and their Jacobians for full-space moments, Stein's identity in v and w and
integration by parts in u for half-space moments).  This test compiles the header for the host
and compares each closed form with the moment-matrix product it replaces, on random states, for
both half spaces and two ratios of specific heats.  It checks the product code against itself (the
GPU parity tests compare the kernels with the oracle); it guards the identities against edits.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2402_02075_amd", "csrc")
ROCM_INC = "/opt/rocm/include"

SRC = r"""
#include <cstdio>
#include <cmath>
#include <random>
#include "gks_device.hpp"
using namespace cgks;
static double rel(const double *a, const double *b) {
    double s = 0, d = 0;
    for (int c = 0; c < 5; ++c) { s = fmax(s, fabs(b[c])); d = fmax(d, fabs(a[c] - b[c])); }
    return d / s;
}
int main() {
    std::mt19937_64 rng(3);
    std::uniform_real_distribution<double> U(-1, 1);
    double e_tr = 0, e_fx = 0, e_jt = 0, e_q2 = 0, e_tan = 0, e_tanu = 0, e_nor = 0, e_rest = 0;
    for (int it = 0; it < 2000; ++it) {
        const double gam = it % 2 ? 1.4 : 5.0 / 3.0, K = (5 - 3 * gam) / (gam - 1), iK3 = 1 / (K + 3);
        double w[5];
        w[0] = 1 + 0.5 * U(rng);
        for (int d = 0; d < 3; ++d) w[1 + d] = w[0] * 1.2 * U(rng);
        const double p = 0.7 + 0.3 * U(rng);
        w[4] = p / (gam - 1) + 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0];
        double g[3][5];
        for (int j = 0; j < 3; ++j) for (int c = 0; c < 5; ++c) g[j][c] = U(rng);
        const Side<double> s = side_of(w, gam);
        double a[3][5], A[5];
        slopes(s, K, iK3, g, a, A);
        // full space: transport moment, Euler flux, time-slope moment, second-order transport
        Tab<double> t;
        tab_vw(t, s, K);
        tab_u_full(t, s);
        double m[15], tr[5] = {0, 0, 0, 0, 0}, fx0[5] = {0, 0, 0, 0, 0}, jt0[5] = {0, 0, 0, 0, 0};
        double q20[5] = {0, 0, 0, 0, 0};
        mmat<1, 0, 0>(t, m); msym_acc(m, a[0], s.rho, tr); mcol0_acc(m, s.rho, fx0); msym_acc(m, A, s.rho, jt0);
        mmat<0, 1, 0>(t, m); msym_acc(m, a[1], s.rho, tr);
        mmat<0, 0, 1>(t, m); msym_acc(m, a[2], s.rho, tr);
        mmat<2, 0, 0>(t, m); msym_acc(m, a[0], s.rho, q20);
        mmat<1, 1, 0>(t, m); msym_acc(m, a[1], s.rho, q20);
        mmat<1, 0, 1>(t, m); msym_acc(m, a[2], s.rho, q20);
        double rtr[5], fx[5], jt[5], q2[5];
        center_terms(s, w, K, iK3, g, rtr, fx, jt, q2);
        for (int c = 0; c < 5; ++c) jt[c] = -jt[c];
        e_tr = fmax(e_tr, rel(rtr, tr));
        e_fx = fmax(e_fx, rel(fx, fx0));
        e_jt = fmax(e_jt, rel(jt, jt0));
        e_q2 = fmax(e_q2, rel(q2, q20));
        // half spaces: tangential terms (weights 1 and u) and the u^2 term
        for (int sg = 0; sg < 2; ++sg) {
            tab_vw(t, s, K);
            tab_u_half(t, s, sg ? 1.0 : -1.0);
            double m0[15], mu[15], ref[5] = {0, 0, 0, 0, 0}, refu[5] = {0, 0, 0, 0, 0}, refn[5] = {0, 0, 0, 0, 0};
            mmat<0, 1, 0>(t, m); msym_acc(m, a[1], 1.0, ref);
            mmat<0, 0, 1>(t, m); msym_acc(m, a[2], 1.0, ref);
            mmat<1, 1, 0>(t, m); msym_acc(m, a[1], 1.0, refu);
            mmat<1, 0, 1>(t, m); msym_acc(m, a[2], 1.0, refu);
            mmat<2, 0, 0>(t, m); msym_acc(m, a[0], 1.0, refn);
            mmat<0, 0, 0>(t, m0);
            mmat<1, 0, 0>(t, mu);
            double y1[5], y2[5], out[5];
            tangential_transport(m0, a[1], a[2], s.V, s.W, s.h, y1, y2, out);
            e_tan = fmax(e_tan, rel(out, ref));
            tangential_transport(mu, a[1], a[2], s.V, s.W, s.h, y1, y2, out);
            e_tanu = fmax(e_tanu, rel(out, refu));
            // the same through one product with mu plus the remaining row terms
            double bb[5], comb[5] = {0, 0, 0, 0, 0};
            for (int c = 0; c < 5; ++c) bb[c] = s.V * a[1][c] + s.W * a[2][c];
            msym_acc(mu, bb, 1.0, comb);
            tangential_rest(mu, a[1], a[2], s.h, 1.0, comb);
            e_rest = fmax(e_rest, rel(comb, refu));
            double y0[5] = {0, 0, 0, 0, 0}, yu[5] = {0, 0, 0, 0, 0};
            msym_acc(m0, a[0], 1.0, y0);
            msym_acc(mu, a[0], 1.0, yu);
            normal_transport(mu, y0, yu, a[0], s.U, s.h, out);
            e_nor = fmax(e_nor, rel(out, refn));
        }
    }
    printf("%.3e %.3e %.3e %.3e %.3e %.3e %.3e %.3e\n", e_tr, e_fx, e_jt, e_q2, e_tan, e_tanu, e_nor, e_rest);
    return 0;
}
"""


@pytest.fixture(scope="module")
def errors(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(ROCM_INC):
        pytest.skip("needs g++ and the ROCm headers")
    d = tmp_path_factory.mktemp("closed_forms")
    src, exe = d / "cf.cpp", d / "cf"
    src.write_text(SRC)
    r = subprocess.run([gxx, "-O2", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INC, "-I", CSRC,
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    names = ["transport", "euler_flux", "time_slope_moment", "second_transport", "tangential", "tangential_u",
             "normal_u2", "tangential_merged"]
    return dict(zip(names, map(float, out)))


@pytest.mark.parametrize("name", ["transport", "euler_flux", "time_slope_moment", "second_transport", "tangential",
                                  "tangential_u", "normal_u2", "tangential_merged"])
def test_closed_form_matches_moment_matrices(errors, name):
    assert errors[name] < 1e-12, errors
