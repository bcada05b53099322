// CPU unit test of the library's hand-written and generated adjoints: each
// vector-Jacobian product of the device math is compared with central
// differences (fourth order) of the forward device function it reverses, on
// seeded random inputs; linear maps are compared through the dot-product
// identity <y-bar, A x> = <A^T y-bar, x>.  Built with g++ against a host
// stand-in of the HIP runtime header.  Prints one line per check:
//   <name> <worst relative error> <OK|FAIL> [branch counts]
#include <cstdio>
#include <functional>
#include <random>
#include <vector>

#include "hweno_vjp.h"

using namespace hw;
using Vec = std::vector<double>;
using Fwd = std::function<void(const Vec&, Vec&)>;             // x -> y
using Rev = std::function<void(const Vec&, const Vec&, Vec&)>; // (x, y-bar) -> x-bar

static std::mt19937_64 rng(2608);
static double nrm() { return std::normal_distribution<double>(0.0, 1.0)(rng); }
static int failures = 0;

static Consts consts(bool linear) {
    Consts K{};
    K.gamma = 1.4;
    K.gm1 = 0.4;
    K.igm1 = 2.5;
    K.Pr = 0.72;
    K.gPr = 1.4 / 0.72;
    K.mu_ref = 0.01;
    K.mu_exp = 0.0;
    K.T_ref = 1.0;
    K.eps_pp = 1e-12;
    K.eps_weno = 1e-8;
    K.linear = linear ? 1 : 0;
    K.dx = K.dy = 0.1;
    K.idx = K.idy = 10.0;
    return K;
}

// worst over coordinates of |fd - adjoint| / max(1, |fd|, |adjoint|)
static double fd_error(const Fwd& f, const Rev& r, const Vec& x, int ny, double hrel = 1e-4) {
    Vec yb(ny), xb(x.size(), 0.0), y(ny);
    for (auto& v : yb) v = nrm();
    r(x, yb, xb);
    double worst = 0.0;
    for (size_t q = 0; q < x.size(); ++q) {
        const double h = hrel * fmax(1e-2, fabs(x[q]));
        auto at = [&](double s) {
            Vec z = x;
            z[q] += s * h;
            f(z, y);
            double d = 0.0;
            for (int k = 0; k < ny; ++k) d += yb[k] * y[k];
            return d;
        };
        const double fd = (8.0 * (at(1) - at(-1)) - (at(2) - at(-2))) / (12.0 * h);
        const double e = fabs(fd - xb[q]) / fmax(1.0, fmax(fabs(fd), fabs(xb[q])));
        worst = std::isfinite(xb[q]) ? fmax(worst, e) : INFINITY;
    }
    return worst;
}

static void report(const char* name, double err, double tol, const char* extra = "") {
    const bool ok = err <= tol;
    if (!ok) ++failures;
    printf("%s %.3e %s%s\n", name, err, ok ? "OK" : "FAIL", extra);
}

// a random admissible 2D state: rho in (0.2, 2), moderate velocity, p in (0.2, 2)
static void state2(double* U, double vel = 1.0, double rho_scale = 1.0) {
    const double r = rho_scale * (0.2 + 1.8 * std::uniform_real_distribution<double>()(rng));
    const double u = vel * nrm(), v = vel * nrm();
    const double p = 0.2 + 1.8 * std::uniform_real_distribution<double>()(rng);
    U[0] = r;
    U[1] = r * u;
    U[2] = r * v;
    U[3] = p / 0.4 + 0.5 * r * (u * u + v * v);
}

static void linear_checks() {
    // p0 maps, point evaluations, moments: <yb, A x> = <A^T yb, x>
    auto dot_identity = [](const char* name, int nx, int ny, auto fwd, auto rev) {
        double worst = 0.0;
        for (int t = 0; t < 20; ++t) {
            Vec x(nx), y(ny), yb(ny), xb(nx, 0.0);
            for (auto& v : x) v = nrm();
            for (auto& v : yb) v = nrm();
            fwd(x.data(), y.data());
            rev(yb.data(), xb.data());
            double a = 0.0, b = 0.0, s = 0.0;
            for (int k = 0; k < ny; ++k) { a += yb[k] * y[k]; s += fabs(yb[k] * y[k]); }
            for (int k = 0; k < nx; ++k) { b += xb[k] * x[k]; s += fabs(xb[k] * x[k]); }
            worst = fmax(worst, fabs(a - b) / s);
        }
        report(name, worst, 1e-14);
    };
    dot_identity("p0_2d_T", 17, 15, [](const double* a, double* c) { hweno_gen::p0_2d(a, c); },
                 [](const double* cb, double* ab) { adj::p0_2d_T(cb, ab); });
    dot_identity("p0_1d_T", 5, 5, [](const double* a, double* c) { hweno_gen::p0_1d(a, c); },
                 [](const double* cb, double* ab) { adj::p0_1d_T(cb, ab); });
    dot_identity("xface_T", 15, 6, [](const double* C, double* y) { eval_xface(C, y); },
                 [](const double* yb, double* Cb) { adj::xface_T(yb, Cb); });
    dot_identity("yface_T", 15, 6, [](const double* C, double* y) { eval_yface(C, y); },
                 [](const double* yb, double* Cb) { adj::yface_T(yb, Cb); });
    dot_identity("vol_T", 15, 9, [](const double* C, double* y) { eval_vol(C, y); },
                 [](const double* yb, double* Cb) { adj::vol_T(yb, Cb); });
    dot_identity("lgl_T", 5, 4, [](const double* C, double* y) { eval1d(C, y); },
                 [](const double* yb, double* Cb) { adj::lgl_T(yb, Cb); });
    dot_identity("moment_xi_T", 15, 1, [](const double* C, double* y) { y[0] = moment_xi(C); },
                 [](const double* yb, double* Cb) { moment_xi_T(yb[0], Cb); });
    dot_identity("moment_eta_T", 15, 1, [](const double* C, double* y) { y[0] = moment_eta(C); },
                 [](const double* yb, double* Cb) { moment_eta_T(yb[0], Cb); });
    dot_identity("moment1d_T", 5, 1, [](const double* C, double* y) { y[0] = moment1d(C); },
                 [](const double* yb, double* Cb) { moment1d_T(yb[0], Cb); });
}

static void reconstruction_checks() {
    double w2 = 0.0, w1 = 0.0, s2 = 0.0, s1 = 0.0, l2 = 0.0;
    for (int t = 0; t < 30; ++t) {
        // smooth-ish and rough stencils: mean + noise of random amplitude
        const double amp = t % 3 == 0 ? 1.0 : 0.05;
        const Consts K = consts(false), KL = consts(true);
        Vec a(17), a1(5), c(15), c1(5);
        for (auto& v : a) v = 1.0 + amp * nrm();
        for (auto& v : a1) v = 1.0 + amp * nrm();
        for (auto& v : c) v = nrm();
        for (auto& v : c1) v = nrm();
        w2 = fmax(w2, fd_error([&](const Vec& x, Vec& y) { hweno2d(x.data(), K, y.data()); },
                               [&](const Vec& x, const Vec& yb, Vec& xb) { hweno2d_vjp(x.data(), K, yb.data(), xb.data()); },
                               a, 15));
        l2 = fmax(l2, fd_error([&](const Vec& x, Vec& y) { hweno2d(x.data(), KL, y.data()); },
                               [&](const Vec& x, const Vec& yb, Vec& xb) { hweno2d_vjp(x.data(), KL, yb.data(), xb.data()); },
                               a, 15));
        w1 = fmax(w1, fd_error([&](const Vec& x, Vec& y) { hweno1d(x.data(), K, y.data()); },
                               [&](const Vec& x, const Vec& yb, Vec& xb) { hweno1d_vjp(x.data(), K, yb.data(), xb.data()); },
                               a1, 5));
        s2 = fmax(s2, fd_error([&](const Vec& x, Vec& y) { y[0] = hweno_gen::sobolev_2d(x.data()); },
                               [&](const Vec& x, const Vec& yb, Vec& xb) {
                                   double g[15];
                                   adj::sobolev_2d_grad(x.data(), g);
                                   for (int k = 0; k < 15; ++k) xb[k] += yb[0] * g[k];
                               }, c, 1, 0.3));   // quadratic: any step is exact up to rounding
        s1 = fmax(s1, fd_error([&](const Vec& x, Vec& y) { y[0] = hweno_gen::sobolev_1d(x.data()); },
                               [&](const Vec& x, const Vec& yb, Vec& xb) {
                                   double g[5];
                                   adj::sobolev_1d_grad(x.data(), g);
                                   for (int k = 0; k < 5; ++k) xb[k] += yb[0] * g[k];
                               }, c1, 1, 0.3));
    }
    report("hweno2d_vjp", w2, 1e-7);
    report("hweno2d_vjp_linear", l2, 1e-7);
    report("hweno1d_vjp", w1, 1e-7);
    report("sobolev_2d_grad", s2, 1e-7);
    report("sobolev_1d_grad", s1, 1e-7);
}

// inputs of the 2D flux functions: U[4], s[6], mu
static void flux_checks() {
    double f0 = 0.0, f1 = 0.0, p2 = 0.0, pr2 = 0.0, e0 = 0.0, e1 = 0.0;
    double sp[2] = {0.0, 0.0};
    int branch[2][2] = {{0, 0}, {0, 0}};
    for (int t = 0; t < 60; ++t) {
        Vec x(11);
        // every third sample: near-vacuum density and steep gradients, where
        // the positivity bound beta_PP exceeds |u_n| + c
        const bool steep = t % 3 == 2;
        state2(x.data(), 1.0, steep ? 1e-3 : 1.0);
        for (int z = 0; z < 6; ++z) x[4 + z] = (steep ? 300.0 : 1.0) * nrm();
        x[10] = 0.01 * (1.0 + std::uniform_real_distribution<double>()(rng));
        auto withmu = [](const Vec& v) { Consts K = consts(false); K.mu_ref = v[10]; return K; };
        auto fwdflux = [&](int d) {
            return [&, d](const Vec& v, Vec& y) {
                const Consts K = withmu(v);
                if (d == 0) flux2<0>(K, v.data(), v.data() + 4, y.data());
                else flux2<1>(K, v.data(), v.data() + 4, y.data());
            };
        };
        auto revflux = [&](int d) {
            return [&, d](const Vec& v, const Vec& yb, Vec& xb) {
                const Consts K = withmu(v);
                double mub = 0.0;
                if (d == 0) flux2_vjp<0>(K, v.data(), v.data() + 4, v[10], yb.data(), xb.data(), xb.data() + 4, mub);
                else flux2_vjp<1>(K, v.data(), v.data() + 4, v[10], yb.data(), xb.data(), xb.data() + 4, mub);
                xb[10] += mub;
            };
        };
        f0 = fmax(f0, fd_error(fwdflux(0), revflux(0), x, 4));
        f1 = fmax(f1, fd_error(fwdflux(1), revflux(1), x, 4));
        for (int d = 0; d < 2; ++d) {
            // the branch of the maximum taken at this point
            const Consts K = withmu(x);
            const double s_all = d == 0 ? speed2<0>(K, x.data(), x.data() + 4) : speed2<1>(K, x.data(), x.data() + 4);
            const double r = x[0];
            const double p = pressure2(K, r, x[1], x[2], x[3]);
            const double ac = fabs(x[1 + d] / r) + sqrt(K.gamma * p / r);
            // acoustic branch if the bound equals |u_d| + c up to rounding
            ++branch[d][ac >= s_all * (1.0 - 1e-12) ? 0 : 1];
            sp[d] = fmax(sp[d], fd_error(
                [&, d](const Vec& v, Vec& y) {
                    const Consts Kv = withmu(v);
                    y[0] = d == 0 ? speed2<0>(Kv, v.data(), v.data() + 4) : speed2<1>(Kv, v.data(), v.data() + 4);
                },
                [&, d](const Vec& v, const Vec& yb, Vec& xb) {
                    const Consts Kv = withmu(v);
                    double mub = 0.0;
                    if (d == 0) speed2_vjp<0>(Kv, v.data(), v.data() + 4, v[10], yb[0], xb.data(), xb.data() + 4, mub);
                    else speed2_vjp<1>(Kv, v.data(), v.data() + 4, v[10], yb[0], xb.data(), xb.data() + 4, mub);
                    xb[10] += mub;
                }, x, 1));
        }
        Vec u4(x.begin(), x.begin() + 4);
        p2 = fmax(p2, fd_error([](const Vec& v, Vec& y) { y[0] = pressure2(consts(false), v[0], v[1], v[2], v[3]); },
                               [](const Vec& v, const Vec& yb, Vec& xb) { adj::pres2_vjp(consts(false), v.data(), yb[0], xb.data()); },
                               u4, 1));
        pr2 = fmax(pr2, fd_error([](const Vec& v, Vec& y) {
                                     const double u = v[1] / v[0], w = v[2] / v[0];
                                     y[0] = u;
                                     y[1] = w;
                                     y[2] = v[3] / v[0] - 0.5 * (u * u + w * w);
                                 },
                                 [](const Vec& v, const Vec& yb, Vec& xb) { adj::prim2_vjp(v.data(), yb.data(), xb.data()); },
                                 u4, 3));
        if (!steep) {
            for (int b = 0; b < 2; ++b) {
                for (int k = 0; k < 4; ++k) {
                    Vec lb(4), rb(4);
                    for (auto& v : lb) v = nrm();
                    for (auto& v : rb) v = nrm();
                    const double e = fd_error(
                        [&](const Vec& v, Vec& y) {
                            double L[4], R[4];
                            eig2_rows(consts(false), v.data(), b, k, L, R);
                            y[0] = 0.0;
                            for (int c = 0; c < 4; ++c) y[0] += L[c] * lb[c] + R[c] * rb[c];
                        },
                        [&](const Vec& v, const Vec& yb, Vec& xb) {
                            double l[4], r[4];
                            for (int c = 0; c < 4; ++c) { l[c] = yb[0] * lb[c]; r[c] = yb[0] * rb[c]; }
                            if (b == 0) adj::eig2_vjp_0(consts(false), v.data(), k, l, r, xb.data());
                            else adj::eig2_vjp_1(consts(false), v.data(), k, l, r, xb.data());
                        }, u4, 1);
                    if (b == 0) e0 = fmax(e0, e);
                    else e1 = fmax(e1, e);
                }
            }
        }
    }
    char br[2][64];
    for (int d = 0; d < 2; ++d) snprintf(br[d], 64, " branches %d %d", branch[d][0], branch[d][1]);
    report("flux2_vjp_0", f0, 1e-7);
    report("flux2_vjp_1", f1, 1e-7);
    report("speed2_vjp_0", sp[0], 1e-7, br[0]);
    report("speed2_vjp_1", sp[1], 1e-7, br[1]);
    report("pres2_vjp", p2, 1e-7);
    report("prim2_vjp", pr2, 1e-7);
    report("eig2_vjp_0", e0, 1e-7);
    report("eig2_vjp_1", e1, 1e-7);
}

// 1D: inputs U[3], u_x, e_x, mu
static void flux1_checks() {
    double f = 0.0, sp = 0.0, p1 = 0.0, pr1 = 0.0, e1 = 0.0;
    int branch[2] = {0, 0};
    for (int t = 0; t < 60; ++t) {
        const bool steep = t % 3 == 2;
        double U4[4];
        state2(U4, 1.0, steep ? 1e-3 : 1.0);
        Vec x = {U4[0], U4[1], U4[3] - 0.5 * U4[2] * U4[2] / U4[0],
                 (steep ? 300.0 : 1.0) * nrm(), (steep ? 300.0 : 1.0) * nrm(),
                 0.01 * (1.0 + std::uniform_real_distribution<double>()(rng))};
        auto withmu = [](const Vec& v) { Consts K = consts(false); K.mu_ref = v[5]; return K; };
        f = fmax(f, fd_error([&](const Vec& v, Vec& y) { flux1(withmu(v), v.data(), v[3], v[4], y.data()); },
                             [&](const Vec& v, const Vec& yb, Vec& xb) {
                                 double mub = 0.0;
                                 adj::flux1_vjp(withmu(v), v.data(), v[3], v[4], v[5], yb.data(), xb.data(), xb[3], xb[4], mub);
                                 xb[5] += mub;
                             }, x, 3));
        // branch of the maximum, as the 1D reverse kernel selects it
        auto rev_speed = [&](const Vec& v, const Vec& yb, Vec& xb) {
            const Consts K = withmu(v);
            const double r = v[0], u = v[1] / r;
            const double p = pressure1(K, r, v[1], v[2]);
            const double ac = fabs(u) + sqrt(K.gamma * p / r);
            const double all = speed1(K, v.data(), v[3], v[4]);
            const double sgu = u > 0 ? 1.0 : (u < 0 ? -1.0 : 0.0);
            double mub = 0.0;
            if (ac >= all) {
                adj::speed1_ac_vjp(K, v.data(), sgu, yb[0], xb.data());
            } else {
                const double q = -K.gamma * v[5] * v[4] / K.Pr;
                const double sgq = q > 0 ? 1.0 : (q < 0 ? -1.0 : 0.0);
                adj::speed1_bpp_vjp(K, v.data(), v[3], v[4], v[5], sgu, sgq, yb[0], xb.data(), xb[3], xb[4], mub);
            }
            xb[5] += mub;
        };
        {
            const Consts K = withmu(x);
            const double p = pressure1(K, x[0], x[1], x[2]);
            const double ac = fabs(x[1] / x[0]) + sqrt(K.gamma * p / x[0]);
            ++branch[ac >= speed1(K, x.data(), x[3], x[4]) ? 0 : 1];
        }
        sp = fmax(sp, fd_error([&](const Vec& v, Vec& y) { y[0] = speed1(withmu(v), v.data(), v[3], v[4]); },
                               rev_speed, x, 1));
        Vec u3(x.begin(), x.begin() + 3);
        p1 = fmax(p1, fd_error([](const Vec& v, Vec& y) { y[0] = pressure1(consts(false), v[0], v[1], v[2]); },
                               [](const Vec& v, const Vec& yb, Vec& xb) { adj::pres1_vjp(consts(false), v.data(), yb[0], xb.data()); },
                               u3, 1));
        pr1 = fmax(pr1, fd_error([](const Vec& v, Vec& y) {
                                     const double u = v[1] / v[0];
                                     y[0] = u;
                                     y[1] = v[2] / v[0] - 0.5 * u * u;
                                 },
                                 [](const Vec& v, const Vec& yb, Vec& xb) { adj::prim1_vjp(v.data(), yb.data(), xb.data()); },
                                 u3, 2));
        if (!steep) {
            Vec lb(9), rb(9);
            for (auto& v : lb) v = nrm();
            for (auto& v : rb) v = nrm();
            e1 = fmax(e1, fd_error(
                [&](const Vec& v, Vec& y) {
                    Eig1 e;
                    eig1(consts(false), v.data(), e);
                    y[0] = 0.0;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) y[0] += e.L[i][j] * lb[3 * i + j] + e.R[i][j] * rb[3 * i + j];
                },
                [&](const Vec& v, const Vec& yb, Vec& xb) {
                    double l[9], r[9];
                    for (int q = 0; q < 9; ++q) { l[q] = yb[0] * lb[q]; r[q] = yb[0] * rb[q]; }
                    adj::eig1_vjp(consts(false), v.data(), l, r, xb.data());
                }, u3, 1));
        }
    }
    char br[64];
    snprintf(br, 64, " branches %d %d", branch[0], branch[1]);
    report("flux1_vjp", f, 1e-7);
    report("speed1_vjp", sp, 1e-7, br);
    report("pres1_vjp", p1, 1e-7);
    report("prim1_vjp", pr1, 1e-7);
    report("eig1_vjp", e1, 1e-7);
}

int main() {
    linear_checks();
    reconstruction_checks();
    flux_checks();
    flux1_checks();
    printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
