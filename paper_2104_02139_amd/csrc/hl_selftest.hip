// hl_selftest.hip -- host-side finite-difference checks of the local
// vector-Jacobian products in hl_adjoint.h (built as libhl_selftest.so; the
// tests call it without a GPU).  Each entry returns the largest relative
// mismatch between <vjp(ybar), e_i> and the central difference of
// <ybar, f(x)> along e_i, over `trials` random inputs.
#include <cmath>
#include <cstdint>
#include <random>

#include "hl_adjoint.h"

namespace {

using namespace hl;

struct Rng {
    std::mt19937_64 g;
    explicit Rng(uint64_t s) : g(s) {}
    double u(double a, double b) { return std::uniform_real_distribution<double>(a, b)(g); }
};

void rand_spd6(Rng &r, double b[6], double amp) {
    double A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = (i == j ? 1.0 : 0.0) + amp * r.u(-1, 1);
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[i][k] * A[j][k];
            B[i][j] = s;
        }
    b[0] = B[0][0];
    b[1] = B[1][1];
    b[2] = B[2][2];
    b[3] = B[0][1];
    b[4] = B[0][2];
    b[5] = B[1][2];
}

double relerr(const double *a, const double *b, int n) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i) {
        num = std::fmax(num, std::fabs(a[i] - b[i]));
        den = std::fmax(den, std::fabs(b[i]));
    }
    return den > 0 ? num / den : num;
}

}  // namespace


// T(tau, b, mu, K): inputs (tau, b[6], mu, K)
extern "C" double st_stress(int trials) {
    Rng r(1);
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        const double rho0 = r.u(500, 3000), mu = r.u(1e5, 1e7), K = r.u(1e6, 1e8);
        double x[9];
        x[0] = r.u(0.8, 1.2) / rho0;
        rand_spd6(r, x + 1, 0.2);
        x[7] = mu;
        x[8] = K;
        double yb[6];
        for (int s = 0; s < 6; ++s) yb[s] = r.u(-1, 1);
        double g[9] = {0};
        stress6_vjp(rho0, x[7], x[8], x[0], x + 1, yb, g[0], g + 1, g[7], g[8]);
        double fd[9];
        for (int i = 0; i < 9; ++i) {
            const double h = 1e-6 * std::fmax(std::fabs(x[i]), 1e-3);
            double xp[9], xm[9], Tp[6], Tm[6];
            for (int k = 0; k < 9; ++k) xp[k] = xm[k] = x[k];
            xp[i] += h;
            xm[i] -= h;
            stress6(rho0, xp[7], xp[8], xp[0], xp + 1, Tp);
            stress6(rho0, xm[7], xm[8], xm[0], xm + 1, Tm);
            double s = 0;
            for (int k = 0; k < 6; ++k) s += yb[k] * (Tp[k] - Tm[k]);
            fd[i] = s / (2 * h);
        }
        // compare component-wise on a common scale per input
        for (int i = 0; i < 9; ++i) {
            const double sc = std::fmax(std::fabs(fd[i]), 1e-300);
            worst = std::fmax(worst, std::fabs(g[i] - fd[i]) / sc);
        }
    }
    return worst;
}

extern "C" double st_impedance(int trials) {
    Rng r(2);
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        const double rho0 = r.u(500, 3000);
        double x[3] = {r.u(0.7, 1.3) / rho0, r.u(1e5, 1e7), r.u(1e6, 1e8)};
        const double zb = r.u(-1, 1);
        double g[3] = {0, 0, 0};
        impedance_vjp(rho0, x[1], x[2], x[0], zb, g[0], g[1], g[2]);
        for (int i = 0; i < 3; ++i) {
            const double h = 1e-6 * std::fabs(x[i]);
            double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
            xp[i] += h;
            xm[i] -= h;
            const double fd = zb * (impedance(rho0, xp[1], xp[2], xp[0]) - impedance(rho0, xm[1], xm[2], xm[0])) / (2 * h);
            worst = std::fmax(worst, std::fabs(g[i] - fd) / std::fmax(std::fabs(fd), 1e-300));
        }
    }
    return worst;
}

template <int D>
static double st_divT_impl(int trials) {
    Rng r(3 + D);
    double worst = 0;
    constexpr int NI = 1 + 6 + D + 6 * D + 2;  // tau, b, gt, gB, mu, K
    for (int t = 0; t < trials; ++t) {
        const double rho0 = r.u(500, 3000);
        double x[NI];
        x[0] = r.u(0.8, 1.2) / rho0;
        rand_spd6(r, x + 1, 0.2);
        if (D == 2) {
            x[3] = 1.0;
            x[5] = 0.0;
            x[6] = 0.0;
        }
        for (int j = 0; j < D; ++j) x[7 + j] = r.u(-1, 1) * x[0];
        for (int k = 0; k < 6 * D; ++k) x[7 + D + k] = r.u(-1, 1);
        if (D == 2)
            for (int j = 0; j < D; ++j) x[7 + D + 2 * D + j] = x[7 + D + 4 * D + j] = x[7 + D + 5 * D + j] = 0.0;
        x[NI - 2] = r.u(1e5, 1e7);
        x[NI - 1] = r.u(1e6, 1e8);
        double dv[D];
        for (int i = 0; i < D; ++i) dv[i] = r.u(-1, 1);
        auto f = [&](const double *xx, double out[D]) {
            double gB[6][D];
            for (int s = 0; s < 6; ++s)
                for (int j = 0; j < D; ++j) gB[s][j] = xx[7 + D + s * D + j];
            divT_fwd<D>(rho0, xx[NI - 2], xx[NI - 1], xx[0], xx + 1, xx + 7, gB, out);
        };
        double g[NI] = {0};
        {
            double gB[6][D], gBb[6][D] = {};
            for (int s = 0; s < 6; ++s)
                for (int j = 0; j < D; ++j) gB[s][j] = x[7 + D + s * D + j];
            divT_vjp<D>(rho0, x[NI - 2], x[NI - 1], x[0], x + 1, x + 7, gB, dv, g[0], g + 1, g + 7, gBb, g[NI - 2],
                        g[NI - 1]);
            for (int s = 0; s < 6; ++s)
                for (int j = 0; j < D; ++j) g[7 + D + s * D + j] = gBb[s][j];
        }
        double fd[NI], scale = 0;
        for (int i = 0; i < NI; ++i) {
            const double h = 1e-6 * std::fmax(std::fabs(x[i]), 1e-4);
            double xp[NI], xm[NI], op[D], om[D];
            for (int k = 0; k < NI; ++k) xp[k] = xm[k] = x[k];
            xp[i] += h;
            xm[i] -= h;
            f(xp, op);
            f(xm, om);
            double s = 0;
            for (int k = 0; k < D; ++k) s += dv[k] * (op[k] - om[k]);
            fd[i] = s / (2 * h);
            scale = std::fmax(scale, std::fabs(fd[i] * x[i]));
        }
        // in 2D the fixed slots (b33, b13, b23 and their gradients) are not inputs
        for (int i = 0; i < NI; ++i) {
            if (D == 2 && (i == 3 || i == 5 || i == 6)) continue;
            if (D == 2 && i >= 7 + D && i < 7 + D + 6 * D) {
                const int s = (i - 7 - D) / D;
                if (s == 2 || s == 4 || s == 5) continue;
            }
            worst = std::fmax(worst, std::fabs(g[i] - fd[i]) * std::fmax(std::fabs(x[i]), 1e-4) / scale);
        }
    }
    return worst;
}
extern "C" double st_divT3(int trials) { return st_divT_impl<3>(trials); }
extern "C" double st_divT2(int trials) { return st_divT_impl<2>(trials); }

// Crank-Nicolson and Euler B updates: inputs (b slots, L0, L1)
template <int D>
static double st_bupdate_impl(int trials, int cn) {
    constexpr int N = D == 3 ? 6 : 3;
    Rng r(10 + D + 2 * cn);
    int sl[N];
    sym_slots<D>(sl);
    double worst = 0;
    constexpr int NI = N + 2 * D * D;
    for (int t = 0; t < trials; ++t) {
        double b6[6];
        rand_spd6(r, b6, 0.2);
        if (D == 2) {
            b6[2] = 1;
            b6[4] = b6[5] = 0;
        }
        double x[NI];
        for (int i = 0; i < N; ++i) x[i] = b6[sl[i]];
        for (int k = 0; k < 2 * D * D; ++k) x[N + k] = r.u(-1, 1);
        const double h = r.u(0.01, 0.1);
        auto f = [&](const double *xx, double out[6]) {
            double bb[6] = {b6[0], b6[1], b6[2], b6[3], b6[4], b6[5]};
            for (int i = 0; i < N; ++i) bb[sl[i]] = xx[i];
            double L0[D][D], L1[D][D];
            for (int i = 0; i < D; ++i)
                for (int j = 0; j < D; ++j) {
                    L0[i][j] = xx[N + i * D + j];
                    L1[i][j] = xx[N + D * D + i * D + j];
                }
            if (cn) {
                cn_update<D>(bb, L0, L1, h, out);
            } else {
                double M[N][N];
                lie_matrix<D>(L0, M);
                for (int s = 0; s < 6; ++s) out[s] = bb[s];
                for (int i = 0; i < N; ++i) {
                    double y = 0;
                    for (int j = 0; j < N; ++j) y += M[i][j] * bb[sl[j]];
                    out[sl[i]] = bb[sl[i]] + 2 * h * y;
                }
            }
        };
        double b1[6], yb[6] = {0, 0, 0, 0, 0, 0};
        f(x, b1);
        for (int i = 0; i < N; ++i) yb[sl[i]] = r.u(-1, 1);
        double bb[6] = {0, 0, 0, 0, 0, 0}, L0b[D][D] = {}, L1b[D][D] = {};
        double bx[6] = {b6[0], b6[1], b6[2], b6[3], b6[4], b6[5]};
        double L0[D][D], L1[D][D];
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                L0[i][j] = x[N + i * D + j];
                L1[i][j] = x[N + D * D + i * D + j];
            }
        if (cn)
            cn_vjp<D>(bx, L0, L1, h, b1, yb, bb, L0b, L1b);
        else
            euler_vjp<D>(bx, L0, 2 * h, yb, bb, L0b);
        double g[NI], fd[NI];
        for (int i = 0; i < N; ++i) g[i] = bb[sl[i]];
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                g[N + i * D + j] = L0b[i][j];
                g[N + D * D + i * D + j] = L1b[i][j];
            }
        for (int i = 0; i < NI; ++i) {
            const double hh = 1e-6;
            double xp[NI], xm[NI], op[6], om[6];
            for (int k = 0; k < NI; ++k) xp[k] = xm[k] = x[k];
            xp[i] += hh;
            xm[i] -= hh;
            f(xp, op);
            f(xm, om);
            double s = 0;
            for (int k = 0; k < 6; ++k) s += yb[k] * (op[k] - om[k]);
            fd[i] = s / (2 * hh);
        }
        worst = std::fmax(worst, relerr(g, fd, NI));
    }
    return worst;
}
extern "C" double st_cn3(int trials) { return st_bupdate_impl<3>(trials, 1); }
extern "C" double st_cn2(int trials) { return st_bupdate_impl<2>(trials, 1); }
extern "C" double st_euler3(int trials) { return st_bupdate_impl<3>(trials, 0); }
extern "C" double st_euler2(int trials) { return st_bupdate_impl<2>(trials, 0); }

// geometry: X -> (C, V)
template <int D>
static double st_geom_impl(int trials) {
    Rng r(20 + D);
    constexpr int NV = D + 1, NI = NV * D;
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        double X[NV][D];
        for (int k = 0; k < NV; ++k)
            for (int i = 0; i < D; ++i) X[k][i] = (k == i + 1 ? 1.0 : 0.0) + 0.2 * r.u(-1, 1);
        double Cb[NV][D], Vb = r.u(-1, 1);
        for (int k = 0; k < NV; ++k)
            for (int i = 0; i < D; ++i) Cb[k][i] = r.u(-1, 1);
        double Xb[NV][D] = {};
        geom_vjp<D>(X, Cb, Vb, Xb);
        double g[NI], fd[NI];
        for (int k = 0; k < NV; ++k)
            for (int i = 0; i < D; ++i) g[k * D + i] = Xb[k][i];
        for (int q = 0; q < NI; ++q) {
            const double h = 1e-6;
            double Xp[NV][D], Xm[NV][D];
            for (int k = 0; k < NV; ++k)
                for (int i = 0; i < D; ++i) Xp[k][i] = Xm[k][i] = X[k][i];
            Xp[q / D][q % D] += h;
            Xm[q / D][q % D] -= h;
            Geo<D> gp, gm;
            geom<D>(Xp, gp);
            geom<D>(Xm, gm);
            double s = Vb * (gp.V - gm.V);
            for (int k = 0; k < NV; ++k)
                for (int i = 0; i < D; ++i) s += Cb[k][i] * (gp.C[k][i] - gm.C[k][i]);
            fd[q] = s / (2 * h);
        }
        worst = std::fmax(worst, relerr(g, fd, NI));
    }
    return worst;
}
extern "C" double st_geom3(int trials) { return st_geom_impl<3>(trials); }
extern "C" double st_geom2(int trials) { return st_geom_impl<2>(trials); }

// C -> C C^T / |C|
template <int D>
static double st_outer_impl(int trials) {
    Rng r(30 + D);
    constexpr int NMS = D == 3 ? 6 : 3;
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        double C[D], Eb[NMS];
        for (int i = 0; i < D; ++i) C[i] = r.u(-1, 1);
        for (int s = 0; s < NMS; ++s) Eb[s] = r.u(-1, 1);
        double g[D] = {};
        outer_norm_vjp<D>(C, Eb, g);
        double fd[D];
        auto f = [&](const double *c) {
            double n = 0;
            for (int i = 0; i < D; ++i) n += c[i] * c[i];
            n = std::sqrt(n);
            double s = 0;
            for (int i = 0; i < D; ++i)
                for (int j = i; j < D; ++j) s += Eb[midx<D>(i, j)] * c[i] * c[j] / n;
            return s;
        };
        for (int i = 0; i < D; ++i) {
            const double h = 1e-6;
            double cp[D], cm[D];
            for (int k = 0; k < D; ++k) cp[k] = cm[k] = C[k];
            cp[i] += h;
            cm[i] -= h;
            fd[i] = (f(cp) - f(cm)) / (2 * h);
        }
        worst = std::fmax(worst, relerr(g, fd, D));
    }
    return worst;
}
extern "C" double st_outer3(int trials) { return st_outer_impl<3>(trials); }
extern "C" double st_outer2(int trials) { return st_outer_impl<2>(trials); }

// nodal solve v = P (P^T M P)^{-1} P^T r with `na` allowed directions
template <int D>
static double st_node_impl(int trials, int na) {
    Rng r(40 + D + 3 * na);
    constexpr int NMS = D == 3 ? 6 : 3, NI = NMS + D;
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        // SPD M
        double A[D][D], Mf[D][D];
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) A[i][j] = (i == j ? 2.0 : 0.0) + 0.3 * r.u(-1, 1);
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                double s = 0;
                for (int k = 0; k < D; ++k) s += A[i][k] * A[j][k];
                Mf[i][j] = s;
            }
        double x[NI];
        for (int i = 0; i < D; ++i)
            for (int j = i; j < D; ++j) x[midx<D>(i, j)] = Mf[i][j];
        for (int i = 0; i < D; ++i) x[NMS + i] = r.u(-1, 1);
        // orthonormal P (first na columns of a random rotation)
        double P[D * D] = {};
        {
            double Q[D][D];
            for (int i = 0; i < D; ++i)
                for (int j = 0; j < D; ++j) Q[i][j] = r.u(-1, 1);
            for (int j = 0; j < D; ++j) {
                for (int k = 0; k < j; ++k) {
                    double s = 0;
                    for (int i = 0; i < D; ++i) s += Q[i][j] * Q[i][k];
                    for (int i = 0; i < D; ++i) Q[i][j] -= s * Q[i][k];
                }
                double n = 0;
                for (int i = 0; i < D; ++i) n += Q[i][j] * Q[i][j];
                n = std::sqrt(n);
                for (int i = 0; i < D; ++i) Q[i][j] /= n;
            }
            for (int i = 0; i < D; ++i)
                for (int a = 0; a < na; ++a) P[i * D + a] = Q[i][a];
        }
        auto f = [&](const double *xx, double v[D]) {
            double Ar[D][D] = {}, br[D] = {};
            for (int a = 0; a < na; ++a) {
                for (int i = 0; i < D; ++i) br[a] += P[i * D + a] * xx[NMS + i];
                for (int c = 0; c < na; ++c)
                    for (int i = 0; i < D; ++i)
                        for (int j = 0; j < D; ++j) Ar[a][c] += P[i * D + a] * xx[midx<D>(i, j)] * P[j * D + c];
            }
            double al[D] = {};
            if (na == 1) al[0] = br[0] / Ar[0][0];
            if (na == 2) {
                double det = Ar[0][0] * Ar[1][1] - Ar[0][1] * Ar[1][0];
                al[0] = (Ar[1][1] * br[0] - Ar[0][1] * br[1]) / det;
                al[1] = (Ar[0][0] * br[1] - Ar[1][0] * br[0]) / det;
            }
            if (na == 3) {
                double inv[6];
                sym_inv3(xx, inv);
                for (int i = 0; i < 3; ++i) {
                    double s = 0;
                    for (int j = 0; j < 3; ++j) s += inv[midx<3>(i, j)] * xx[NMS + j];
                    v[i] = s;
                }
                return;
            }
            for (int i = 0; i < D; ++i) {
                double s = 0;
                for (int a = 0; a < na; ++a) s += P[i * D + a] * al[a];
                v[i] = s;
            }
        };
        double v[D], vb[D];
        f(x, v);
        for (int i = 0; i < D; ++i) vb[i] = r.u(-1, 1);
        double rb[D] = {}, Mb[NMS] = {};
        node_solve_vjp<D>(x, P, na == D ? D : na, v, vb, rb, Mb);
        double g[NI], fd[NI];
        for (int s = 0; s < NMS; ++s) g[s] = Mb[s];
        for (int i = 0; i < D; ++i) g[NMS + i] = rb[i];
        for (int i = 0; i < NI; ++i) {
            const double h = 1e-6;
            double xp[NI], xm[NI], vp[D], vm[D];
            for (int k = 0; k < NI; ++k) xp[k] = xm[k] = x[k];
            xp[i] += h;
            xm[i] -= h;
            f(xp, vp);
            f(xm, vm);
            double s = 0;
            for (int k = 0; k < D; ++k) s += vb[k] * (vp[k] - vm[k]);
            fd[i] = s / (2 * h);
        }
        worst = std::fmax(worst, relerr(g, fd, NI));
    }
    return worst;
}
extern "C" double st_node3(int trials, int na) { return st_node_impl<3>(trials, na); }
extern "C" double st_node2(int trials, int na) { return st_node_impl<2>(trials, na); }

