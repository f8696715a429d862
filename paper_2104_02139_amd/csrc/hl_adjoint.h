// hl_adjoint.h -- reverse-mode (vector-Jacobian) products of the local
// pieces of one ADER-MOOD step with frozen dt and cascade choice: the
// neo-Hookean stress and impedance, the chain-rule divergence of the stress
// used by the predictor, simplex geometry, the corner matrix shape, the
// Crank-Nicolson and Euler updates of B and the nodal solve.  Each function
// accumulates (+=) into its output adjoints.  Host-callable for the
// finite-difference self-test.
#pragma once

#include "hl_device.h"

namespace hl {

// ------------------------------------------------------------ stress
// T_s = -p(J) d_s + mu J^{-5/3} (b_s - tr(b)/3 d_s), J = rho0 tau,
// p = -(K/2)(J - 1 + ln J / J); d_s = 1 for diagonal s.  Tb, bb in the
// 6-vector order (the adjoint of an off-diagonal stored component covers
// both matrix positions).
HL_HD void stress6_vjp(double rho0, double mu, double K, double tau, const double b[6], const double Tb[6],
                       double &taub, double bb[6], double &mub, double &Kb) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double cJ = cbrt(J);
    const double J53 = 1.0 / (J * cJ * cJ);
    const double J83 = J53 / J;
    const double tr3 = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
    const double sd = Tb[0] + Tb[1] + Tb[2];
    double dev_dot = 0.0;  // sum_s Tb_s dev_s
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const double dev = b[s] - (s < 3 ? tr3 : 0.0);
        dev_dot += Tb[s] * dev;
        bb[s] += mu * J53 * (Tb[s] - (s < 3 ? sd * (1.0 / 3.0) : 0.0));
    }
    const double mdp = 0.5 * K * (1.0 + (1.0 - lj) / (J * J));  // -dp/dJ
    taub += rho0 * (mdp * sd - (5.0 / 3.0) * mu * J83 * dev_dot);
    mub += J53 * dev_dot;
    Kb += 0.5 * (J - 1.0 + lj / J) * sd;
}

// z = a / tau = sqrt((K_t + 4 mu / 3) / tau), K_t = (K/2)(J + (1 - ln J)/J)
// (impedance() itself is with the stress in hl_device.h)
HL_HD void impedance_vjp(double rho0, double mu, double K, double tau, double zb, double &taub, double &mub,
                         double &Kb) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double Kt = 0.5 * K * (J + (1.0 - lj) / J);
    const double z = sqrt((Kt + (4.0 / 3.0) * mu) / tau);
    const double dKt = 0.5 * K * (1.0 + (lj - 2.0) / (J * J));
    const double f = zb / (2.0 * z * tau);
    taub += f * rho0 * dKt - zb * z / (2.0 * tau);
    mub += f * (4.0 / 3.0);
    Kb += f * 0.5 * (J + (1.0 - lj) / J);
}

// ------------------------------------------------- divergence of T
// divT_i = rho0 (q(J) gt_i - (5/3) mu J^{-8/3} sum_j dev_ij gt_j)
//          + mu J^{-5/3} (sum_j gB_{(ij), j} - (1/3) sum_k gB_{(kk), i}),
// q = -dp/dJ; gt = grad tau, gB[s][j] = d b_s / d x_j (6-vector order).
template <int D>
HL_HD void divT_fwd(double rho0, double mu, double K, double tau, const double b[6], const double gt[D],
                    const double gB[6][D], double out[D]) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double cJ = cbrt(J);
    const double J53 = 1.0 / (J * cJ * cJ);
    const double J83 = J53 / J;
    const double q = 0.5 * K * (1.0 + (1.0 - lj) / (J * J));
    const double tr3 = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double dev = b[sidx(i, j)] - (i == j ? tr3 : 0.0);
            s1 += dev * gt[j];
            s2 += gB[sidx(i, j)][j];
        }
        const double dtr = gB[0][i] + gB[1][i] + gB[2][i];
        out[i] = rho0 * (q * gt[i] - (5.0 / 3.0) * mu * J83 * s1) + mu * J53 * (s2 - dtr * (1.0 / 3.0));
    }
}

template <int D>
HL_HD void divT_vjp(double rho0, double mu, double K, double tau, const double b[6], const double gt[D],
                    const double gB[6][D], const double dv[D], double &taub, double bb[6], double gtb[D],
                    double gBb[6][D], double &mub, double &Kb) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double cJ = cbrt(J);
    const double J53 = 1.0 / (J * cJ * cJ);
    const double J83 = J53 / J;
    const double q = 0.5 * K * (1.0 + (1.0 - lj) / (J * J));
    const double dq = 0.5 * K * (2.0 * lj - 3.0) / (J * J * J);
    const double dJ83 = -(8.0 / 3.0) * J83 / J;
    const double dJ53 = -(5.0 / 3.0) * J53 / J;
    const double tr3 = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
    double dJsum = 0.0, trdev = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double dev = b[sidx(i, j)] - (i == j ? tr3 : 0.0);
            s1 += dev * gt[j];
            s2 += gB[sidx(i, j)][j];
            // d/d gt_j and d/d dev_ij
            gtb[j] += dv[i] * rho0 * ((i == j ? q : 0.0) - (5.0 / 3.0) * mu * J83 * dev);
            const double devb = -dv[i] * rho0 * (5.0 / 3.0) * mu * J83 * gt[j];
            bb[sidx(i, j)] += devb;
            if (i == j) trdev += devb;
            gBb[sidx(i, j)][j] += dv[i] * mu * J53;
        }
        const double dtr = gB[0][i] + gB[1][i] + gB[2][i];
        gBb[0][i] -= dv[i] * mu * J53 * (1.0 / 3.0);
        gBb[1][i] -= dv[i] * mu * J53 * (1.0 / 3.0);
        gBb[2][i] -= dv[i] * mu * J53 * (1.0 / 3.0);
        dJsum += dv[i] * (rho0 * (dq * gt[i] - (5.0 / 3.0) * mu * dJ83 * s1) + mu * dJ53 * (s2 - dtr * (1.0 / 3.0)));
        mub += dv[i] * (-rho0 * (5.0 / 3.0) * J83 * s1 + J53 * (s2 - dtr * (1.0 / 3.0)));
        Kb += dv[i] * rho0 * (q / K) * gt[i];
    }
    // dev_ii = b_ii - tr(b)/3: the trace part feeds every diagonal entry
    bb[0] -= trdev * (1.0 / 3.0);
    bb[1] -= trdev * (1.0 / 3.0);
    bb[2] -= trdev * (1.0 / 3.0);
    taub += rho0 * dJsum;
}

// --------------------------------------------- X -> L X + X L^T maps
// adjoint of the entries of lie_matrix3 / lie_matrix2 onto L
HL_HD void lie_matrix3_T(const double Mb[6][6], double Lb[3][3]) {
    Lb[0][0] += 2 * Mb[0][0] + Mb[3][3] + Mb[4][4];
    Lb[0][1] += 2 * Mb[0][3] + Mb[3][1] + Mb[4][5];
    Lb[0][2] += 2 * Mb[0][4] + Mb[3][5] + Mb[4][2];
    Lb[1][0] += 2 * Mb[1][3] + Mb[3][0] + Mb[5][4];
    Lb[1][1] += 2 * Mb[1][1] + Mb[3][3] + Mb[5][5];
    Lb[1][2] += 2 * Mb[1][5] + Mb[3][4] + Mb[5][2];
    Lb[2][0] += 2 * Mb[2][4] + Mb[4][0] + Mb[5][3];
    Lb[2][1] += 2 * Mb[2][5] + Mb[4][3] + Mb[5][1];
    Lb[2][2] += 2 * Mb[2][2] + Mb[4][4] + Mb[5][5];
}

HL_HD void lie_matrix2_T(const double Mb[3][3], double Lb[2][2]) {
    Lb[0][0] += 2 * Mb[0][0] + Mb[2][2];
    Lb[0][1] += 2 * Mb[0][2] + Mb[2][1];
    Lb[1][0] += 2 * Mb[1][2] + Mb[2][0];
    Lb[1][1] += 2 * Mb[1][1] + Mb[2][2];
}

// B update adjoints.  The 3D unknowns are the 6-vector; in 2D the three
// unknowns are slots (0, 1, 3) of the 6-vector (B33 == 1 is not a variable).
template <int D>
HL_HD void sym_slots(int slot[D == 3 ? 6 : 3]) {
    if (D == 3) {
        for (int s = 0; s < 6; ++s) slot[s] = s;
    } else {
        slot[0] = 0;
        slot[1] = 1;
        slot[2] = 3;
    }
}

template <int D>
HL_HD void lie_matrix(const double L[D][D], double M[D == 3 ? 6 : 3][D == 3 ? 6 : 3]);
template <>
HL_HD void lie_matrix<3>(const double L[3][3], double M[6][6]) { lie_matrix3(L, M); }
template <>
HL_HD void lie_matrix<2>(const double L[2][2], double M[3][3]) { lie_matrix2(L, M); }
template <int D>
HL_HD void lie_matrix_T(const double Mb[D == 3 ? 6 : 3][D == 3 ? 6 : 3], double Lb[D][D]);
template <>
HL_HD void lie_matrix_T<3>(const double Mb[6][6], double Lb[3][3]) { lie_matrix3_T(Mb, Lb); }
template <>
HL_HD void lie_matrix_T<2>(const double Mb[3][3], double Lb[2][2]) { lie_matrix2_T(Mb, Lb); }

// Crank-Nicolson: (I - h Mat(L1)) b1 = b + h Mat(L0) b.  Given b1 (the
// forward result) and b1b, accumulate bb (6-vector slots), L0b, L1b.
template <int D>
HL_HD void cn_vjp(const double b[6], const double L0[D][D], const double L1[D][D], double h, const double b1[6],
                  const double b1b[6], double bb[6], double L0b[D][D], double L1b[D][D]) {
    constexpr int N = D == 3 ? 6 : 3;
    int sl[N];
    sym_slots<D>(sl);
    double A[N][N], y[N];
    lie_matrix<D>(L1, A);
    double At[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) At[j][i] = (i == j ? 1.0 : 0.0) - h * A[i][j];
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = b1b[sl[i]];
    gepp<N>(At, y);  // y = A^{-T} b1b = adjoint of the right-hand side
    double Mb[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Mb[i][j] = h * y[i] * b1[sl[j]];
    lie_matrix_T<D>(Mb, L1b);
    double M0[N][N];
    lie_matrix<D>(L0, M0);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double t = y[j];
#pragma unroll
        for (int i = 0; i < N; ++i) t += h * M0[i][j] * y[i];
        bb[sl[j]] += t;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Mb[i][j] = h * y[i] * b[sl[j]];
    lie_matrix_T<D>(Mb, L0b);
}

// Euler: b1 = b + dt Mat(L) b
template <int D>
HL_HD void euler_vjp(const double b[6], const double L[D][D], double dt, const double b1b[6], double bb[6],
                     double Lb[D][D]) {
    constexpr int N = D == 3 ? 6 : 3;
    int sl[N];
    sym_slots<D>(sl);
    double M[N][N];
    lie_matrix<D>(L, M);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double t = b1b[sl[j]];
#pragma unroll
        for (int i = 0; i < N; ++i) t += dt * M[i][j] * b1b[sl[i]];
        bb[sl[j]] += t;
    }
    double Mb[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Mb[i][j] = dt * b1b[sl[i]] * b[sl[j]];
    lie_matrix_T<D>(Mb, Lb);
}

// ------------------------------------------------------------ geometry
// Adjoint of geom3 / geom2 (corner vectors C_k and measure V) onto the
// vertex positions.
HL_HD void cross_acc(const double a[3], const double b[3], double s, double o[3]) {
    o[0] += s * (a[1] * b[2] - a[2] * b[1]);
    o[1] += s * (a[2] * b[0] - a[0] * b[2]);
    o[2] += s * (a[0] * b[1] - a[1] * b[0]);
}

HL_HD void geom3_vjp(const double X[4][3], const double Cb[4][3], double Vb, double Xb[4][3]) {
    double e1[3], e2[3], e3[3], c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0}, c3[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e1[i] = X[1][i] - X[0][i];
        e2[i] = X[2][i] - X[0][i];
        e3[i] = X[3][i] - X[0][i];
    }
    double h1[3], h2[3], h3[3];  // C0 = -(C1 + C2 + C3)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        h1[i] = Cb[1][i] - Cb[0][i];
        h2[i] = Cb[2][i] - Cb[0][i];
        h3[i] = Cb[3][i] - Cb[0][i];
    }
    double b1[3] = {0, 0, 0}, b2[3] = {0, 0, 0}, b3[3] = {0, 0, 0};
    const double s6 = 1.0 / 6.0;
    // V = e1 . (e2 x e3) / 6
    cross_acc(e2, e3, Vb * s6, b1);
    cross_acc(e3, e1, Vb * s6, b2);
    cross_acc(e1, e2, Vb * s6, b3);
    // C1 = e2 x e3 / 6 ; C2 = e3 x e1 / 6 ; C3 = e1 x e2 / 6
    cross_acc(e3, h1, s6, b2);
    cross_acc(h1, e2, s6, b3);
    cross_acc(e1, h2, s6, b3);
    cross_acc(h2, e3, s6, b1);
    cross_acc(e2, h3, s6, b1);
    cross_acc(h3, e1, s6, b2);
    (void)c1;
    (void)c2;
    (void)c3;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Xb[1][i] += b1[i];
        Xb[2][i] += b2[i];
        Xb[3][i] += b3[i];
        Xb[0][i] -= b1[i] + b2[i] + b3[i];
    }
}

HL_HD void geom2_vjp(const double X[3][2], const double Cb[3][2], double Vb, double Xb[3][2]) {
    const double e1x = X[1][0] - X[0][0], e1y = X[1][1] - X[0][1];
    const double e2x = X[2][0] - X[0][0], e2y = X[2][1] - X[0][1];
    const double h1x = Cb[1][0] - Cb[0][0], h1y = Cb[1][1] - Cb[0][1];
    const double h2x = Cb[2][0] - Cb[0][0], h2y = Cb[2][1] - Cb[0][1];
    // C1 = (e2y, -e2x)/2, C2 = (-e1y, e1x)/2, V = (e1x e2y - e1y e2x)/2
    double b1x = 0.5 * h2y + 0.5 * Vb * e2y;
    double b1y = -0.5 * h2x - 0.5 * Vb * e2x;
    double b2x = -0.5 * h1y - 0.5 * Vb * e1y;
    double b2y = 0.5 * h1x + 0.5 * Vb * e1x;
    Xb[1][0] += b1x;
    Xb[1][1] += b1y;
    Xb[2][0] += b2x;
    Xb[2][1] += b2y;
    Xb[0][0] -= b1x + b2x;
    Xb[0][1] -= b1y + b2y;
}

template <int D>
HL_HD void geom_vjp(const double X[D + 1][D], const double Cb[D + 1][D], double Vb, double Xb[D + 1][D]);
template <>
HL_HD void geom_vjp<3>(const double X[4][3], const double Cb[4][3], double Vb, double Xb[4][3]) {
    geom3_vjp(X, Cb, Vb, Xb);
}
template <>
HL_HD void geom_vjp<2>(const double X[3][2], const double Cb[3][2], double Vb, double Xb[3][2]) {
    geom2_vjp(X, Cb, Vb, Xb);
}

// E = C C^T / |C| (stored symmetric, midx order); Eb stored adjoint
template <int D>
HL_HD void outer_norm_vjp(const double C[D], const double Eb[D == 3 ? 6 : 3], double Cb[D]) {
    double F[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) F[i][j] = (i == j) ? Eb[midx<D>(i, i)] : 0.5 * Eb[midx<D>(i, j)];
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) n2 += C[i] * C[i];
    const double n = sqrt(n2);
    double FC[D], cfc = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) s += F[i][j] * C[j];
        FC[i] = s;
        cfc += C[i] * s;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) Cb[i] += 2.0 * FC[i] / n - cfc * C[i] / (n * n2);
}

// --------------------------------------------------------- nodal solve
// v = P (P^T M P)^{-1} P^T r (P = I for a free node).  Given v (forward)
// and vb: rb = G vb and Mb = -sym(G vb v^T), G = P (P^T M P)^{-1} P^T.
template <int D>
HL_HD void node_solve_vjp(const double M[D == 3 ? 6 : 3], const double *P, int na, const double v[D],
                          const double vb[D], double rb[D], double Mb[D == 3 ? 6 : 3]) {
    double s[D];
#pragma unroll
    for (int i = 0; i < D; ++i) s[i] = 0.0;
    if (na == D) {
        double inv[D == 3 ? 6 : 3];
        if (D == 3)
            sym_inv3(M, inv);
        else
            sym_inv2(M, inv);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) t += inv[midx<D>(i, j)] * vb[j];
            s[i] = t;
        }
    } else if (na > 0) {
        double Ar[D][D], br[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) t += P[i * D + a] * vb[i];
            br[a] = t;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                double m = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) m += P[i * D + a] * M[midx<D>(i, j)] * P[j * D + c];
                Ar[a][c] = m;
            }
        }
        double al[D];
#pragma unroll
        for (int a = 0; a < D; ++a) al[a] = 0.0;
        if (na == 1) {
            al[0] = br[0] / Ar[0][0];
        } else {
            const double det = Ar[0][0] * Ar[1][1] - Ar[0][1] * Ar[1][0];
            al[0] = (Ar[1][1] * br[0] - Ar[0][1] * br[1]) / det;
            al[1] = (Ar[0][0] * br[1] - Ar[1][0] * br[0]) / det;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) t += (a < na) ? P[i * D + a] * al[a] : 0.0;
            s[i] = t;
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rb[i] += s[i];
#pragma unroll
        for (int j = i; j < D; ++j) Mb[midx<D>(i, j)] -= (i == j) ? s[i] * v[i] : s[i] * v[j] + s[j] * v[i];
    }
}

}  // namespace hl
