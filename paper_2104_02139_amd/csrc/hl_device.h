// hl_device.h -- device-side building blocks of the ADER-MOOD step:
// simplex geometry, the neo-Hookean law and small dense solves, all FP64.
//
// Symmetric 3x3 tensors are held as s[6] = (11, 22, 33, 12, 13, 23).  In 2D
// (plane strain) s[2] = 1 and s[4] = s[5] = 0 always; vectors carry D
// components.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

// callable from kernels and, for the self-tests, from host code
#define HL_HD __host__ __device__ __forceinline__

namespace hl {

template <int D>
struct Dims {
    static constexpr int NV = D + 1;                 // nodes per simplex
    static constexpr int NB = D == 3 ? 6 : 3;        // stored B components
    static constexpr int NW = 1 + D + NB;            // reconstructed scalars
    static constexpr int NMS = D == 3 ? 6 : 3;       // symmetric DxD entries
    static constexpr int CW = D == 3 ? 9 : 5;        // corner record: M_cp, r_cp
    // node aggregate record: n, Sy, Syy, SW, SyW, rho min, rho max, W min,
    // W max
    static constexpr int O_SY = 1;
    static constexpr int O_SYY = 1 + D;
    static constexpr int O_SW = 1 + D + NMS;
    static constexpr int O_SYW = O_SW + NW;
    static constexpr int O_RMM = O_SYW + D * NW;
    static constexpr int NA_BASE = O_RMM + 2;        // 52 (3D) / 26 (2D)
    // min / max of each W over the node's cells (limited cascade level only)
    static constexpr int O_WMIN = NA_BASE;
    static constexpr int O_WMAX = O_WMIN + NW;
    static constexpr int NA = O_WMAX + NW;           // 72 (3D) / 38 (2D)
    static constexpr int GR = D == 3 ? 16 : 10;      // gather record: W, centroid, eps, pad
    // the stiffened gas (R31) also reconstructs eps = e - |v|^2 / 2: slot
    // G_EPS of the gather record; sum eps and sum y eps in the aggregates
    // after the base record (the W bounds of the limited level are not
    // used with it)
    static constexpr int G_EPS = NW + D;
    static constexpr int O_SE = NA_BASE;
    static constexpr int O_SYE = NA_BASE + 1;
    static constexpr int NA_SG = NA_BASE + 1 + D + (D == 3 ? 0 : 1);  // whole pairs
};

// index of the symmetric entry (i, j) in the 6-vector
__host__ __device__ constexpr int sidx(int i, int j) {
    return i == j ? i : (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5));
}

// index in the DxD symmetric storage used by corner records: 3D uses the
// 6-vector order, 2D uses (11, 22, 12)
template <int D>
__host__ __device__ constexpr int midx(int i, int j) {
    return D == 3 ? sidx(i, j) : (i == j ? i : 2);
}

// ---------------------------------------------------------------- geometry
// Corner vectors C_k = dV/dx_k of a simplex (Section 3.1, eq. def_lcpncp)
// from edge cross products; V is the signed measure.
template <int D>
struct Geo {
    double V;
    double C[D + 1][D];
    double cn[D + 1];   // |C_k|
};

HL_HD void geom3(const double X[4][3], Geo<3> &g) {
    double e1[3], e2[3], e3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        e1[i] = X[1][i] - X[0][i];
        e2[i] = X[2][i] - X[0][i];
        e3[i] = X[3][i] - X[0][i];
    }
    const double s = 1.0 / 6.0;
    g.C[1][0] = s * (e2[1] * e3[2] - e2[2] * e3[1]);
    g.C[1][1] = s * (e2[2] * e3[0] - e2[0] * e3[2]);
    g.C[1][2] = s * (e2[0] * e3[1] - e2[1] * e3[0]);
    g.C[2][0] = s * (e3[1] * e1[2] - e3[2] * e1[1]);
    g.C[2][1] = s * (e3[2] * e1[0] - e3[0] * e1[2]);
    g.C[2][2] = s * (e3[0] * e1[1] - e3[1] * e1[0]);
    g.C[3][0] = s * (e1[1] * e2[2] - e1[2] * e2[1]);
    g.C[3][1] = s * (e1[2] * e2[0] - e1[0] * e2[2]);
    g.C[3][2] = s * (e1[0] * e2[1] - e1[1] * e2[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) g.C[0][i] = -(g.C[1][i] + g.C[2][i] + g.C[3][i]);
    g.V = e1[0] * g.C[1][0] + e1[1] * g.C[1][1] + e1[2] * g.C[1][2];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        g.cn[k] = sqrt(g.C[k][0] * g.C[k][0] + g.C[k][1] * g.C[k][1] + g.C[k][2] * g.C[k][2]);
}

HL_HD void geom2(const double X[3][2], Geo<2> &g) {
    double e1x = X[1][0] - X[0][0], e1y = X[1][1] - X[0][1];
    double e2x = X[2][0] - X[0][0], e2y = X[2][1] - X[0][1];
    g.C[1][0] = 0.5 * e2y;
    g.C[1][1] = -0.5 * e2x;
    g.C[2][0] = -0.5 * e1y;
    g.C[2][1] = 0.5 * e1x;
    g.C[0][0] = -(g.C[1][0] + g.C[2][0]);
    g.C[0][1] = -(g.C[1][1] + g.C[2][1]);
    g.V = e1x * g.C[1][0] + e1y * g.C[1][1];
#pragma unroll
    for (int k = 0; k < 3; ++k) g.cn[k] = sqrt(g.C[k][0] * g.C[k][0] + g.C[k][1] * g.C[k][1]);
}

template <int D>
HL_HD void geom(const double X[D + 1][D], Geo<D> &g);
template <>
HL_HD void geom<3>(const double X[4][3], Geo<3> &g) { geom3(X, g); }
template <>
HL_HD void geom<2>(const double X[3][2], Geo<2> &g) { geom2(X, g); }

// ------------------------------------------------------- constitutive law
// Neo-Hookean law (Section 2.2.4) with the bulk modulus K in the
// volumetric energy: p = -(K/2)(J - 1 + ln J / J), T = -p I + mu J^{-5/3}
// dev(B), J = rho0 tau.
HL_HD void stress6(double rho0, double mu, double K, double tau,
                                        const double b[6], double t[6]) {
    // one reciprocal of J: ln J / J and J^{-5/3} = J^{1/3} (1/J)^2
    double J = rho0 * tau;
    double rJ = 1.0 / J;
    double lj = log(J);
    double p = -0.5 * K * (J - 1.0 + lj * rJ);
    double c = cbrt(J);
    double s = mu * c * rJ * rJ;
    double tr3 = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
    t[0] = s * (b[0] - tr3) - p;
    t[1] = s * (b[1] - tr3) - p;
    t[2] = s * (b[2] - tr3) - p;
    t[3] = s * b[3];
    t[4] = s * b[4];
    t[5] = s * b[5];
}

// Shear energy family (eq. familiy_energies) with the stress of eq. cst:
// T = -p I + (mu / J) [-a dev(Bbar) - c I2(Bbar) dev(Bbar^-1)], c = (1+a)/3,
// Bbar = J^{-2/3} B, I2 the second principal invariant.  a = -1 is the
// neo-Hookean law of stress6.  6-vectors in sidx order.
HL_HD double inv2_6(const double b[6]) {
    const double tr = b[0] + b[1] + b[2];
    const double tr2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + 2.0 * (b[3] * b[3] + b[4] * b[4] + b[5] * b[5]);
    return 0.5 * (tr * tr - tr2);
}

HL_HD double sym_inv3(const double a[6], double inv[6]);

HL_HD void stress6_family(double rho0, double mu, double K, double a, double tau, const double b[6],
                          double t[6]) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double p = -0.5 * K * (J - 1.0 + lj / J);
    const double cJ = cbrt(J);
    const double s = 1.0 / (cJ * cJ);
    double bb[6], bi[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) bb[q] = s * b[q];
    sym_inv3(bb, bi);
    const double tr = bb[0] + bb[1] + bb[2], tri = bi[0] + bi[1] + bi[2];
    const double c = (1.0 + a) / 3.0;
    const double I2 = inv2_6(bb);
    const double mj = mu / J;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double e = q < 3 ? 1.0 : 0.0;
        t[q] = mj * (-a * (bb[q] - e * tr / 3.0) - c * I2 * (bi[q] - e * tri / 3.0)) - e * p;
    }
}

// Derivative of stress6_family along (dtau, db): with dJ = rho0 dtau,
// dBbar = J^{-2/3} dB - (2/3)(dJ/J) Bbar, d(Bbar^-1) = -Bbar^-1 dBbar Bbar^-1,
// dI2 = tr(Bbar) tr(dBbar) - Bbar : dBbar,
// dT = -p'(J) dJ I - (dJ/J) T_0 + (mu/J) [-a dev(dBbar)
//      - c (dI2 dev(Bbar^-1) + I2 dev(d(Bbar^-1)))].
HL_HD void stress6_dir_family(double rho0, double mu, double K, double a, double tau, const double b[6],
                              double dtau, const double db[6], double dt[6]) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double dpdJ = -0.5 * K * (1.0 + (1.0 - lj) / (J * J));
    const double dJ = rho0 * dtau;
    const double cJ = cbrt(J);
    const double s = 1.0 / (cJ * cJ);
    double bb[6], dbb[6], bi[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        bb[q] = s * b[q];
        dbb[q] = s * db[q] - (2.0 / 3.0) * (dJ / J) * bb[q];
    }
    sym_inv3(bb, bi);
    const double Bi[3][3] = {{bi[0], bi[3], bi[4]}, {bi[3], bi[1], bi[5]}, {bi[4], bi[5], bi[2]}};
    const double dB[3][3] = {{dbb[0], dbb[3], dbb[4]}, {dbb[3], dbb[1], dbb[5]}, {dbb[4], dbb[5], dbb[2]}};
    double tmp[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double u = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) u += dB[i][k] * Bi[k][j];
            tmp[i][j] = u;
        }
    double dbi[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int i = q < 3 ? q : (q == 5 ? 1 : 0);
        const int j = q < 3 ? q : (q == 3 ? 1 : 2);
        double u = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) u += Bi[i][k] * tmp[k][j];
        dbi[q] = -u;
    }
    const double c = (1.0 + a) / 3.0;
    const double I2 = inv2_6(bb);
    const double trB = bb[0] + bb[1] + bb[2], trdB = dbb[0] + dbb[1] + dbb[2];
    const double BdB = bb[0] * dbb[0] + bb[1] * dbb[1] + bb[2] * dbb[2] +
                       2.0 * (bb[3] * dbb[3] + bb[4] * dbb[4] + bb[5] * dbb[5]);
    const double dI2 = trB * trdB - BdB;
    const double trBi = bi[0] + bi[1] + bi[2], trdBi = dbi[0] + dbi[1] + dbi[2];
    const double mj = mu / J;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double e = q < 3 ? 1.0 : 0.0;
        const double T0 = mj * (-a * (bb[q] - e * trB / 3.0) - c * I2 * (bi[q] - e * trBi / 3.0));
        const double dsh = -a * (dbb[q] - e * trdB / 3.0) -
                           c * (dI2 * (bi[q] - e * trBi / 3.0) + I2 * (dbi[q] - e * trdBi / 3.0));
        dt[q] = -dpdJ * dJ * e - (dJ / J) * T0 + mj * dsh;
    }
}

// specific free energy Psi_v + Psi_s of the family (energy diagnostics)
HL_HD double free_energy_family(double rho0, double mu, double K, double a, double tau, const double b[6]) {
    const double J = rho0 * tau;
    const double lj = log(J);
    const double cJ = cbrt(J);
    const double s = 1.0 / (cJ * cJ);
    const double I1b = (b[0] + b[1] + b[2]) * s;
    const double psi_v = K / (4.0 * rho0) * ((J - 1.0) * (J - 1.0) + lj * lj);
    if (a == -1.0) return psi_v + mu / (2.0 * rho0) * (I1b - 3.0);
    double bb[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) bb[q] = s * b[q];
    const double I2b = inv2_6(bb);
    return psi_v + mu / (4.0 * rho0) * (-2.0 * a * (I1b - 3.0) + (1.0 + a) / 3.0 * (I2b * I2b - 9.0));
}

// a = sqrt(tau (K_t + 4 mu / 3)), K_t = (K/2)(J + (1 - ln J)/J) = -J dp/dJ
// ------------------------------------------------- stiffened gas (R31)
// The stiffened gas (eq. EOS_stiffened_gas) in place of the volumetric
// energy: with Psi_s the shear energy of the family (the family's energy
// with K = 0) and eps the specific internal energy,
//   p = (gamma - 1) (eps - Psi_s) / tau - gamma p_inf,
//   T = T_s - p I (T_s the family's stress with K = 0),
//   a^2 = tau (gamma (p + p_inf) + 4 mu / 3).
HL_HD double shear_energy6(double rho0, double mu, double a, double tau, const double b[6]) {
    return free_energy_family(rho0, mu, 0.0, a, tau, b);
}

// derivative of Psi_s along (dtau, db): mu/(4 rho0) [-2a dI1b + (2/3)(1+a) I2b dI2b]
HL_HD double shear_energy_dir6(double rho0, double mu, double a, double tau, const double b[6], double dtau,
                               const double db[6]) {
    const double J = rho0 * tau, dJ = rho0 * dtau;
    const double cJ = cbrt(J);
    const double s = 1.0 / (cJ * cJ);
    double bb[6], dbb[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        bb[q] = s * b[q];
        dbb[q] = s * db[q] - (2.0 / 3.0) * (dJ / J) * bb[q];
    }
    const double trB = bb[0] + bb[1] + bb[2], trdB = dbb[0] + dbb[1] + dbb[2];
    const double BdB = bb[0] * dbb[0] + bb[1] * dbb[1] + bb[2] * dbb[2] +
                       2.0 * (bb[3] * dbb[3] + bb[4] * dbb[4] + bb[5] * dbb[5]);
    const double I2 = inv2_6(bb);
    return mu / (4.0 * rho0) * (-2.0 * a * trdB + (2.0 / 3.0) * (1.0 + a) * I2 * (trB * trdB - BdB));
}

HL_HD double sg_pressure6(double rho0, double mu, double a, double gam, double pinf, double tau, const double b[6],
                          double eps) {
    return (gam - 1.0) * (eps - shear_energy6(rho0, mu, a, tau, b)) / tau - gam * pinf;
}

HL_HD void stress6_sg(double rho0, double mu, double a, double gam, double pinf, double tau, const double b[6],
                      double eps, double t[6]) {
    stress6_family(rho0, mu, 0.0, a, tau, b, t);
    const double p = sg_pressure6(rho0, mu, a, gam, pinf, tau, b, eps);
#pragma unroll
    for (int q = 0; q < 3; ++q) t[q] -= p;
}

HL_HD double sound_sg(double rho0, double mu, double a, double gam, double pinf, double tau, const double b[6],
                      double eps) {
    return sqrt(tau * (gam * (sg_pressure6(rho0, mu, a, gam, pinf, tau, b, eps) + pinf) + (4.0 / 3.0) * mu));
}

// derivative of stress6_sg along (dtau, db, deps):
//   dT = dT_s - dp I, dp = (gamma - 1) [(deps - dPsi_s) / tau - (eps - Psi_s) dtau / tau^2]
HL_HD void stress6_dir_sg(double rho0, double mu, double a, double gam, double pinf, double tau, const double b[6],
                          double eps, double dtau, const double db[6], double deps, double dt[6]) {
    stress6_dir_family(rho0, mu, 0.0, a, tau, b, dtau, db, dt);
    const double psi = shear_energy6(rho0, mu, a, tau, b);
    const double dpsi = shear_energy_dir6(rho0, mu, a, tau, b, dtau, db);
    const double dp = (gam - 1.0) * ((deps - dpsi) / tau - (eps - psi) * dtau / (tau * tau));
#pragma unroll
    for (int q = 0; q < 3; ++q) dt[q] -= dp;
}

HL_HD double sound(double rho0, double mu, double K, double tau) {
    double J = rho0 * tau;
    double Kt = 0.5 * K * (J + (1.0 - log(J)) * (1.0 / J));
    return sqrt(tau * (Kt + (4.0 / 3.0) * mu));
}

// acoustic impedance per unit volume, z = a / tau = a rho0 / J
HL_HD double impedance(double rho0, double mu, double K, double tau) {
    const double rJ = 1.0 / (rho0 * tau);
    return sound(rho0, mu, K, tau) * (rho0 * rJ);
}

HL_HD double det6(const double b[6]) {
    return b[0] * (b[1] * b[2] - b[5] * b[5]) - b[3] * (b[3] * b[2] - b[5] * b[4]) +
           b[4] * (b[3] * b[5] - b[1] * b[4]);
}

// ------------------------------------------------------------- solves
// inverse of a symmetric DxD matrix given in midx storage; returns det
HL_HD double sym_inv3(const double a[6], double inv[6]) {
    double c00 = a[1] * a[2] - a[5] * a[5];
    double c01 = a[4] * a[5] - a[3] * a[2];
    double c02 = a[3] * a[5] - a[4] * a[1];
    double det = a[0] * c00 + a[3] * c01 + a[4] * c02;
    double r = 1.0 / det;
    inv[0] = c00 * r;
    inv[3] = c01 * r;
    inv[4] = c02 * r;
    inv[1] = (a[0] * a[2] - a[4] * a[4]) * r;
    inv[5] = (a[3] * a[4] - a[0] * a[5]) * r;
    inv[2] = (a[0] * a[1] - a[3] * a[3]) * r;
    return det;
}

HL_HD double sym_inv2(const double a[3], double inv[3]) {
    double det = a[0] * a[1] - a[2] * a[2];
    double r = 1.0 / det;
    inv[0] = a[1] * r;
    inv[1] = a[0] * r;
    inv[2] = -a[2] * r;
    return det;
}

// Dense n x n solve with partial pivoting, fully unrolled; A row-major.
template <int N>
HL_HD void gepp(double A[N][N], double b[N]) {
    double rp[N];  // reciprocals of the pivots, reused by the back substitution
#pragma unroll
    for (int col = 0; col < N; ++col) {
        // pivot search
        int piv = col;
        double best = fabs(A[col][col]);
#pragma unroll
        for (int r = col + 1; r < N; ++r) {
            double v = fabs(A[r][col]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        // swap rows col <-> piv with selects (no dynamic register indexing)
#pragma unroll
        for (int r = col + 1; r < N; ++r) {
            const bool sw = piv == r;
#pragma unroll
            for (int k = col; k < N; ++k) {
                const double u = A[col][k], t = A[r][k];
                A[col][k] = sw ? t : u;
                A[r][k] = sw ? u : t;
            }
            const double u = b[col], t = b[r];
            b[col] = sw ? t : u;
            b[r] = sw ? u : t;
        }
        const double inv = 1.0 / A[col][col];
        rp[col] = inv;
#pragma unroll
        for (int r = col + 1; r < N; ++r) {
            double f = A[r][col] * inv;
#pragma unroll
            for (int k = col + 1; k < N; ++k) A[r][k] -= f * A[col][k];
            b[r] -= f * b[col];
        }
    }
#pragma unroll
    for (int r = N - 1; r >= 0; --r) {
        double s = b[r];
#pragma unroll
        for (int k = r + 1; k < N; ++k) s -= A[r][k] * b[k];
        b[r] = s * rp[r];
    }
}

// Matrix of X -> L X + X L^T on the symmetric components, unknowns in the
// order (11, 22, 33, 12, 13, 23) in 3D and (11, 22, 12) in 2D; entry
// (row (i,j), col (a,c)) is the coefficient of X_ac in
// (L X + X L^T)_ij = sum_k L_ik X_kj + X_ik L_jk.
HL_HD void lie_matrix3(const double L[3][3], double M[6][6]) {
    const double l00 = L[0][0], l01 = L[0][1], l02 = L[0][2];
    const double l10 = L[1][0], l11 = L[1][1], l12 = L[1][2];
    const double l20 = L[2][0], l21 = L[2][1], l22 = L[2][2];
    M[0][0] = 2 * l00; M[0][1] = 0;       M[0][2] = 0;       M[0][3] = 2 * l01;   M[0][4] = 2 * l02;   M[0][5] = 0;
    M[1][0] = 0;       M[1][1] = 2 * l11; M[1][2] = 0;       M[1][3] = 2 * l10;   M[1][4] = 0;         M[1][5] = 2 * l12;
    M[2][0] = 0;       M[2][1] = 0;       M[2][2] = 2 * l22; M[2][3] = 0;         M[2][4] = 2 * l20;   M[2][5] = 2 * l21;
    M[3][0] = l10;     M[3][1] = l01;     M[3][2] = 0;       M[3][3] = l00 + l11; M[3][4] = l12;       M[3][5] = l02;
    M[4][0] = l20;     M[4][1] = 0;       M[4][2] = l02;     M[4][3] = l21;       M[4][4] = l00 + l22; M[4][5] = l01;
    M[5][0] = 0;       M[5][1] = l21;     M[5][2] = l12;     M[5][3] = l20;       M[5][4] = l10;       M[5][5] = l11 + l22;
}

HL_HD void lie_matrix2(const double L[2][2], double M[3][3]) {
    M[0][0] = 2 * L[0][0]; M[0][1] = 0;           M[0][2] = 2 * L[0][1];
    M[1][0] = 0;           M[1][1] = 2 * L[1][1]; M[1][2] = 2 * L[1][0];
    M[2][0] = L[1][0];     M[2][1] = L[0][1];     M[2][2] = L[0][0] + L[1][1];
}

// Crank-Nicolson update of B (Section 3.4, eq. CN_B with dt/2 on both
// sides):  X - h (L1 X + X L1^T) = Bn + h (Ln Bn + Bn Ln^T),  h = dt/2,
// for the symmetric unknown X.  L are DxD (L_ij = dv_i/dx_j).
HL_HD void cn_update3(const double b[6], const double Ln[3][3], const double L1[3][3], double h,
                                           double out[6]) {
    double A[6][6], r[6];
    lie_matrix3(Ln, A);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) y += A[i][j] * b[j];
        r[i] = b[i] + h * y;
    }
    lie_matrix3(L1, A);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - h * A[i][j];
    gepp<6>(A, r);
#pragma unroll
    for (int s = 0; s < 6; ++s) out[s] = r[s];
}

HL_HD void cn_update2(const double b[6], const double Ln[2][2], const double L1[2][2], double h,
                                           double out[6]) {
    double A[3][3], r[3];
    const double bs[3] = {b[0], b[1], b[3]};
    lie_matrix2(Ln, A);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) y += A[i][j] * bs[j];
        r[i] = bs[i] + h * y;
    }
    lie_matrix2(L1, A);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - h * A[i][j];
    gepp<3>(A, r);
    out[0] = r[0];
    out[1] = r[1];
    out[2] = 1.0;
    out[3] = r[2];
    out[4] = 0.0;
    out[5] = 0.0;
}

template <int D>
HL_HD void cn_update(const double b[6], const double Ln[D][D], const double L1[D][D], double h,
                                          double out[6]);
template <>
HL_HD void cn_update<3>(const double b[6], const double Ln[3][3], const double L1[3][3], double h,
                                             double out[6]) {
    cn_update3(b, Ln, L1, h, out);
}
template <>
HL_HD void cn_update<2>(const double b[6], const double Ln[2][2], const double L1[2][2], double h,
                                             double out[6]) {
    cn_update2(b, Ln, L1, h, out);
}

}  // namespace hl
