// hl_device.h -- device-side building blocks of the ADER-MOOD step:
// simplex geometry, the neo-Hookean law and small dense solves, all FP64.
//
// Symmetric 3x3 tensors are held as s[6] = (11, 22, 33, 12, 13, 23).  In 2D
// (plane strain) s[2] = 1 and s[4] = s[5] = 0 always; vectors carry D
// components.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hl {

template <int D>
struct Dims {
    static constexpr int NV = D + 1;                 // nodes per simplex
    static constexpr int NB = D == 3 ? 6 : 3;        // stored B components
    static constexpr int NW = 1 + D + NB;            // reconstructed scalars
    static constexpr int NMS = D == 3 ? 6 : 3;       // symmetric DxD entries
    static constexpr int CW = D == 3 ? 10 : 6;       // corner record (padded)
    // node aggregate record: n, Sy, Syy, SW, SyW, rho min, rho max
    static constexpr int O_SY = 1;
    static constexpr int O_SYY = 1 + D;
    static constexpr int O_SW = 1 + D + NMS;
    static constexpr int O_SYW = O_SW + NW;
    static constexpr int O_RMM = O_SYW + D * NW;
    static constexpr int NA = O_RMM + 2;             // 52 (3D) / 26 (2D)
    static constexpr int GR = D == 3 ? 16 : 10;      // gather record: W, centroid, pad
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

__device__ __forceinline__ void geom3(const double X[4][3], Geo<3> &g) {
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

__device__ __forceinline__ void geom2(const double X[3][2], Geo<2> &g) {
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
__device__ __forceinline__ void geom(const double X[D + 1][D], Geo<D> &g);
template <>
__device__ __forceinline__ void geom<3>(const double X[4][3], Geo<3> &g) { geom3(X, g); }
template <>
__device__ __forceinline__ void geom<2>(const double X[3][2], Geo<2> &g) { geom2(X, g); }

// ------------------------------------------------------- constitutive law
// Neo-Hookean law (Section 2.2.4) with the bulk modulus K in the
// volumetric energy: p = -(K/2)(J - 1 + ln J / J), T = -p I + mu J^{-5/3}
// dev(B), J = rho0 tau.
__device__ __forceinline__ void stress6(double rho0, double mu, double K, double tau,
                                        const double b[6], double t[6]) {
    double J = rho0 * tau;
    double lj = log(J);
    double p = -0.5 * K * (J - 1.0 + lj / J);
    double c = cbrt(J);
    double s = mu / (J * c * c);
    double tr3 = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
    t[0] = s * (b[0] - tr3) - p;
    t[1] = s * (b[1] - tr3) - p;
    t[2] = s * (b[2] - tr3) - p;
    t[3] = s * b[3];
    t[4] = s * b[4];
    t[5] = s * b[5];
}

// a = sqrt(tau (K_t + 4 mu / 3)), K_t = (K/2)(J + (1 - ln J)/J) = -J dp/dJ
__device__ __forceinline__ double sound(double rho0, double mu, double K, double tau) {
    double J = rho0 * tau;
    double Kt = 0.5 * K * (J + (1.0 - log(J)) / J);
    return sqrt(tau * (Kt + (4.0 / 3.0) * mu));
}

__device__ __forceinline__ double det6(const double b[6]) {
    return b[0] * (b[1] * b[2] - b[5] * b[5]) - b[3] * (b[3] * b[2] - b[5] * b[4]) +
           b[4] * (b[3] * b[5] - b[1] * b[4]);
}

// ------------------------------------------------------------- solves
// inverse of a symmetric DxD matrix given in midx storage; returns det
__device__ __forceinline__ double sym_inv3(const double a[6], double inv[6]) {
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

__device__ __forceinline__ double sym_inv2(const double a[3], double inv[3]) {
    double det = a[0] * a[1] - a[2] * a[2];
    double r = 1.0 / det;
    inv[0] = a[1] * r;
    inv[1] = a[0] * r;
    inv[2] = -a[2] * r;
    return det;
}

// Dense n x n solve with partial pivoting, fully unrolled; A row-major.
template <int N>
__device__ __forceinline__ void gepp(double A[N][N], double b[N]) {
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
        // swap rows col <-> piv
#pragma unroll
        for (int r = col + 1; r < N; ++r) {
            if (piv == r) {
#pragma unroll
                for (int k = col; k < N; ++k) {
                    double t = A[col][k];
                    A[col][k] = A[r][k];
                    A[r][k] = t;
                }
                double t = b[col];
                b[col] = b[r];
                b[r] = t;
            }
        }
        double inv = 1.0 / A[col][col];
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
        b[r] = s / A[r][r];
    }
}

// Crank-Nicolson update of B (Section 3.4, eq. CN_B with dt/2 on both
// sides):  X - h (L1 X + X L1^T) = Bn + h (Ln Bn + Bn Ln^T),  h = dt/2,
// for the symmetric unknown X.  L are DxD (L_ij = dv_i/dx_j).
template <int D>
__device__ __forceinline__ void cn_update(const double b[6], const double Ln[D][D],
                                          const double L1[D][D], double h, double out[6]) {
    constexpr int N = D == 3 ? 6 : 3;
    // unknown slot s -> (i, j)
    constexpr int PI[6] = {0, 1, 2, 0, 0, 1};
    constexpr int PJ[6] = {0, 1, 2, 1, 2, 2};
    constexpr int PI2[3] = {0, 1, 0};
    constexpr int PJ2[3] = {0, 1, 1};
    double B3[3][3] = {{b[0], b[3], b[4]}, {b[3], b[1], b[5]}, {b[4], b[5], b[2]}};
    double L0[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double L1f[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            L0[i][j] = Ln[i][j];
            L1f[i][j] = L1[i][j];
        }
    double A[N][N], r[N];
#pragma unroll
    for (int row = 0; row < N; ++row) {
        const int i = D == 3 ? PI[row] : PI2[row];
        const int j = D == 3 ? PJ[row] : PJ2[row];
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) y += L0[i][k] * B3[k][j] + B3[i][k] * L0[j][k];
        r[row] = B3[i][j] + h * y;
#pragma unroll
        for (int col = 0; col < N; ++col) {
            const int a = D == 3 ? PI[col] : PI2[col];
            const int c = D == 3 ? PJ[col] : PJ2[col];
            // coefficient of X_ac (= X_ca) in (L X + X L^T)_ij
            double m = L1f[i][a] * (j == c ? 1.0 : 0.0) + L1f[j][c] * (i == a ? 1.0 : 0.0);
            if (a != c) m += L1f[i][c] * (j == a ? 1.0 : 0.0) + L1f[j][a] * (i == c ? 1.0 : 0.0);
            A[row][col] = (row == col ? 1.0 : 0.0) - h * m;
        }
    }
    gepp<N>(A, r);
    if (D == 3) {
#pragma unroll
        for (int s = 0; s < 6; ++s) out[s] = r[s < N ? s : 0];
    } else {
        out[0] = r[0];
        out[1] = r[1];
        out[2] = 1.0;
        out[3] = r[2];
        out[4] = 0.0;
        out[5] = 0.0;
    }
}

}  // namespace hl
