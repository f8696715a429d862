/*
 * hl_oracle.c -- FP64 CPU oracle for one cell-centred Lagrangian
 * ADER-MOOD time step of neo-Hookean hyperelasticity on simplicial meshes
 * (Boscheri, Loubere & Maire, "A cell-centered Lagrangian ADER-MOOD finite
 * volume scheme on unstructured meshes for a class of hyper-elasticity
 * models", arXiv 2104.02139).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, serial
 * reference that the HIP library is compared with.  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * Built plain (serial) for the tests.  The loops over output cells and
 * nodes carry OpenMP pragmas for the timed CPU baseline: every output is
 * computed by one thread in the same order, sums over cells (the
 * diagnostics) stay serial and the minima / maxima do not depend on the
 * order, so the threaded build gives bitwise the serial results.
 *
 * Every quantity is FP64.  Tensors are held as full 3x3 arrays; in 2D
 * (plane strain) the third row and column of L and G are zero, B33 == 1 and
 * the in-plane vectors carry a zero third component.  Loops run in the
 * canonical order: local node order k = 0..d inside a cell, corner order of
 * the node->corner list (cells ascending, then k) inside a node.
 *
 * Readings of the paper taken here (each is restated where it is used):
 *  R1  volumetric energy uses the bulk modulus K = lambda + 2 mu / 3.
 *  R2  J = rho0 * tau.
 *  R3  2D is plane strain.
 *  R4  M_cp = z_cp * sum over faces f of c through p of l_cpf n_f (x) n_f,
 *      with l_cpf = |f| / d.
 *  R5  z_cp = a(tau*)/tau*, a^2 = tau (K_t + 4 mu / 3), K_t = -J dp/dJ.
 *  R6  L_ij = dv_i/dx_j, L_c = (1/V) sum_p v_p (x) C_cp.
 *  R7  second-order predictor: one Cauchy-Kovalevskaya half step
 *      evaluated at the corner, geometry frozen at t^n.
 *  R8  reconstruction stencil: every cell sharing a node, one visit per
 *      shared node (multiplicity weights), unweighted least squares.
 *  R9  carried node velocity vhat^{n+1} = 2 v*_p - vhat^n.
 *  R10 Crank-Nicolson with dt/2 on both sides.
 *  R11 first-order B update uses L built from the step's node velocities.
 *  R12 tau^{n+1} = V(x^{n+1}) / m.
 *  R16 admissibility: finite, V > 0, det B > 0, eps >= -tol (|e|+|v|^2/2).
 *  R17 relaxed DMP on rho with absolute delta0 and relative delta1.
 *  R18 a flagged cell drops to the next scheme of the cascade; the step is
 *      recomputed from t^n until no new flag appears.  Cascade level per
 *      cell (the mask): 0 unlimited P1, 1 P1 with the Barth-Jespersen
 *      limiter, 2 P0 (the parachute).  The two-level cascade goes 0 -> 2,
 *      the three-level one 0 -> 1 -> 2.
 *  R27 shear energy family (eq. familiy_energies) with parameter a:
 *      T = -p I + (mu / J) [-a dev(Bbar) - ((1 + a)/3) I2(Bbar) dev(Bbar^-1)]
 *      (eq. cst), I2 the principal invariant, Bbar^-1 the matrix inverse;
 *      a = -1 is neo-Hookean.  The sound speed of R5 is kept for every a
 *      (the family's small-strain shear modulus is mu).
 *  R28 prescribed traction T^BC on a boundary face f: each node p of f gets
 *      the additional right-hand side T^BC (|f|/d) n_f in the nodal solver
 *      ((|f|/d) n_f = -C_ck for the face opposite node k of cell c).
 *  R29 prescribed normal velocity v_n on boundary faces: with
 *      d_p = sum_f (|f|/d) n_f and V = sum_f v_n |f|/d over the node's
 *      loaded faces, v_p = M_p^-1 (r - pi d_p) with pi such that
 *      v_p . d_p = V.  Wall and symmetry constraints come first (the
 *      paper's hierarchy): at a constrained node the same multiplier acts
 *      in the allowed directions, v = P a, (P^T M P) a = P^T (r - pi d_p),
 *      a . P^T d_p = V; the load is dropped where P^T d_p vanishes
 *      (|P^T d|^2 <= 1e-20 |d|^2).
 *  R26 Barth-Jespersen: per reconstructed scalar, bounds = min / max over
 *      {c} and its reconstruction stencil at t^n, ratio evaluated at the
 *      d+1 vertices of c; the limited gradient replaces the unlimited one
 *      in the corner values and in the predictor's time derivatives.
 *  R20 dt_vol = C_v dt min V1/|V1 - V0|, dt_incr = (1 + C_i) dt.
 *  R21 L_c = in-sphere diameter.
 *  R22 slip walls: v = P (P^T M P)^{-1} P^T r with P an orthonormal basis of
 *      the allowed directions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* public structures (mirrored by oracle/oracle.py)                    */
/* ------------------------------------------------------------------ */
typedef struct {
    double c_cfl, c_v, c_i; /* time-step control (Section 3.6, eq. CFL2) */
    double delta0, delta1;  /* relaxed DMP tolerances (eq. RDMP)          */
    double eps_tol;         /* relative tolerance of the eps >= 0 test    */
    int detect;             /* 0: accept the unlimited candidate          */
    int cascade;            /* 2: P1 -> P0; 3: P1 -> P1+BJ -> P0 (R18)    */
    double shear_a;         /* shear energy family parameter (R27)        */
    int eos;                /* 0: volumetric energy of eq. EOS_neoHook;
                               1: stiffened gas (eq. EOS_stiffened_gas, R31) */
    int pad_;
    double sg_gamma, sg_pinf; /* stiffened-gas gamma and p_inf              */
} orc_params;

typedef struct {
    double dt_next, dt_acoustic, dt_volume;
    double mass, mom[3], energy, kinetic, elastic;
    int64_t n_p0;          /* cells computed at first order at the end     */
    int64_t n_flag_first;  /* cells flagged on the first candidate         */
    int32_t mood_iters;    /* number of candidate evaluations              */
    int32_t status;        /* 0 ok, 1 a parachute cell is not admissible   */
    int64_t n_lim;         /* cells computed with the limited slopes       */
    int64_t n_recomp;      /* cell updates redone by the MOOD loop: per
                              iteration, the cells that share a node with a
                              newly flagged cell (R18)                      */
    double gcl_defect;     /* max_c |V(x^{n+1}) - V(x^n) - dt sum_p Cbar_cp .
                              v*_p| / V(x^n), Cbar the Simpson average of
                              the corner vectors over the step (eq. GCL)    */
    double detB_defect;    /* max_c |sqrt(det B^{n+1}) - rho0 tau^{n+1}|
                              (eq. test_detB_rho, reading R19)             */
    int64_t n_detB;        /* cells where that difference is >= L_c^3      */
} orc_info;

typedef struct {
    int dim, nv, nB, nW;
    int64_t nn, nc;
    int32_t *c2n;     /* [nc][nv]                                          */
    int64_t *n2c_off; /* [nn+1] node -> corner list offsets                */
    int64_t *n2c;     /* corner id = c * nv + k                            */
    int *nallow;      /* number of allowed directions per node (d - walls) */
    double *allow;    /* [nn][3][3], column a = allowed unit direction a   */
    /* boundary loads (Appendix B; R28, R29): face = (cell, local face k,
     * the face opposite the cell's k-th node); kind 1 traction tensor,
     * kind 2 normal velocity; value[6] (tensor in SYM3 order, or v_n) */
    int64_t nload;
    int32_t *ld_cell;
    int *ld_face, *ld_kind;
    double *ld_val;
} orc_mesh;

/* symmetric component ordering of B in the state arrays                 */
static const int SYM3[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
static const int SYM2[3][2] = {{0, 0}, {1, 1}, {0, 1}};

static const int (*sym_pairs(int d))[2] { return d == 3 ? SYM3 : SYM2; }

/* ------------------------------------------------------------------ */
/* small dense algebra                                                 */
/* ------------------------------------------------------------------ */
static void zero33(double A[3][3]) { memset(A, 0, 9 * sizeof(double)); }

static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

static double det33(const double A[3][3]) {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Gaussian elimination with partial pivoting on an n x n system (n <= 6).
 * A (row-major, n*n) and b are overwritten; the solution is left in b.
 * Returns -1 on an exactly zero pivot. */
static int gepp(int n, double *A, double *b) {
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs(A[col * n + col]);
        for (int r = col + 1; r < n; ++r) {
            if (fabs(A[r * n + col]) > best) {
                best = fabs(A[r * n + col]);
                piv = r;
            }
        }
        if (best == 0.0) return -1;
        if (piv != col) {
            for (int k = 0; k < n; ++k) {
                double t = A[col * n + k];
                A[col * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = A[r * n + col] / A[col * n + col];
            for (int k = col; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* geometry (Section 3.1, "Geometrical entities", eq. def_lcpncp)      */
/* ------------------------------------------------------------------ */
typedef struct {
    double V;        /* signed measure (area in 2D, volume in 3D)        */
    double xc[3];    /* centroid of a simplex = vertex mean              */
    double A[4][3];  /* |f| n_f of the face opposite local node j        */
    double C[4][3];  /* corner vector l_cp n_cp = sum_{f ni p} (|f|/d) n_f */
    double Lc;       /* in-sphere diameter, 2 d V / sum_f |f| (R21)      */
} orc_geo;

/* Outward face vectors are taken from the vertex ordering of a positively
 * oriented simplex, so they stay continuous (and C = dV/dx_p holds) even
 * for a cell that has inverted. */
static void geometry(int d, const double X[4][3], orc_geo *g) {
    memset(g, 0, sizeof(*g));
    int nv = d + 1;
    for (int k = 0; k < nv; ++k)
        for (int i = 0; i < 3; ++i) g->xc[i] += X[k][i] / (double)nv;
    if (d == 3) {
        double e1[3], e2[3], e3[3], w[3];
        for (int i = 0; i < 3; ++i) {
            e1[i] = X[1][i] - X[0][i];
            e2[i] = X[2][i] - X[0][i];
            e3[i] = X[3][i] - X[0][i];
        }
        cross3(e2, e3, w);
        g->V = dot3(e1, w) / 6.0;
        /* face opposite 0: (1,2,3) ; opposite 1: (0,3,2) ;
         * opposite 2: (0,1,3) ; opposite 3: (0,2,1)  (all outward)      */
        static const int F[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
        for (int j = 0; j < 4; ++j) {
            double a[3], b[3];
            for (int i = 0; i < 3; ++i) {
                a[i] = X[F[j][1]][i] - X[F[j][0]][i];
                b[i] = X[F[j][2]][i] - X[F[j][0]][i];
            }
            cross3(a, b, g->A[j]);
            for (int i = 0; i < 3; ++i) g->A[j][i] *= 0.5;
        }
    } else {
        double e1[3], e2[3];
        for (int i = 0; i < 3; ++i) {
            e1[i] = X[1][i] - X[0][i];
            e2[i] = X[2][i] - X[0][i];
        }
        g->V = 0.5 * (e1[0] * e2[1] - e1[1] * e2[0]);
        /* edge opposite j traversed counter-clockwise a -> b; its outward
         * normal scaled by its length is (b-a) turned by -90 degrees     */
        static const int E[3][2] = {{1, 2}, {2, 0}, {0, 1}};
        for (int j = 0; j < 3; ++j) {
            double t0 = X[E[j][1]][0] - X[E[j][0]][0];
            double t1 = X[E[j][1]][1] - X[E[j][0]][1];
            g->A[j][0] = t1;
            g->A[j][1] = -t0;
            g->A[j][2] = 0.0;
        }
    }
    double S = 0.0;
    for (int j = 0; j < nv; ++j) S += norm3(g->A[j]);
    for (int p = 0; p < nv; ++p)
        for (int j = 0; j < nv; ++j) {
            if (j == p) continue;
            for (int i = 0; i < 3; ++i) g->C[p][i] += g->A[j][i] / (double)d;
        }
    g->Lc = 2.0 * d * g->V / S;
}

/* M_cp / z_cp = sum over the faces f of c that contain p of
 * (|f|/d) n_f (x) n_f  (eq. Mcp, reading R4) */
static void corner_matrix_shape(int d, const orc_geo *g, int p, double N[3][3]) {
    zero33(N);
    for (int j = 0; j <= d; ++j) {
        if (j == p) continue;
        double area = norm3(g->A[j]);
        double n[3] = {g->A[j][0] / area, g->A[j][1] / area, g->A[j][2] / area};
        double l = area / (double)d;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) N[a][b] += l * n[a] * n[b];
    }
}

/* ------------------------------------------------------------------ */
/* constitutive law (Section 2.2.4, eqs. EOS_neoHook, cstnh; R1, R2)   */
/* ------------------------------------------------------------------ */
typedef struct {
    double rho0, mu, K;
    double a; /* shear energy family (eq. familiy_energies); -1: neo-Hookean */
    int eos;  /* 1: stiffened gas (R31): p from the internal energy           */
    double gam, pinf;
} orc_mat;

/* p = -(K/2)(J - 1 + ln J / J) */
static double pressure(const orc_mat *m, double J) {
    return -0.5 * m->K * (J - 1.0 + log(J) / J);
}

/* inverse of a 3x3 matrix by cofactors */
static void inv33(const double A[3][3], double Ai[3][3]) {
    double det = det33(A);
    Ai[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    Ai[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    Ai[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

/* second principal invariant 1/2 ((tr A)^2 - tr(A A)) */
static double inv2(const double A[3][3]) {
    double tr = A[0][0] + A[1][1] + A[2][2], tr2 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) tr2 += A[i][k] * A[k][i];
    return 0.5 * (tr * tr - tr2);
}

/* Shear part of the specific free energy (eq. familiy_energies):
 *   Psi_s = mu/(4 rho0) [-2a (I1b - 3) + (1+a)/3 (I2b^2 - 9)],
 * Bbar = J^{-2/3} B, I1b = tr Bbar, I2b its second invariant. */
static double shear_energy(const orc_mat *m, double tau, const double B[3][3]) {
    double J = m->rho0 * tau;
    double s = pow(J, -2.0 / 3.0);
    double Bb[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Bb[i][j] = s * B[i][j];
    double I1b = Bb[0][0] + Bb[1][1] + Bb[2][2];
    double I2b = inv2(Bb);
    return m->mu / (4.0 * m->rho0) * (-2.0 * m->a * (I1b - 3.0) + (1.0 + m->a) / 3.0 * (I2b * I2b - 9.0));
}

/* Derivative of Psi_s along (dtau, dB):
 *   dPsi_s = mu/(4 rho0) [-2a dI1b + (2/3)(1+a) I2b dI2b],
 *   dBbar = J^{-2/3} dB - (2/3)(dJ/J) Bbar, dI1b = tr dBbar,
 *   dI2b = tr Bbar tr dBbar - tr(Bbar dBbar). */
static double shear_energy_direction(const orc_mat *m, double tau, const double B[3][3], double dtau,
                                     const double dB[3][3]) {
    double J = m->rho0 * tau, dJ = m->rho0 * dtau;
    double s = pow(J, -2.0 / 3.0);
    double Bb[3][3], dBb[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Bb[i][j] = s * B[i][j];
            dBb[i][j] = s * dB[i][j] - (2.0 / 3.0) * (dJ / J) * s * B[i][j];
        }
    double tr = Bb[0][0] + Bb[1][1] + Bb[2][2], dtr = dBb[0][0] + dBb[1][1] + dBb[2][2];
    double BdB = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) BdB += Bb[i][k] * dBb[k][i];
    double I2b = inv2(Bb), dI2b = tr * dtr - BdB;
    return m->mu / (4.0 * m->rho0) * (-2.0 * m->a * dtr + (2.0 / 3.0) * (1.0 + m->a) * I2b * dI2b);
}

/* Stiffened gas (eq. EOS_stiffened_gas; reading R31): the volumetric part
 * of the specific internal energy is eps_v = eps - Psi_s, and
 * eps_v = (p + gamma p_inf) / ((gamma - 1) rho) gives
 *   p = (gamma - 1) (eps - Psi_s) / tau - gamma p_inf. */
static double sg_pressure(const orc_mat *m, double tau, const double B[3][3], double eps) {
    return (m->gam - 1.0) * (eps - shear_energy(m, tau, B)) / tau - m->gam * m->pinf;
}

/* T = -p I + (mu / J) [-a dev(Bbar) - ((1+a)/3) I2(Bbar) dev(Bbar^-1)],
 * Bbar = J^{-2/3} B (eqs. cst, familiy_energies; R27).  For a = -1 this is
 * (mu / J) dev(Bbar) - p I (eq. cstnh). */
static void stress(const orc_mat *m, double tau, const double B[3][3], double eps, double T[3][3]) {
    double J = m->rho0 * tau;
    double p = m->eos ? sg_pressure(m, tau, B, eps) : pressure(m, J);
    double s = pow(J, -2.0 / 3.0);
    double Bb[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Bb[i][j] = s * B[i][j];
    double tr = Bb[0][0] + Bb[1][1] + Bb[2][2];
    double c = (1.0 + m->a) / 3.0;
    double Bi[3][3] = {{0}}, tri = 0.0, I2 = 0.0;
    if (c != 0.0) {
        inv33(Bb, Bi);
        tri = Bi[0][0] + Bi[1][1] + Bi[2][2];
        I2 = inv2(Bb);
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dev = Bb[i][j] - (i == j ? tr / 3.0 : 0.0);
            double sh = -m->a * dev;
            if (c != 0.0) sh -= c * I2 * (Bi[i][j] - (i == j ? tri / 3.0 : 0.0));
            T[i][j] = (m->mu / J) * sh - (i == j ? p : 0.0);
        }
}

/* sound speed a = sqrt(tau (K_t + 4 mu / 3)), K_t = -J dp/dJ (R5); for the
 * stiffened gas K_t = gamma (p + p_inf), the isentropic bulk modulus (R31) */
static double sound_speed(const orc_mat *m, double tau, const double B[3][3], double eps) {
    if (m->eos) return sqrt(tau * (m->gam * (sg_pressure(m, tau, B, eps) + m->pinf) + 4.0 * m->mu / 3.0));
    double J = m->rho0 * tau;
    double Kt = 0.5 * m->K * (J + (1.0 - log(J)) / J);
    return sqrt(tau * (Kt + 4.0 * m->mu / 3.0));
}

/* Specific free energy Psi_v + Psi_s (Section 2.2.4, eq. familiy_energies),
 * used by the energy diagnostics only; the stiffened gas reports Psi_s. */
static double free_energy(const orc_mat *m, double tau, const double B[3][3]) {
    if (m->eos) return shear_energy(m, tau, B);
    double J = m->rho0 * tau;
    double lj = log(J);
    double s = pow(J, -2.0 / 3.0);
    double I1b = s * (B[0][0] + B[1][1] + B[2][2]);
    double psi_v = m->K / (4.0 * m->rho0) * ((J - 1.0) * (J - 1.0) + lj * lj);
    if (m->a == -1.0) return psi_v + m->mu / (2.0 * m->rho0) * (I1b - 3.0);
    double Bb[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Bb[i][j] = s * B[i][j];
    double I2b = inv2(Bb);
    return psi_v + m->mu / (4.0 * m->rho0) *
                       (-2.0 * m->a * (I1b - 3.0) + (1.0 + m->a) / 3.0 * (I2b * I2b - 9.0));
}

/* Derivative of T(tau, B) along a direction (dtau, dB), J = rho0 tau:
 *   neo-Hookean (a = -1), T = -p(J) I + mu J^{-5/3} dev(B):
 *     dT = rho0 [ -p'(J) I - (5/3) mu J^{-8/3} dev(B) ] dtau + mu J^{-5/3} dev(dB)
 *   family (R27), with dJ = rho0 dtau, dBbar = J^{-2/3} dB - (2/3)(dJ/J) Bbar,
 *   d(Bbar^-1) = -Bbar^-1 dBbar Bbar^-1, dI2 = tr(Bbar) tr(dBbar) - tr(Bbar dBbar):
 *     dT = -dp I - (dJ/J) T_0 + (mu/J) [-a dev(dBbar)
 *          - c (dI2 dev(Bbar^-1) + I2 dev(d(Bbar^-1)))],  c = (1+a)/3,
 *   with dp = p'(J) dJ, or for the stiffened gas (R31) the derivative of
 *   p(tau, eps, B) along (dtau, deps, dB). */
static void stress_direction(const orc_mat *m, double tau, const double B[3][3], double eps, double dtau,
                             const double dB[3][3], double deps, double dT[3][3]) {
    double J = m->rho0 * tau;
    double lj = log(J);
    double dpdJ = -0.5 * m->K * (1.0 + (1.0 - lj) / (J * J));
    if (m->a == -1.0 && !m->eos) {
        double J53 = pow(J, -5.0 / 3.0);
        double J83 = pow(J, -8.0 / 3.0);
        double trB = B[0][0] + B[1][1] + B[2][2];
        double trdB = dB[0][0] + dB[1][1] + dB[2][2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double devB = B[i][j] - (i == j ? trB / 3.0 : 0.0);
                double devdB = dB[i][j] - (i == j ? trdB / 3.0 : 0.0);
                dT[i][j] = m->rho0 * ((i == j ? -dpdJ : 0.0) - (5.0 / 3.0) * m->mu * J83 * devB) * dtau +
                           m->mu * J53 * devdB;
            }
        return;
    }
    double dJ = m->rho0 * dtau;
    double s = pow(J, -2.0 / 3.0);
    double Bb[3][3], dBb[3][3], Bi[3][3], dBi[3][3], tmp[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Bb[i][j] = s * B[i][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dBb[i][j] = s * dB[i][j] - (2.0 / 3.0) * (dJ / J) * Bb[i][j];
    inv33(Bb, Bi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += dBb[i][k] * Bi[k][j];
            tmp[i][j] = t;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += Bi[i][k] * tmp[k][j];
            dBi[i][j] = -t;
        }
    double c = (1.0 + m->a) / 3.0;
    double I2 = inv2(Bb);
    double trBb = Bb[0][0] + Bb[1][1] + Bb[2][2], trdBb = dBb[0][0] + dBb[1][1] + dBb[2][2];
    double BdB = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) BdB += Bb[i][k] * dBb[k][i];
    double dI2 = trBb * trdBb - BdB;
    double trBi = Bi[0][0] + Bi[1][1] + Bi[2][2], trdBi = dBi[0][0] + dBi[1][1] + dBi[2][2];
    /* dp: -p'(J) dJ, or for the stiffened gas (R31)
     * (gamma - 1) [(deps - dPsi_s) / tau - (eps - Psi_s) dtau / tau^2] */
    double dpv = dpdJ * dJ;
    if (m->eos)
        dpv = (m->gam - 1.0) * ((deps - shear_energy_direction(m, tau, B, dtau, dB)) / tau -
                                (eps - shear_energy(m, tau, B)) * dtau / (tau * tau));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double e = (i == j) ? 1.0 : 0.0;
            double T0 = (m->mu / J) * (-m->a * (Bb[i][j] - e * trBb / 3.0) - c * I2 * (Bi[i][j] - e * trBi / 3.0));
            double dsh = -m->a * (dBb[i][j] - e * trdBb / 3.0) -
                         c * (dI2 * (Bi[i][j] - e * trBi / 3.0) + I2 * (dBi[i][j] - e * trdBi / 3.0));
            dT[i][j] = -dpv * e - (dJ / J) * T0 + (m->mu / J) * dsh;
        }
}

static void unpack_B(int d, const double *b, double B[3][3]) {
    zero33(B);
    const int(*sp)[2] = sym_pairs(d);
    int nB = d == 3 ? 6 : 3;
    for (int s = 0; s < nB; ++s) {
        B[sp[s][0]][sp[s][1]] = b[s];
        B[sp[s][1]][sp[s][0]] = b[s];
    }
    if (d == 2) B[2][2] = 1.0;
}

static void pack_B(int d, const double B[3][3], double *b) {
    const int(*sp)[2] = sym_pairs(d);
    int nB = d == 3 ? 6 : 3;
    for (int s = 0; s < nB; ++s) b[s] = B[sp[s][0]][sp[s][1]];
}

static void cell_nodes(const orc_mesh *M, const double *x, int64_t c, double X[4][3]) {
    memset(X, 0, 4 * 3 * sizeof(double));
    for (int k = 0; k < M->nv; ++k) {
        int64_t p = M->c2n[c * M->nv + k];
        for (int i = 0; i < M->dim; ++i) X[k][i] = x[p * M->dim + i];
    }
}

/* ------------------------------------------------------------------ */
/* mesh set-up                                                         */
/* ------------------------------------------------------------------ */
/* orthonormal basis of the directions a wall node may move in, built by
 * Gram-Schmidt: first the wall normals, then the coordinate axes with the
 * largest residual (R22) */
static int allowed_basis(int d, int nw, const double *normals, double P[3][3]) {
    double Q[3][3];
    int nq = 0;
    for (int r = 0; r < nw; ++r) {
        double w[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) w[i] = normals[r * d + i];
        for (int q = 0; q < nq; ++q) {
            double s = dot3(w, Q[q]);
            for (int i = 0; i < 3; ++i) w[i] -= s * Q[q][i];
        }
        double n = norm3(w);
        if (n < 1e-8) continue; /* dependent normal */
        for (int i = 0; i < 3; ++i) Q[nq][i] = w[i] / n;
        ++nq;
    }
    zero33(P);
    int m = d - nq;
    for (int t = 0; t < m; ++t) {
        double bestw[3] = {0, 0, 0}, bestn = -1.0;
        for (int a = 0; a < d; ++a) {
            double w[3] = {0, 0, 0};
            w[a] = 1.0;
            for (int q = 0; q < nq; ++q) {
                double s = dot3(w, Q[q]);
                for (int i = 0; i < 3; ++i) w[i] -= s * Q[q][i];
            }
            for (int q = 0; q < t; ++q) {
                double col[3] = {P[0][q], P[1][q], P[2][q]};
                double s = dot3(w, col);
                for (int i = 0; i < 3; ++i) w[i] -= s * col[i];
            }
            double n = norm3(w);
            if (n > bestn) {
                bestn = n;
                memcpy(bestw, w, sizeof bestw);
            }
        }
        for (int i = 0; i < 3; ++i) P[i][t] = bestw[i] / bestn;
    }
    return m;
}

void orc_mesh_free(orc_mesh *M) {
    if (!M) return;
    free(M->ld_cell);
    free(M->ld_face);
    free(M->ld_kind);
    free(M->ld_val);
    free(M->c2n);
    free(M->n2c_off);
    free(M->n2c);
    free(M->nallow);
    free(M->allow);
    free(M);
}

orc_mesh *orc_mesh_new(int dim, int64_t nn, int64_t nc, const int32_t *c2n, const uint8_t *nwall,
                       const double *normals) {
    if (dim != 2 && dim != 3) return NULL;
    orc_mesh *M = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    M->dim = dim;
    M->nv = dim + 1;
    M->nB = dim == 3 ? 6 : 3;
    M->nW = 1 + dim + M->nB;
    M->nn = nn;
    M->nc = nc;
    M->c2n = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc * M->nv + 1));
    memcpy(M->c2n, c2n, sizeof(int32_t) * (size_t)(nc * M->nv));
    M->n2c_off = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
    M->n2c = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc * M->nv + 1));
    for (int64_t q = 0; q < nc * M->nv; ++q) {
        int32_t p = c2n[q];
        if (p < 0 || p >= nn) {
            orc_mesh_free(M);
            return NULL;
        }
        M->n2c_off[p + 1]++;
    }
    for (int64_t p = 0; p < nn; ++p) M->n2c_off[p + 1] += M->n2c_off[p];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn + 1));
    memcpy(fill, M->n2c_off, sizeof(int64_t) * (size_t)(nn + 1));
    for (int64_t q = 0; q < nc * M->nv; ++q) M->n2c[fill[c2n[q]]++] = q;
    free(fill);
    M->nallow = (int *)malloc(sizeof(int) * (size_t)(nn + 1));
    M->allow = (double *)calloc((size_t)nn * 9 + 1, sizeof(double));
    for (int64_t p = 0; p < nn; ++p) {
        double P[3][3];
        int nw = nwall ? nwall[p] : 0;
        M->nallow[p] = allowed_basis(dim, nw, normals ? normals + p * dim * dim : NULL, P);
        memcpy(M->allow + p * 9, P, sizeof P);
    }
    return M;
}

/* Replace the boundary loads of the mesh (n = 0 clears them). */
int orc_set_loads(orc_mesh *M, int64_t n, const int32_t *cell, const uint8_t *face, const uint8_t *kind,
                  const double *value) {
    free(M->ld_cell);
    free(M->ld_face);
    free(M->ld_kind);
    free(M->ld_val);
    M->ld_cell = NULL;
    M->ld_face = M->ld_kind = NULL;
    M->ld_val = NULL;
    M->nload = 0;
    if (n <= 0) return 0;
    M->ld_cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    M->ld_face = (int *)malloc(sizeof(int) * (size_t)n);
    M->ld_kind = (int *)malloc(sizeof(int) * (size_t)n);
    M->ld_val = (double *)malloc(sizeof(double) * (size_t)n * 6);
    for (int64_t l = 0; l < n; ++l) {
        if (cell[l] < 0 || cell[l] >= M->nc || face[l] >= M->nv || (kind[l] != 1 && kind[l] != 2)) return -1;
        M->ld_cell[l] = cell[l];
        M->ld_face[l] = face[l];
        M->ld_kind[l] = kind[l];
        for (int q = 0; q < 6; ++q) M->ld_val[l * 6 + q] = value[l * 6 + q];
    }
    M->nload = n;
    return 0;
}

/* Replace the wall normals of node p (nw rows of dim components), for
 * boundary conditions that change type during a run (Section 3.8). */
int orc_set_node_walls(orc_mesh *M, int64_t p, int nw, const double *normals) {
    if (p < 0 || p >= M->nn || nw < 0 || nw > 3) return -1;
    double P[3][3];
    M->nallow[p] = allowed_basis(M->dim, nw, nw ? normals : NULL, P);
    memcpy(M->allow + p * 9, P, sizeof P);
    return 0;
}

/* ------------------------------------------------------------------ */
/* initial state (Section 4 preamble; reading R25)                    */
/* ------------------------------------------------------------------ */
/* project a node vector onto the allowed directions of node p */
static void project_allowed(const orc_mesh *M, int64_t p, const double v[3], double out[3]) {
    const double *P = M->allow + p * 9;
    int m = M->nallow[p];
    out[0] = out[1] = out[2] = 0.0;
    for (int t = 0; t < m; ++t) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += P[i * 3 + t] * v[i];
        for (int i = 0; i < 3; ++i) out[i] += s * P[i * 3 + t];
    }
}

int orc_init_state(const orc_mesh *M, const double *x, const double *rho0, const double *mu,
                   const double *lam, const double *v_cell, const double *v_node, double *m_out,
                   double *K_out, double *tau, double *v, double *e, double *B, double *vhat) {
    int d = M->dim;
    int bad = 0;
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(d, X, &g);
        if (!(g.V > 0.0)) bad = 1;
        m_out[c] = rho0[c] * g.V;
        K_out[c] = lam[c] + 2.0 * mu[c] / 3.0;
        tau[c] = 1.0 / rho0[c];
        double k2 = 0.0;
        for (int i = 0; i < d; ++i) {
            v[c * d + i] = v_cell[c * d + i];
            k2 += v_cell[c * d + i] * v_cell[c * d + i];
        }
        e[c] = 0.5 * k2;
        double I[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        pack_B(d, I, B + c * M->nB);
    }
    for (int64_t p = 0; p < M->nn; ++p) {
        double w[3] = {0, 0, 0}, o[3];
        for (int i = 0; i < d; ++i) w[i] = v_node[p * d + i];
        project_allowed(M, p, w, o);
        for (int i = 0; i < d; ++i) vhat[p * d + i] = o[i];
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* least-squares gradients (reading R8)                                */
/* ------------------------------------------------------------------ */
/* W = (tau, v_1..v_d, B components in state order, eps = e - |v|^2 / 2);
 * eps (index nW) is reconstructed for the stiffened gas (R31) and is 0
 * when e is NULL */
static void cell_W(const orc_mesh *M, const double *tau, const double *v, const double *B, const double *e,
                   int64_t c, double *W) {
    int d = M->dim;
    W[0] = tau[c];
    double k2 = 0.0;
    for (int i = 0; i < d; ++i) {
        W[1 + i] = v[c * d + i];
        k2 += v[c * d + i] * v[c * d + i];
    }
    for (int s = 0; s < M->nB; ++s) W[1 + d + s] = B[c * M->nB + s];
    W[M->nW] = e ? e[c] - 0.5 * k2 : 0.0;
}

/* grad[c][w][j] = d W_w / d x_j from an unweighted least-squares fit over
 * all cells sharing a node with c, each visited once per shared node.  A
 * stencil with fewer than d visits, or whose normal matrix is singular
 * (det A <= 1e-12 (tr A / d)^d), gives a zero gradient. */
static void lsq_gradients(const orc_mesh *M, const double *xc, const double *tau, const double *v,
                          const double *B, const double *e, double *grad) {
    int d = M->dim, nW = M->nW + 1, nv = M->nv;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < M->nc; ++c) {
        double A[3][3] = {{0}};
        double b[11][3] = {{0}};
        double Wc[11], Wk[11];
        int visits = 0;
        cell_W(M, tau, v, B, e, c, Wc);
        for (int k = 0; k < nv; ++k) {
            int64_t p = M->c2n[c * nv + k];
            for (int64_t q = M->n2c_off[p]; q < M->n2c_off[p + 1]; ++q) {
                int64_t j = M->n2c[q] / nv;
                if (j == c) continue;
                ++visits;
                double dx[3] = {0, 0, 0};
                for (int i = 0; i < d; ++i) dx[i] = xc[j * 3 + i] - xc[c * 3 + i];
                cell_W(M, tau, v, B, e, j, Wk);
                for (int a = 0; a < d; ++a)
                    for (int bb = 0; bb < d; ++bb) A[a][bb] += dx[a] * dx[bb];
                for (int w = 0; w < nW; ++w)
                    for (int a = 0; a < d; ++a) b[w][a] += dx[a] * (Wk[w] - Wc[w]);
            }
        }
        double detA, trA = 0.0;
        for (int a = 0; a < d; ++a) trA += A[a][a];
        if (d == 3)
            detA = det33(A);
        else
            detA = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        double scale = pow(trA / d, d);
        double *g = grad + c * nW * 3;
        memset(g, 0, sizeof(double) * nW * 3);  /* nW includes eps here */
        if (visits < d || !(trA > 0.0) || !(detA > 1e-12 * scale)) continue;
        for (int w = 0; w < nW; ++w) {
            double Am[9], rhs[3];
            for (int a = 0; a < d; ++a) {
                rhs[a] = b[w][a];
                for (int bb = 0; bb < d; ++bb) Am[a * d + bb] = A[a][bb];
            }
            gepp(d, Am, rhs);
            for (int a = 0; a < d; ++a) g[w * 3 + a] = rhs[a];
        }
    }
}

/* Barth-Jespersen limiter, the second scheme of the cascade (Section 3.5;
 * reading R26).  For every reconstructed scalar W_w of cell c, with m and M
 * the min and max of W_w over {c} and its reconstruction stencil and
 * D_k = grad W_w . (x_k - x_c) at the vertices x_k of c,
 *   phi = min over k of  min(1, (M - W_c) / D_k)  if D_k > 0,
 *                        min(1, (m - W_c) / D_k)  if D_k < 0,
 *                        1                        if D_k = 0,
 * and the limited gradient is phi grad W_w. */
static void bj_limit(const orc_mesh *M, const double *x, const double *xc, const double *tau,
                     const double *v, const double *B, const double *grad, double *glim) {
    int d = M->dim, nW = M->nW, nv = M->nv, st = M->nW + 1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < M->nc; ++c) {
        double Wc[11], Wk[11], lo[11], hi[11];
        cell_W(M, tau, v, B, NULL, c, Wc);
        for (int w = 0; w < nW; ++w) lo[w] = hi[w] = Wc[w];
        for (int k = 0; k < nv; ++k) {
            int64_t p = M->c2n[c * nv + k];
            for (int64_t q = M->n2c_off[p]; q < M->n2c_off[p + 1]; ++q) {
                cell_W(M, tau, v, B, NULL, M->n2c[q] / nv, Wk);
                for (int w = 0; w < nW; ++w) {
                    lo[w] = fmin(lo[w], Wk[w]);
                    hi[w] = fmax(hi[w], Wk[w]);
                }
            }
        }
        const double *g = grad + c * st * 3;
        double *o = glim + c * st * 3;
        for (int i = 0; i < 3; ++i) o[nW * 3 + i] = g[nW * 3 + i]; /* eps: not limited */
        for (int w = 0; w < nW; ++w) {
            double phi = 1.0;
            for (int k = 0; k < nv; ++k) {
                int64_t p = M->c2n[c * nv + k];
                double D = 0.0;
                for (int i = 0; i < d; ++i) D += g[w * 3 + i] * (x[p * d + i] - xc[c * 3 + i]);
                double r = 1.0;
                if (D > 0.0)
                    r = fmin(1.0, (hi[w] - Wc[w]) / D);
                else if (D < 0.0)
                    r = fmin(1.0, (lo[w] - Wc[w]) / D);
                phi = fmin(phi, r);
            }
            for (int i = 0; i < 3; ++i) o[w * 3 + i] = phi * g[w * 3 + i];
        }
    }
}

/* ------------------------------------------------------------------ */
/* ADER predictor (Section 3.4, eq. NCPDE2; reading R7)                */
/* ------------------------------------------------------------------ */
typedef struct {
    double tau, v[3], B[3][3]; /* predicted state at the corner */
    double eps;                /* predicted specific internal energy (R31) */
    double T[3][3];            /* stress of the predicted state */
    double z;                  /* swept mass flux a / tau (R5)  */
} orc_corner;

/* Corner state of cell c at node k.  P0 cells use the cell values; P1
 * cells evolve the linear reconstruction by a half step:
 *   W* = W_c + grad W . (x_p - x_c) + (dt/2) dW/dt,
 *   dtau/dt = tau tr G,  dv/dt = tau div T,  dB/dt = G B + B G^T,
 *   G = grad v, div T by the chain rule through T(tau, B). */
static void predict_corner(const orc_mesh *M, const orc_mat *mat, const orc_geo *g, const double *X,
                           double tau, const double *vc, const double Bc[3][3], double eps, const double *grad,
                           int p1, double dt, orc_corner *out) {
    int d = M->dim;
    memset(out, 0, sizeof(*out));
    out->tau = tau;
    out->eps = eps;
    for (int i = 0; i < d; ++i) out->v[i] = vc[i];
    memcpy(out->B, Bc, sizeof(out->B));
    if (p1) {
        const int(*sp)[2] = sym_pairs(d);
        double h = 0.5 * dt;
        double gt[3] = {0, 0, 0}, G[3][3] = {{0}}, gB[3][3][3] = {{{0}}};
        for (int j = 0; j < d; ++j) {
            gt[j] = grad[0 * 3 + j];
            for (int i = 0; i < d; ++i) G[i][j] = grad[(1 + i) * 3 + j];
            for (int s = 0; s < M->nB; ++s) {
                double val = grad[(1 + d + s) * 3 + j];
                gB[j][sp[s][0]][sp[s][1]] = val;
                gB[j][sp[s][1]][sp[s][0]] = val;
            }
        }
        double trG = 0.0;
        for (int i = 0; i < d; ++i) trG += G[i][i];
        double dtau = tau * trG;
        double dB[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += G[i][k] * Bc[k][j] + Bc[i][k] * G[j][k];
                dB[i][j] = s;
            }
        double ge[3] = {0, 0, 0};
        for (int j = 0; j < d; ++j) ge[j] = grad[M->nW * 3 + j];
        double divT[3] = {0, 0, 0};
        for (int j = 0; j < d; ++j) {
            double dTj[3][3];
            stress_direction(mat, tau, Bc, eps, gt[j], gB[j], ge[j], dTj);
            for (int i = 0; i < 3; ++i) divT[i] += dTj[i][j];
        }
        /* internal energy (R31): d eps / dt = tau T : grad v */
        double Tc[3][3], TG = 0.0;
        stress(mat, tau, Bc, eps, Tc);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) TG += Tc[i][j] * G[i][j];
        double delta[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) delta[i] = X[i] - g->xc[i];
        double s = 0.0;
        for (int j = 0; j < d; ++j) s += gt[j] * delta[j];
        out->tau = tau + s + h * dtau;
        double se = 0.0;
        for (int j = 0; j < d; ++j) se += ge[j] * delta[j];
        out->eps = eps + se + h * tau * TG;
        for (int i = 0; i < d; ++i) {
            double a = 0.0;
            for (int j = 0; j < d; ++j) a += G[i][j] * delta[j];
            out->v[i] = vc[i] + a + h * tau * divT[i];
        }
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                double a = 0.0;
                for (int j = 0; j < d; ++j) a += gB[j][i][k] * delta[j];
                out->B[i][k] = Bc[i][k] + a + h * dB[i][k];
            }
        if (d == 2) out->B[2][2] = 1.0;
    }
    stress(mat, out->tau, out->B, out->eps, out->T);
    out->z = sound_speed(mat, out->tau, out->B, out->eps) / out->tau;
}

/* ------------------------------------------------------------------ */
/* B update (Section 3.4, eqs. firstB and CN_B; readings R10, R11)     */
/* ------------------------------------------------------------------ */
static void lie_term(const double L[3][3], const double X[3][3], double Y[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += L[i][k] * X[k][j] + X[i][k] * L[j][k];
            Y[i][j] = s;
        }
}

/* Solve  X - (dt/2)(L1 X + X L1^T) = Bn + (dt/2)(Ln Bn + Bn Ln^T)  for the
 * symmetric X by assembling the linear map on the symmetric components and
 * eliminating with partial pivoting. */
static int cn_solve(int d, const double Bn[3][3], const double Ln[3][3], const double L1[3][3],
                    double dt, double Xout[3][3]) {
    const int(*sp)[2] = sym_pairs(d);
    int n = d == 3 ? 6 : 3;
    double A[36], r[6], Y[3][3];
    lie_term(Ln, Bn, Y);
    for (int s = 0; s < n; ++s) r[s] = Bn[sp[s][0]][sp[s][1]] + 0.5 * dt * Y[sp[s][0]][sp[s][1]];
    for (int col = 0; col < n; ++col) {
        double E[3][3] = {{0}};
        E[sp[col][0]][sp[col][1]] = 1.0;
        E[sp[col][1]][sp[col][0]] = 1.0;
        lie_term(L1, E, Y);
        for (int row = 0; row < n; ++row) {
            int i = sp[row][0], j = sp[row][1];
            A[row * n + col] = E[i][j] - 0.5 * dt * Y[i][j];
        }
    }
    int st = gepp(n, A, r);
    zero33(Xout);
    for (int s = 0; s < n; ++s) {
        Xout[sp[s][0]][sp[s][1]] = r[s];
        Xout[sp[s][1]][sp[s][0]] = r[s];
    }
    if (d == 2) Xout[2][2] = 1.0;
    return st;
}

/* L = (1/V) sum_p v_p (x) C_p   (eq. div_grad_v, orientation R6) */
static void velocity_gradient(int d, const orc_geo *g, const double vp[4][3], double L[3][3]) {
    zero33(L);
    for (int k = 0; k <= d; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) L[i][j] += vp[k][i] * g->C[k][j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) L[i][j] /= g->V;
}

/* ------------------------------------------------------------------ */
/* one step                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_mesh *M;
    const double *rho0, *mu, *K, *m;
    const double *x, *vhat, *tau, *v, *e, *B;
    double dt;
    double a;        /* shear energy family parameter (R27) */
    int eos;         /* stiffened gas (R31) and its parameters */
    double gam, pinf;
    /* derived at t^n */
    orc_geo *geo;
    double *xc;      /* [nc][3] */
    double *grad;    /* [nc][nW][3] */
    double *glim;    /* [nc][nW][3] Barth-Jespersen limited gradients */
    double *rmin, *rmax;
    /* candidate */
    orc_corner *cor; /* [nc*nv] */
    double *vstar;   /* [nn][3] */
    double *x1, *vhat1, *tau1, *v1, *e1, *B1;
} orc_work;

static orc_mat mat_of(const orc_work *w, int64_t c) {
    orc_mat m = {w->rho0[c], w->mu[c], w->K[c], w->a, w->eos, w->gam, w->pinf};
    return m;
}

static void candidate(orc_work *w, const uint8_t *mask) {
    const orc_mesh *M = w->M;
    int d = M->dim, nv = M->nv;
    /* predictor at every corner */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < M->nc; ++c) {
        orc_mat mat = mat_of(w, c);
        double Bc[3][3];
        unpack_B(d, w->B + c * M->nB, Bc);
        for (int k = 0; k < nv; ++k) {
            int64_t p = M->c2n[c * nv + k];
            double X[3] = {0, 0, 0};
            for (int i = 0; i < d; ++i) X[i] = w->x[p * d + i];
            const double *gc = (mask[c] == 1 ? w->glim : w->grad) + c * (M->nW + 1) * 3;
            double k2 = 0.0;
            for (int i = 0; i < d; ++i) k2 += w->v[c * d + i] * w->v[c * d + i];
            predict_corner(M, &mat, &w->geo[c], X, w->tau[c], w->v + c * d, Bc, w->e[c] - 0.5 * k2, gc,
                           mask[c] < 2, w->dt, &w->cor[c * nv + k]);
        }
    }
    /* nodal solver (eq. nodal_solver^n, readings R14, R15, R22) */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < M->nn; ++p) {
        double Mp[3][3] = {{0}}, r[3] = {0, 0, 0};
        for (int64_t q = M->n2c_off[p]; q < M->n2c_off[p + 1]; ++q) {
            int64_t c = M->n2c[q] / nv;
            int k = (int)(M->n2c[q] % nv);
            const orc_corner *cr = &w->cor[c * nv + k];
            double N[3][3];
            corner_matrix_shape(d, &w->geo[c], k, N);
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int b = 0; b < 3; ++b) {
                    Mp[a][b] += cr->z * N[a][b];
                    s += cr->z * N[a][b] * cr->v[b] - cr->T[a][b] * w->geo[c].C[k][b];
                }
                r[a] += s;
            }
        }
        /* boundary loads of the faces through p (readings R28, R29) */
        double dv[3] = {0, 0, 0}, Vn = 0.0;
        int has_v = 0;
        for (int64_t l = 0; l < M->nload; ++l) {
            int64_t c = M->ld_cell[l];
            int k = M->ld_face[l], on = 0;
            for (int j = 0; j < nv; ++j)
                if (j != k && M->c2n[c * nv + j] == p) on = 1;
            if (!on) continue;
            double ln[3];
            for (int a = 0; a < 3; ++a) ln[a] = -w->geo[c].C[k][a]; /* (|f|/d) n_f */
            const double *val = M->ld_val + l * 6;
            if (M->ld_kind[l] == 1) {
                double T[3][3];
                for (int q = 0; q < 6; ++q) {
                    T[SYM3[q][0]][SYM3[q][1]] = val[q];
                    T[SYM3[q][1]][SYM3[q][0]] = val[q];
                }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) r[a] += T[a][b] * ln[b];
            } else {
                has_v = 1;
                for (int a = 0; a < 3; ++a) dv[a] += ln[a];
                Vn += val[0] * norm3(ln);
            }
        }
        const double *P = M->allow + p * 9;
        int m = M->nallow[p];
        double vs[3] = {0, 0, 0};
        if (m == d && has_v && M->n2c_off[p + 1] > M->n2c_off[p]) {
            /* v = M_p^-1 (r - pi d), v . d = V */
            double A1[9], A2[9], y[3], z[3];
            for (int a = 0; a < d; ++a) {
                y[a] = r[a];
                z[a] = dv[a];
                for (int b = 0; b < d; ++b) A1[a * d + b] = A2[a * d + b] = Mp[a][b];
            }
            gepp(d, A1, y);
            gepp(d, A2, z);
            double yd = 0.0, zd = 0.0;
            for (int a = 0; a < d; ++a) {
                yd += y[a] * dv[a];
                zd += z[a] * dv[a];
            }
            double pi = (yd - Vn) / zd;
            for (int a = 0; a < d; ++a) vs[a] = y[a] - pi * z[a];
        } else if (m > 0) {
            /* Galerkin projection on the allowed directions (R22); a
               velocity load is then met within them, unless they are
               orthogonal to d (R29: walls and symmetry first) */
            double Ar[9], br[3], A2[9], e[3], z[3];
            double ee = 0.0, dd = 0.0;
            for (int s = 0; s < m; ++s) {
                br[s] = 0.0;
                e[s] = 0.0;
                for (int i = 0; i < 3; ++i) br[s] += P[i * 3 + s] * r[i];
                for (int i = 0; i < 3; ++i) e[s] += P[i * 3 + s] * dv[i];
                ee += e[s] * e[s];
                for (int t = 0; t < m; ++t) {
                    double a = 0.0;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) a += P[i * 3 + s] * Mp[i][j] * P[j * 3 + t];
                    Ar[s * m + t] = a;
                    A2[s * m + t] = a;
                }
            }
            for (int a = 0; a < 3; ++a) dd += dv[a] * dv[a];
            gepp(m, Ar, br);
            if (has_v && ee > 1e-20 * dd) {
                for (int s = 0; s < m; ++s) z[s] = e[s];
                gepp(m, A2, z);
                double ye = 0.0, ze = 0.0;
                for (int s = 0; s < m; ++s) {
                    ye += br[s] * e[s];
                    ze += z[s] * e[s];
                }
                double pi = (ye - Vn) / ze;
                for (int s = 0; s < m; ++s) br[s] -= pi * z[s];
            }
            for (int i = 0; i < 3; ++i)
                for (int t = 0; t < m; ++t) vs[i] += P[i * 3 + t] * br[t];
        }
        for (int i = 0; i < 3; ++i) w->vstar[p * 3 + i] = vs[i];
        for (int i = 0; i < d; ++i) {
            w->x1[p * d + i] = w->x[p * d + i] + w->dt * vs[i];  /* R13 */
            w->vhat1[p * d + i] = 2.0 * vs[i] - w->vhat[p * d + i]; /* R9 */
        }
    }
    /* cell update (eqs. tau_c^n .. subforce^n; readings R12, R15) */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < M->nc; ++c) {
        const orc_geo *g = &w->geo[c];
        double F[3] = {0, 0, 0}, W = 0.0;
        double vsk[4][3], vhn[4][3], vh1[4][3];
        for (int k = 0; k < nv; ++k) {
            int64_t p = M->c2n[c * nv + k];
            const orc_corner *cr = &w->cor[c * nv + k];
            double N[3][3];
            corner_matrix_shape(d, g, k, N);
            const double *vp = w->vstar + p * 3;
            double f[3];
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int b = 0; b < 3; ++b)
                    s += cr->T[a][b] * g->C[k][b] + cr->z * N[a][b] * (vp[b] - cr->v[b]);
                f[a] = s;
            }
            for (int a = 0; a < 3; ++a) F[a] += f[a];
            W += dot3(f, vp);
            for (int i = 0; i < 3; ++i) {
                vsk[k][i] = vp[i];
                vhn[k][i] = i < d ? w->vhat[p * d + i] : 0.0;
                vh1[k][i] = i < d ? w->vhat1[p * d + i] : 0.0;
            }
        }
        double mc = w->m[c];
        for (int i = 0; i < d; ++i) w->v1[c * d + i] = w->v[c * d + i] + w->dt / mc * F[i];
        w->e1[c] = w->e[c] + w->dt / mc * W;
        double X1[4][3];
        orc_geo g1;
        cell_nodes(M, w->x1, c, X1);
        geometry(d, X1, &g1);
        w->tau1[c] = g1.V / mc;
        double Bn[3][3], Bnew[3][3];
        unpack_B(d, w->B + c * M->nB, Bn);
        if (mask[c] < 2) {
            double Ln[3][3], L1[3][3];
            velocity_gradient(d, g, vhn, Ln);
            velocity_gradient(d, &g1, vh1, L1);
            cn_solve(d, Bn, Ln, L1, w->dt, Bnew);
        } else {
            double Ls[3][3], Y[3][3];
            velocity_gradient(d, g, vsk, Ls);
            lie_term(Ls, Bn, Y);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Bnew[i][j] = Bn[i][j] + w->dt * Y[i][j];
            if (d == 2) Bnew[2][2] = 1.0;
        }
        pack_B(d, Bnew, w->B1 + c * M->nB);
    }
}

/* physical admissibility (eq. PAD, reading R16): 1 = inadmissible */
static int inadmissible(const orc_work *w, const orc_params *prm, int64_t c) {
    const orc_mesh *M = w->M;
    int d = M->dim;
    double vals[16];
    int n = 0;
    vals[n++] = w->tau1[c];
    vals[n++] = w->e1[c];
    for (int i = 0; i < d; ++i) vals[n++] = w->v1[c * d + i];
    for (int s = 0; s < M->nB; ++s) vals[n++] = w->B1[c * M->nB + s];
    for (int i = 0; i < n; ++i)
        if (!isfinite(vals[i])) return 1;
    if (!(w->tau1[c] > 0.0)) return 1;
    double B1[3][3];
    unpack_B(d, w->B1 + c * M->nB, B1);
    if (!(det33(B1) > 0.0)) return 1;
    double k2 = 0.0;
    for (int i = 0; i < d; ++i) k2 += w->v1[c * d + i] * w->v1[c * d + i];
    double eps = w->e1[c] - 0.5 * k2;
    if (eps < -prm->eps_tol * (fabs(w->e1[c]) + 0.5 * k2)) return 1;
    if (prm->eos) {
        /* stiffened gas (R31): hyperbolic only while p + p_inf > 0 */
        orc_mat mat = mat_of(w, c);
        if (!(sg_pressure(&mat, w->tau1[c], B1, eps) + prm->sg_pinf > 0.0)) return 1;
    }
    return 0;
}

/* detection (eqs. PAD and RDMP; readings R16, R17): 0 = accepted,
 * 1 = not physically admissible, 2 = outside the relaxed DMP bounds */
static int troubled(const orc_work *w, const orc_params *prm, int64_t c) {
    if (inadmissible(w, prm, c)) return 1;
    double rho1 = 1.0 / w->tau1[c];
    double lo = w->rmin[c], hi = w->rmax[c];
    double delta = fmax(prm->delta0, prm->delta1 * (hi - lo));
    if (rho1 < lo - delta || rho1 > hi + delta) return 2;
    return 0;
}

/* Relaxed-DMP bounds (eq. RDMP, reading R17): min and max of rho^n = 1/tau^n
 * over {c} and its reconstruction stencil, the cells sharing a node with c. */
static void rdmp_bounds(const orc_mesh *M, const double *tau, double *rmin, double *rmax) {
    int nv = M->nv;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < M->nc; ++c) {
        double lo = 1.0 / tau[c], hi = lo;
        for (int k = 0; k < nv; ++k) {
            int64_t p = M->c2n[c * nv + k];
            for (int64_t q = M->n2c_off[p]; q < M->n2c_off[p + 1]; ++q) {
                double r = 1.0 / tau[M->n2c[q] / nv];
                lo = fmin(lo, r);
                hi = fmax(hi, r);
            }
        }
        rmin[c] = lo;
        rmax[c] = hi;
    }
}

/* Involution monitors of the step just taken (Section 3.5): the discrete
 * GCL (eq. GCL) with the corner vectors averaged over the step by Simpson's
 * rule, which is exact for straight node paths (V is a cubic in time, its
 * rate sum_p C_cp(t) . v*_p a quadratic), and |sqrt(det B) - J| against
 * L_c^3 (eq. test_detB_rho, reading R19). */
static void involutions(const orc_mesh *M, const double *rho0, const double *x, const double *vstar3, double dt,
                        const double *x1, const double *tau1, const double *B1, orc_info *info) {
    int d = M->dim, nv = M->nv;
    info->gcl_defect = 0.0;
    info->detB_defect = 0.0;
    info->n_detB = 0;
    double *xh = (double *)malloc(sizeof(double) * (size_t)(M->nn * d + 1));
    for (int64_t p = 0; p < M->nn; ++p)
        for (int i = 0; i < d; ++i) xh[p * d + i] = x[p * d + i] + 0.5 * dt * vstar3[p * 3 + i];
    double gmax = 0.0, bmax = 0.0;
    int64_t ndet = 0;
#pragma omp parallel for schedule(static) reduction(max : gmax, bmax) reduction(+ : ndet)
    for (int64_t c = 0; c < M->nc; ++c) {
        double X0[4][3], Xh[4][3], X1[4][3];
        orc_geo g0, gh, g1;
        cell_nodes(M, x, c, X0);
        cell_nodes(M, xh, c, Xh);
        cell_nodes(M, x1, c, X1);
        geometry(d, X0, &g0);
        geometry(d, Xh, &gh);
        geometry(d, X1, &g1);
        double flux = 0.0;
        for (int k = 0; k < nv; ++k) {
            int64_t p = M->c2n[c * nv + k];
            for (int i = 0; i < d; ++i)
                flux += (g0.C[k][i] + 4.0 * gh.C[k][i] + g1.C[k][i]) / 6.0 * vstar3[p * 3 + i];
        }
        double gcl = fabs(g1.V - g0.V - dt * flux) / g0.V;
        if (gcl > gmax) gmax = gcl;
        double Bc[3][3];
        unpack_B(d, B1 + c * M->nB, Bc);
        double dB = fabs(sqrt(det33(Bc)) - rho0[c] * tau1[c]);
        if (dB > bmax) bmax = dB;
        if (dB >= g1.Lc * g1.Lc * g1.Lc) ndet++;
    }
    info->gcl_defect = gmax;
    info->detB_defect = bmax;
    info->n_detB = ndet;
    free(xh);
}

static void diagnostics(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
                        const orc_params *prm, const double *m, const double *tau, const double *v,
                        const double *e, const double *B, orc_info *info) {
    int d = M->dim;
    info->mass = info->energy = info->kinetic = info->elastic = 0.0;
    info->mom[0] = info->mom[1] = info->mom[2] = 0.0;
    for (int64_t c = 0; c < M->nc; ++c) {
        orc_mat mat = {rho0[c], mu[c], K[c], prm->shear_a, prm->eos, prm->sg_gamma, prm->sg_pinf};
        double Bc[3][3];
        unpack_B(d, B + c * M->nB, Bc);
        double k2 = 0.0;
        for (int i = 0; i < d; ++i) {
            info->mom[i] += m[c] * v[c * d + i];
            k2 += v[c * d + i] * v[c * d + i];
        }
        info->mass += m[c];
        info->energy += m[c] * e[c];
        info->kinetic += 0.5 * m[c] * k2;
        info->elastic += m[c] * free_energy(&mat, tau[c], Bc);
    }
}

/* Time step (eqs. CFL, CFL2; readings R20, R21).  dt_prev <= 0 requests the
 * acoustic bound only (first step). */
static void time_step(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
                      const double *x1, const double *tau1, const double *v1, const double *e1,
                      const double *B1, const double *m, const double *V0, double dt_prev,
                      const orc_params *prm, orc_info *info) {
    int d = M->dim;
    double ac = INFINITY, vol = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : ac, vol)
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x1, c, X);
        geometry(d, X, &g);
        orc_mat mat = {rho0[c], mu[c], K[c], prm->shear_a, prm->eos, prm->sg_gamma, prm->sg_pinf};
        double Bc[3][3], k2 = 0.0;
        unpack_B(d, B1 + c * M->nB, Bc);
        for (int i = 0; i < d; ++i) k2 += v1[c * d + i] * v1[c * d + i];
        double a = sound_speed(&mat, tau1[c], Bc, e1[c] - 0.5 * k2);
        ac = fmin(ac, g.Lc / a);
        if (V0) {
            double V1 = m[c] * tau1[c];
            double dV = fabs(V1 - V0[c]);
            if (dV > 0.0) vol = fmin(vol, V1 / dV);
        }
    }
    info->dt_acoustic = prm->c_cfl * ac;
    info->dt_volume = dt_prev > 0.0 ? prm->c_v * dt_prev * vol : INFINITY;
    double dt = info->dt_acoustic;
    if (dt_prev > 0.0) {
        dt = fmin(dt, info->dt_volume);
        dt = fmin(dt, (1.0 + prm->c_i) * dt_prev);
    }
    info->dt_next = dt;
}

double orc_initial_dt(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
                      const double *x, const double *tau, const double *v, const double *e, const double *B,
                      const double *m, const orc_params *prm) {
    orc_info info;
    memset(&info, 0, sizeof info);
    time_step(M, rho0, mu, K, x, tau, v, e, B, m, NULL, 0.0, prm, &info);
    return info.dt_next;
}

/* One ADER-MOOD step (Section 3.7 and Figure "sketch").
 *  mask  in: cells forced to first order; out: final cascade choice.
 *  replay != 0: take the mask as given, no detection. */
int orc_step(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
             const double *m, const double *x, const double *vhat, const double *tau,
             const double *v, const double *e, const double *B, double dt, const orc_params *prm,
             uint8_t *mask, int replay, double *x1, double *vhat1, double *tau1, double *v1,
             double *e1, double *B1, double *vstar_out, orc_info *info) {
    int d = M->dim, nv = M->nv;
    orc_work w;
    memset(&w, 0, sizeof w);
    w.M = M;
    w.rho0 = rho0;
    w.mu = mu;
    w.K = K;
    w.m = m;
    w.x = x;
    w.vhat = vhat;
    w.tau = tau;
    w.v = v;
    w.e = e;
    w.B = B;
    w.dt = dt;
    w.a = prm->shear_a;
    w.eos = prm->eos;
    w.gam = prm->sg_gamma;
    w.pinf = prm->sg_pinf;
    w.x1 = x1;
    w.vhat1 = vhat1;
    w.tau1 = tau1;
    w.v1 = v1;
    w.e1 = e1;
    w.B1 = B1;
    w.geo = (orc_geo *)malloc(sizeof(orc_geo) * (size_t)(M->nc + 1));
    w.xc = (double *)malloc(sizeof(double) * (size_t)(M->nc * 3 + 1));
    w.grad = (double *)malloc(sizeof(double) * (size_t)(M->nc * (M->nW + 1) * 3 + 1));
    w.glim = (double *)malloc(sizeof(double) * (size_t)(M->nc * (M->nW + 1) * 3 + 1));
    w.rmin = (double *)malloc(sizeof(double) * (size_t)(M->nc + 1));
    w.rmax = (double *)malloc(sizeof(double) * (size_t)(M->nc + 1));
    w.cor = (orc_corner *)malloc(sizeof(orc_corner) * (size_t)(M->nc * nv + 1));
    w.vstar = (double *)malloc(sizeof(double) * (size_t)(M->nn * 3 + 1));
    double *V0 = (double *)malloc(sizeof(double) * (size_t)(M->nc + 1));
    uint8_t *flag = (uint8_t *)calloc((size_t)M->nc + 1, 1);

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        cell_nodes(M, x, c, X);
        geometry(d, X, &w.geo[c]);
        for (int i = 0; i < 3; ++i) w.xc[c * 3 + i] = w.geo[c].xc[i];
        V0[c] = m[c] * tau[c];
    }
    lsq_gradients(M, w.xc, tau, v, B, e, w.grad);
    bj_limit(M, x, w.xc, tau, v, B, w.grad, w.glim);
    rdmp_bounds(M, tau, w.rmin, w.rmax);

    int iters = 0;
    int64_t first = -1, recomp = 0;
    uint8_t *touch = (uint8_t *)calloc((size_t)M->nn + 1, 1);
    for (;;) {
        candidate(&w, mask);
        ++iters;
        if (replay || !prm->detect) break;
        int64_t nflag = 0;
#pragma omp parallel for schedule(static) reduction(+ : nflag)
        for (int64_t c = 0; c < M->nc; ++c) {
            flag[c] = 0;
            if (mask[c] < 2 && troubled(&w, prm, c)) {
                flag[c] = 1;
                ++nflag;
            }
        }
        if (first < 0) first = nflag;
        if (nflag == 0) break;
        for (int64_t c = 0; c < M->nc; ++c)
            if (flag[c]) mask[c] = (prm->cascade == 3 && mask[c] == 0) ? 1 : 2;
        /* the next evaluation changes only the cells that share a node with
           a flagged cell (R18): count them */
        memset(touch, 0, (size_t)M->nn);
        for (int64_t c = 0; c < M->nc; ++c)
            if (flag[c])
                for (int k = 0; k < nv; ++k) touch[M->c2n[c * nv + k]] = 1;
#pragma omp parallel for schedule(static) reduction(+ : recomp)
        for (int64_t c = 0; c < M->nc; ++c) {
            int hit = 0;
            for (int k = 0; k < nv; ++k) hit |= touch[M->c2n[c * nv + k]];
            recomp += hit;
        }
    }
    free(touch);

    memset(info, 0, sizeof(*info));
    info->n_recomp = recomp;
    info->mood_iters = iters;
    info->n_flag_first = first < 0 ? 0 : first;
    for (int64_t c = 0; c < M->nc; ++c) {
        if (mask[c] == 1) info->n_lim++;
        if (mask[c] == 2) {
            info->n_p0++;
            if (inadmissible(&w, prm, c)) info->status = 1;
        }
    }
    if (vstar_out)
        for (int64_t p = 0; p < M->nn; ++p)
            for (int i = 0; i < d; ++i) vstar_out[p * d + i] = w.vstar[p * 3 + i];
    time_step(M, rho0, mu, K, x1, tau1, v1, e1, B1, m, V0, dt, prm, info);
    diagnostics(M, rho0, mu, K, prm, m, tau1, v1, e1, B1, info);
    involutions(M, rho0, x, w.vstar, dt, x1, tau1, B1, info);

    free(w.geo);
    free(w.xc);
    free(w.grad);
    free(w.glim);
    free(w.rmin);
    free(w.rmax);
    free(w.cor);
    free(w.vstar);
    free(V0);
    free(flag);
    return 0;
}

/* ------------------------------------------------------------------ */
/* unit-level entry points used by the pin tests                       */
/* ------------------------------------------------------------------ */
/* Detection of a given candidate state (eqs. PAD, RDMP; readings R16, R17)
 * with the relaxed-DMP bounds of the state tau0 at t^n: code[c] = 0
 * accepted, 1 not physically admissible, 2 outside the relaxed DMP bounds.
 * Cells at first order (mask >= 2) are accepted as the parachute. */
void orc_detect(const orc_mesh *M, const double *rho0, const double *mu, const double *K, const double *tau0,
                const double *tau1, const double *v1, const double *e1, const double *B1, const uint8_t *mask,
                const orc_params *prm, uint8_t *code) {
    orc_work w;
    memset(&w, 0, sizeof w);
    w.M = M;
    w.rho0 = rho0;
    w.mu = mu;
    w.K = K;
    w.a = prm->shear_a;
    w.eos = prm->eos;
    w.gam = prm->sg_gamma;
    w.pinf = prm->sg_pinf;
    w.tau1 = (double *)tau1;
    w.v1 = (double *)v1;
    w.e1 = (double *)e1;
    w.B1 = (double *)B1;
    w.rmin = (double *)malloc(sizeof(double) * (size_t)(M->nc + 1));
    w.rmax = (double *)malloc(sizeof(double) * (size_t)(M->nc + 1));
    rdmp_bounds(M, tau0, w.rmin, w.rmax);
    for (int64_t c = 0; c < M->nc; ++c) code[c] = (uint8_t)((mask && mask[c] >= 2) ? 0 : troubled(&w, prm, c));
    free(w.rmin);
    free(w.rmax);
}

/* Time-step control of a given end-of-step state (eqs. CFL, CFL2; R20, R21):
 * V0 (may be NULL: first step) holds V^n per cell, dt_prev the step's dt. */
void orc_time_step(const orc_mesh *M, const double *rho0, const double *mu, const double *K, const double *x1,
                   const double *tau1, const double *v1, const double *e1, const double *B1, const double *m,
                   const double *V0, double dt_prev, const orc_params *prm, orc_info *info) {
    memset(info, 0, sizeof(*info));
    time_step(M, rho0, mu, K, x1, tau1, v1, e1, B1, m, V0, dt_prev, prm, info);
}
/* X: [(d+1)][d] -> V, xc[3], C[(d+1)][3], A[(d+1)][3], Lc */
void orc_cell_geometry(int d, const double *Xin, double *V, double *xc, double *C, double *A,
                       double *Lc) {
    double X[4][3] = {{0}};
    for (int k = 0; k <= d; ++k)
        for (int i = 0; i < d; ++i) X[k][i] = Xin[k * d + i];
    orc_geo g;
    geometry(d, X, &g);
    *V = g.V;
    *Lc = g.Lc;
    memcpy(xc, g.xc, sizeof g.xc);
    for (int k = 0; k <= d; ++k)
        for (int i = 0; i < 3; ++i) {
            C[k * 3 + i] = g.C[k][i];
            A[k * 3 + i] = g.A[k][i];
        }
}

/* corner matrix M_cp / z for local node p: N[3][3] */
void orc_corner_shape(int d, const double *Xin, int p, double *N) {
    double X[4][3] = {{0}};
    for (int k = 0; k <= d; ++k)
        for (int i = 0; i < d; ++i) X[k][i] = Xin[k * d + i];
    orc_geo g;
    geometry(d, X, &g);
    double Nm[3][3];
    corner_matrix_shape(d, &g, p, Nm);
    memcpy(N, Nm, sizeof Nm);
}

/* full 3x3 B in, full 3x3 T out, plus p, a, Psi */
void orc_point_stress(double rho0, double mu, double K, double tau, const double *B, double *T,
                      double *p, double *a, double *psi, double shear_a) {
    orc_mat m = {rho0, mu, K, shear_a, 0, 0.0, 0.0};
    double Bm[3][3], Tm[3][3];
    memcpy(Bm, B, sizeof Bm);
    stress(&m, tau, Bm, 0.0, Tm);
    memcpy(T, Tm, sizeof Tm);
    *p = pressure(&m, rho0 * tau);
    *a = sound_speed(&m, tau, Bm, 0.0);
    *psi = free_energy(&m, tau, Bm);
}

void orc_point_stress_direction(double rho0, double mu, double K, double tau, const double *B,
                                double dtau, const double *dB, double *dT, double shear_a) {
    orc_mat m = {rho0, mu, K, shear_a, 0, 0.0, 0.0};
    double Bm[3][3], dBm[3][3], dTm[3][3];
    memcpy(Bm, B, sizeof Bm);
    memcpy(dBm, dB, sizeof dBm);
    stress_direction(&m, tau, Bm, 0.0, dtau, dBm, 0.0, dTm);
    memcpy(dT, dTm, sizeof dTm);
}

/* stiffened gas with the shear family (R31): T, p, a, Psi_s at (tau, B, eps) */
void orc_point_stress_sg(double rho0, double mu, double shear_a, double gam, double pinf, double tau,
                         const double *B, double eps, double *T, double *p, double *a, double *psi_s) {
    orc_mat m = {rho0, mu, 0.0, shear_a, 1, gam, pinf};
    double Bm[3][3], Tm[3][3];
    memcpy(Bm, B, sizeof Bm);
    stress(&m, tau, Bm, eps, Tm);
    memcpy(T, Tm, sizeof Tm);
    *p = sg_pressure(&m, tau, Bm, eps);
    *a = sound_speed(&m, tau, Bm, eps);
    *psi_s = shear_energy(&m, tau, Bm);
}

void orc_point_stress_direction_sg(double rho0, double mu, double shear_a, double gam, double pinf, double tau,
                                   const double *B, double eps, double dtau, const double *dB, double deps,
                                   double *dT) {
    orc_mat m = {rho0, mu, 0.0, shear_a, 1, gam, pinf};
    double Bm[3][3], dBm[3][3], dTm[3][3];
    memcpy(Bm, B, sizeof Bm);
    memcpy(dBm, dB, sizeof dBm);
    stress_direction(&m, tau, Bm, eps, dtau, dBm, deps, dTm);
    memcpy(dT, dTm, sizeof dTm);
}

/* CN update of one cell, full 3x3 matrices */
int orc_point_cn(int d, const double *Bn, const double *Ln, const double *L1, double dt,
                 double *Bout) {
    double a[3][3], b[3][3], c[3][3], o[3][3];
    memcpy(a, Bn, sizeof a);
    memcpy(b, Ln, sizeof b);
    memcpy(c, L1, sizeof c);
    int st = cn_solve(d, a, b, c, dt, o);
    memcpy(Bout, o, sizeof o);
    return st;
}

/* least-squares gradients of all cells: grad [nc][nW][3] */
void orc_lsq(const orc_mesh *M, const double *x, const double *tau, const double *v,
             const double *B, double *grad) {
    double *xc = (double *)malloc(sizeof(double) * (size_t)(M->nc * 3 + 1));
    double *gw = (double *)malloc(sizeof(double) * (size_t)(M->nc * (M->nW + 1) * 3 + 1));
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(M->dim, X, &g);
        for (int i = 0; i < 3; ++i) xc[c * 3 + i] = g.xc[i];
    }
    lsq_gradients(M, xc, tau, v, B, NULL, gw);
    for (int64_t c = 0; c < M->nc; ++c)
        memcpy(grad + c * M->nW * 3, gw + c * (M->nW + 1) * 3, sizeof(double) * M->nW * 3);
    free(gw);
    free(xc);
}

/* Barth-Jespersen limited gradients of all cells: glim [nc][nW][3] */
void orc_bj(const orc_mesh *M, const double *x, const double *tau, const double *v,
            const double *B, double *glim) {
    const int st = M->nW + 1;
    double *xc = (double *)malloc(sizeof(double) * (size_t)(M->nc * 3 + 1));
    double *grad = (double *)malloc(sizeof(double) * (size_t)(M->nc * st * 3 + 1));
    double *gl = (double *)malloc(sizeof(double) * (size_t)(M->nc * st * 3 + 1));
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(M->dim, X, &g);
        for (int i = 0; i < 3; ++i) xc[c * 3 + i] = g.xc[i];
    }
    lsq_gradients(M, xc, tau, v, B, NULL, grad);
    bj_limit(M, x, xc, tau, v, B, grad, gl);
    for (int64_t c = 0; c < M->nc; ++c)
        memcpy(glim + c * M->nW * 3, gl + c * st * 3, sizeof(double) * M->nW * 3);
    free(gl);
    free(grad);
    free(xc);
}

/* predicted corner states for every corner at the cascade level of each
 * cell (mask: 0 unlimited, 1 limited, 2 first order): tau*[nc*nv],
 * v*[nc*nv][3], B*[nc*nv][9], T*[nc*nv][9], z*[nc*nv] */
void orc_predict(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
                 const double *x, const double *tau, const double *v, const double *B, double dt,
                 double shear_a, const uint8_t *mask, double *tau_s, double *v_s, double *B_s, double *T_s,
                 double *z_s) {
    int d = M->dim, nv = M->nv, st = M->nW + 1;
    double *grad = (double *)malloc(sizeof(double) * (size_t)(M->nc * st * 3 + 1));
    double *glim = (double *)malloc(sizeof(double) * (size_t)(M->nc * st * 3 + 1));
    double *xc = (double *)malloc(sizeof(double) * (size_t)(M->nc * 3 + 1));
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(d, X, &g);
        for (int i = 0; i < 3; ++i) xc[c * 3 + i] = g.xc[i];
    }
    lsq_gradients(M, xc, tau, v, B, NULL, grad);
    bj_limit(M, x, xc, tau, v, B, grad, glim);
    free(xc);
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(d, X, &g);
        orc_mat mat = {rho0[c], mu[c], K[c], shear_a, 0, 0.0, 0.0};
        double Bc[3][3];
        unpack_B(d, B + c * M->nB, Bc);
        for (int k = 0; k < nv; ++k) {
            orc_corner cr;
            predict_corner(M, &mat, &g, X[k], tau[c], v + c * d, Bc, 0.0,
                           (mask[c] == 1 ? glim : grad) + c * st * 3, mask[c] < 2, dt, &cr);
            int64_t q = c * nv + k;
            tau_s[q] = cr.tau;
            for (int i = 0; i < 3; ++i) v_s[q * 3 + i] = cr.v[i];
            memcpy(B_s + q * 9, cr.B, sizeof cr.B);
            memcpy(T_s + q * 9, cr.T, sizeof cr.T);
            z_s[q] = cr.z;
        }
    }
    free(grad);
    free(glim);
}

/* predicted corner states with the equation of state of prm (the
 * stiffened gas needs e): tau*[nc*nv], eps*[nc*nv], T*[nc*nv][9],
 * z*[nc*nv]; mask as for orc_predict */
void orc_predict_eos(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
                     const double *x, const double *tau, const double *v, const double *e, const double *B,
                     double dt, const orc_params *prm, const uint8_t *mask, double *tau_s, double *eps_s,
                     double *T_s, double *z_s) {
    int d = M->dim, nv = M->nv, st = M->nW + 1;
    double *grad = (double *)malloc(sizeof(double) * (size_t)(M->nc * st * 3 + 1));
    double *glim = (double *)malloc(sizeof(double) * (size_t)(M->nc * st * 3 + 1));
    double *xc = (double *)malloc(sizeof(double) * (size_t)(M->nc * 3 + 1));
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(d, X, &g);
        for (int i = 0; i < 3; ++i) xc[c * 3 + i] = g.xc[i];
    }
    lsq_gradients(M, xc, tau, v, B, e, grad);
    bj_limit(M, x, xc, tau, v, B, grad, glim);
    free(xc);
    for (int64_t c = 0; c < M->nc; ++c) {
        double X[4][3];
        orc_geo g;
        cell_nodes(M, x, c, X);
        geometry(d, X, &g);
        orc_mat mat = {rho0[c], mu[c], K[c], prm->shear_a, prm->eos, prm->sg_gamma, prm->sg_pinf};
        double Bc[3][3], k2 = 0.0;
        unpack_B(d, B + c * M->nB, Bc);
        for (int i = 0; i < d; ++i) k2 += v[c * d + i] * v[c * d + i];
        for (int k = 0; k < nv; ++k) {
            orc_corner cr;
            predict_corner(M, &mat, &g, X[k], tau[c], v + c * d, Bc, e[c] - 0.5 * k2,
                           (mask[c] == 1 ? glim : grad) + c * st * 3, mask[c] < 2, dt, &cr);
            int64_t q = c * nv + k;
            tau_s[q] = cr.tau;
            eps_s[q] = cr.eps;
            memcpy(T_s + q * 9, cr.T, sizeof cr.T);
            z_s[q] = cr.z;
        }
    }
    free(grad);
    free(glim);
}

void orc_diagnostics(const orc_mesh *M, const double *rho0, const double *mu, const double *K,
                     const double *m, const double *tau, const double *v, const double *e,
                     const double *B, orc_info *info, const orc_params *prm) {
    memset(info, 0, sizeof(*info));
    diagnostics(M, rho0, mu, K, prm, m, tau, v, e, B, info);
}

int orc_info_size(void) { return (int)sizeof(orc_info); }
int orc_params_size(void) { return (int)sizeof(orc_params); }
