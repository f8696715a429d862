// hl_adjoint.hip -- reverse sweep of one ADER-MOOD step with frozen dt and
// frozen cascade choice (the forward map is then smooth): given the adjoint
// lambda^{n+1} of (x, vhat, tau, v, B) after the step, produce lambda^n and
// accumulate the adjoint of the shear modulus.  The forward intermediates
// (node aggregates, corner records, v*, x^{n+1}, vhat^{n+1}, B^{n+1}) come
// from recomputing the step with the replayed mask just before.
//
// Every pass is a gather: cells read node data, nodes read their corners in
// CSR order; per-corner adjoint contributions go to per-corner records that
// the nodes sum.  Passes:
//   A1 cells: update^T (forces, GCL volume, B update, both geometries)
//   A2 nodes: x^{n+1} = x + dt v*, vhat^{n+1} = 2 v* - vhat, nodal solve^T
//   A3 cells: predictor^T (corner stress, impedance, corner matrix, half
//             step, chain-rule div T), least-squares solve^T
//   A4 nodes: aggregates of the least-squares adjoint over the node's cells
//   A5 cells: least-squares sums^T (as neighbour and as centre), cell lambda
//   A6 nodes: node lambda from the per-corner position adjoints
#include "hl_adjoint.h"
#include "hl_kernels.h"

namespace hl {

namespace {

__device__ __forceinline__ int64_t tid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Node gathers run AG lanes per node: lane l sums the corners l, l + AG, ...
// of the node in CSR order, then a butterfly over the group gives every
// lane the same total (each partial sum pairs with its commuted twin).
constexpr int AG = 8;
template <int N>
__device__ __forceinline__ void group_sum(double (&v)[N]) {
#pragma unroll
    for (int o = 1; o < AG; o <<= 1)
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += __shfl_xor(v[n], o, AG);
}

__device__ __forceinline__ double dtof(const double *dtm, const int32_t *mesh_id, int64_t i) {
    return dtm[mesh_id ? mesh_id[i] : 0];
}

template <int D>
__device__ __forceinline__ void loadB(const double *__restrict__ B, int64_t nc, int64_t c, double b[6]) {
    if (D == 3) {
#pragma unroll
        for (int s = 0; s < 6; ++s) b[s] = B[s * nc + c];
    } else {
        b[0] = B[c];
        b[1] = B[nc + c];
        b[2] = 1.0;
        b[3] = B[2 * nc + c];
        b[4] = 0.0;
        b[5] = 0.0;
    }
}

// 6-vector slot of stored component q
template <int D>
__host__ __device__ constexpr int slot(int q) {
    return D == 3 ? q : (q == 2 ? 3 : q);
}

template <int D>
__device__ __forceinline__ void sym_mul(const double M[D == 3 ? 6 : 3], const double x[D], double y[D]) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) s += M[midx<D>(i, j)] * x[j];
        y[i] = s;
    }
}

// stored adjoint of the symmetric outer product a b^T + b a^T style term
// x -> M x: adjoint of M (stored) for y = M x with ybar: diag ybar_i x_i,
// off (i<j): ybar_i x_j + ybar_j x_i
template <int D>
__device__ __forceinline__ void sym_outer_acc(const double yb[D], const double x[D], double Mb[D == 3 ? 6 : 3]) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) Mb[midx<D>(i, j)] += (i == j) ? yb[i] * x[i] : yb[i] * x[j] + yb[j] * x[i];
}

}  // namespace

// ------------------------------------------------------------------ A1
// Cell c's part: the corner records rec (returned for the caller to store)
// and the cell record's W adjoint (stored here).
template <int D>
__device__ __forceinline__ void adj_update_cell(const StepArgs &a, const AdjArgs &j, const int64_t c,
                                                double (&rec)[D + 1][AdjArgs::CA]) {
    using Dm = Dims<D>;
    constexpr int NV = D + 1;
    constexpr int NMS = Dm::NMS;
    const int64_t nc = a.nc, nn = a.nn;
    const double m = a.mass[c];
    const double dt = dtof(a.dt, a.cell_mesh, c);
    const bool p1 = a.mask[c] == 0;
    int64_t nid[NV];
    double X0[NV][D], X1[NV][D], vs[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        nid[k] = a.c2n[c * NV + k];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            X0[k][i] = a.x[i * nn + nid[k]];
            X1[k][i] = a.x1[i * nn + nid[k]];
            vs[k][i] = a.vstar[i * nn + nid[k]];
        }
    }
    // forces: v1 = v + dt/m sum_k (M_k v*_k - r_k)
    double fb[D];
#pragma unroll
    for (int i = 0; i < D; ++i) fb[i] = dt / m * j.lv_in[i * nc + c];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int q = 0; q < AdjArgs::CA; ++q) rec[k][q] = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double *cr = a.corner + corner_slot<D>(c, k) * Dm::CW;
        double Mk[NMS];
#pragma unroll
        for (int q = 0; q < NMS; ++q) Mk[q] = cr[q];
        double Mf[D];
        sym_mul<D>(Mk, fb, Mf);
        double Mb[NMS] = {};
        sym_outer_acc<D>(fb, vs[k], Mb);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            rec[k][AdjArgs::O_VS + i] += Mf[i];
            rec[k][AdjArgs::O_R + i] = -fb[i];
        }
#pragma unroll
        for (int q = 0; q < NMS; ++q) rec[k][AdjArgs::O_M + q] = Mb[q];
    }
    // geometry, GCL volume, B update
    Geo<D> g0, g1;
    geom<D>(X0, g0);
    geom<D>(X1, g1);
    double C0b[NV][D] = {}, C1b[NV][D] = {};
    double V0b = 0.0, V1b = j.ltau_in[c] / m;
    double b[6], b1[6], b1b[6] = {0, 0, 0, 0, 0, 0}, bb[6] = {0, 0, 0, 0, 0, 0};
    loadB<D>(a.B, nc, c, b);
    loadB<D>(a.B1, nc, c, b1);
#pragma unroll
    for (int q = 0; q < Dm::NB; ++q) b1b[slot<D>(q)] = j.lB_in[q * nc + c];
    double u0[NV][D], u1[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            u0[k][i] = p1 ? a.vhat[i * nn + nid[k]] : vs[k][i];
            u1[k][i] = p1 ? a.vhat1[i * nn + nid[k]] : 0.0;
        }
    double L0[D][D], L1[D][D], L0b[D][D] = {}, L1b[D][D] = {};
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int q = 0; q < D; ++q) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                s0 += u0[k][i] * g0.C[k][q];
                s1 += u1[k][i] * g1.C[k][q];
            }
            L0[i][q] = s0 / g0.V;
            L1[i][q] = s1 / g1.V;
        }
    if (p1)
        cn_vjp<D>(b, L0, L1, 0.5 * dt, b1, b1b, bb, L0b, L1b);
    else
        euler_vjp<D>(b, L0, dt, b1b, bb, L0b);
    // L = (1/V) sum_k u_k (x) C_k
    double l0l = 0.0, l1l = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int q = 0; q < D; ++q) {
            l0l += L0b[i][q] * L0[i][q];
            l1l += L1b[i][q] * L1[i][q];
        }
    V0b -= l0l / g0.V;
    V1b -= l1l / g1.V;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double su0 = 0.0, su1 = 0.0, sc0 = 0.0, sc1 = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                su0 += L0b[i][q] * g0.C[k][q];
                su1 += L1b[i][q] * g1.C[k][q];
                sc0 += L0b[q][i] * u0[k][q];
                sc1 += L1b[q][i] * u1[k][q];
            }
            // i indexes the velocity component for su*, the C component for sc*
            if (p1) {
                rec[k][AdjArgs::O_VH0 + i] += su0 / g0.V;
            } else {
                rec[k][AdjArgs::O_VS + i] += su0 / g0.V;
            }
            rec[k][AdjArgs::O_VH1 + i] += su1 / g1.V;
            C0b[k][i] += sc0 / g0.V;
            C1b[k][i] += sc1 / g1.V;
        }
    double X0b[NV][D] = {}, X1b[NV][D] = {};
    geom_vjp<D>(X0, C0b, V0b, X0b);
    geom_vjp<D>(X1, C1b, V1b, X1b);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            rec[k][AdjArgs::O_X0 + i] = X0b[k][i];
            rec[k][AdjArgs::O_X1 + i] = X1b[k][i];
        }
    }
    // cell partial adjoint of W = (tau, v, B): v1 = v + ..., B via the update
    double *cw = j.cell + c * AdjArgs::CL + AdjArgs::O_WB;
    cw[0] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) cw[1 + i] = j.lv_in[i * nc + c];
#pragma unroll
    for (int q = 0; q < Dm::NB; ++q) cw[1 + D + q] = bb[slot<D>(q)];
}

// The block's corner records go out corner by corner through LDS: a
// thread that wrote its own 192-byte record made every wave store touch
// one cache line per lane; copied out in address order, 16 bytes per lane,
// a wave store covers about five whole records.
constexpr int ADJ_UB = 256;
template <int D>
__global__ __launch_bounds__(ADJ_UB) void k_adj_update(StepArgs a, AdjArgs j) {
    constexpr int NV = D + 1, CA = AdjArgs::CA, CP = CA / 2;
    static_assert(CA % 2 == 0, "corner adjoint records hold value pairs");
    __shared__ double2 st[ADJ_UB * CP];
    const int64_t c0 = (int64_t)blockIdx.x * ADJ_UB, c = c0 + threadIdx.x;
    const bool live = c < a.nc;
    double rec[NV][CA];
    if (live) adj_update_cell<D>(a, j, c, rec);
    const int ncell = (int)min((int64_t)ADJ_UB, a.nc - c0);
    double2 *dst = reinterpret_cast<double2 *>(j.cadj);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        __syncthreads();  // the previous corner's copy-out has read st
        if (live) {
#pragma unroll
            for (int q = 0; q < CP; ++q) st[threadIdx.x * CP + q] = make_double2(rec[k][2 * q], rec[k][2 * q + 1]);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < ncell * CP; r += ADJ_UB) {
            const int ci = r / CP, q = r - ci * CP;
            dst[((c0 + ci) * NV + k) * CP + q] = st[r];
        }
    }
}

// ------------------------------------------------------------------ A2
template <int D>
__global__ __launch_bounds__(256) void k_adj_node1(StepArgs a, AdjArgs j) {
    using Dm = Dims<D>;
    constexpr int NMS = Dm::NMS;
    const int64_t p = tid() / AG;  // the group's lanes share p: they exit together
    const int l = (int)(threadIdx.x & (AG - 1));
    if (p >= a.nn) return;
    const int64_t nn = a.nn;
    const double dt = dtof(a.dt, a.node_mesh, p);
    // corner sums: x1b, vh1b, v*b, x0b, vh0b (D each), then M
    double acc[5 * D + NMS] = {};
    const int32_t q0 = a.n2c_off[p], q1 = a.n2c_off[p + 1];
    for (int32_t q = q0 + l; q < q1; q += AG) {
        const int64_t cid = a.n2c[q];
        const double *r = j.cadj + cid * AdjArgs::CA;
        const double *cr = a.corner + corner_slot_of<D>(cid) * Dm::CW;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            acc[i] += r[AdjArgs::O_X1 + i];
            acc[D + i] += r[AdjArgs::O_VH1 + i];
            acc[2 * D + i] += r[AdjArgs::O_VS + i];
            acc[3 * D + i] += r[AdjArgs::O_X0 + i];
            acc[4 * D + i] += r[AdjArgs::O_VH0 + i];
        }
#pragma unroll
        for (int s = 0; s < NMS; ++s) acc[5 * D + s] += cr[s];
    }
    group_sum(acc);
    double x1b[D], vh1b[D], M[NMS];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        x1b[i] = j.lx_in[i * nn + p] + acc[i];
        vh1b[i] = j.lvh_in[i * nn + p] + acc[D + i];
    }
#pragma unroll
    for (int s = 0; s < NMS; ++s) M[s] = acc[5 * D + s];
    double v[D], vb[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        v[i] = a.vstar[i * nn + p];
        vb[i] = dt * x1b[i] + 2.0 * vh1b[i] + acc[2 * D + i];
        if (l == i) {
            j.lx_out[i * nn + p] = x1b[i] + acc[3 * D + i];
            j.lvh_out[i * nn + p] = -vh1b[i] + acc[4 * D + i];
        }
    }
    double rb[D] = {}, Mb[NMS] = {};
    if (q1 > q0) node_solve_vjp<D>(M, a.allow + p * D * D, a.nallow[p], v, vb, rb, Mb);
    double *o = j.nadj + p * AdjArgs::NAD;
    if (l == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) o[i] = rb[i];
#pragma unroll
        for (int s = 0; s < NMS; ++s) o[D + s] = Mb[s];
    }
}

// ------------------------------------------------------------------ A3
// The reverse corner loop's accumulators (W0bar, gradbar) live in LDS, a
// column per thread: in registers, next to the forward values, they made
// the kernel spill.
constexpr int ADJ_PB = 128;   // threads per block of k_adj_predict

template <int D>
constexpr int adj_pred_nacc() {
    return Dims<D>::NW * (D + 1) + 2 * (D + 1) * D;
}

// Cell c's part: the accumulators live in the block's LDS (acc_lds,
// ADJ_PB-strided), the cell's xadj values and its cell record are returned
// for the caller to store, mu_bar is updated here.
template <int D>
__device__ __forceinline__ void adj_predict_cell(const StepArgs &a, const AdjArgs &j, const int64_t c,
                                                 double *acc_lds, double (&xo)[(D + 1) * D],
                                                 double (&cl)[AdjArgs::CL]) {
    using Dm = Dims<D>;
    constexpr int NV = D + 1;
    constexpr int NMS = Dm::NMS;
    constexpr int NW = Dm::NW;
    double *acc = acc_lds + threadIdx.x;
    auto W0b = [&](int w) -> double & { return acc[w * ADJ_PB]; };
    auto gradb = [&](int w, int q) -> double & { return acc[(Dims<D>::NW + w * D + q) * ADJ_PB]; };
    auto Cb = [&](int k, int q) -> double & { return acc[(Dims<D>::NW * (D + 1) + k * D + q) * ADJ_PB]; };
    auto Xb = [&](int k, int q) -> double & {
        return acc[(Dims<D>::NW * (D + 1) + (D + 1) * D + k * D + q) * ADJ_PB];
    };
    const int64_t nc = a.nc, nn = a.nn;
    int64_t nid[NV];
    double X[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        nid[k] = a.c2n[c * NV + k];
#pragma unroll
        for (int i = 0; i < D; ++i) X[k][i] = a.x[i * nn + nid[k]];
    }
    Geo<D> g;
    geom<D>(X, g);
    double xc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) s += X[k][i];
        xc[i] = s * (1.0 / NV);
    }
    double dl[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) dl[k][i] = X[k][i] - xc[i];
    const double tau = a.tau[c];
    double b[6];
    loadB<D>(a.B, nc, c, b);
    const double rho0 = a.rho0[c], mu = a.mu[c], K = a.K[c];
    const bool p1 = a.mask[c] == 0;
    const double h = 0.5 * dtof(a.dt, a.cell_mesh, c);
    double Wc[NW];
    Wc[0] = tau;
#pragma unroll
    for (int i = 0; i < D; ++i) Wc[1 + i] = a.v[i * nc + c];
#pragma unroll
    for (int q = 0; q < Dm::NB; ++q) Wc[1 + D + q] = b[slot<D>(q)];

    // ---- forward: least squares and half step (as in the predictor)
    double grad[NW][D];
    double A[NMS] = {}, inv[NMS] = {};
    bool ok = false;
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int i = 0; i < D; ++i) grad[w][i] = 0.0;
    double W0[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) W0[w] = Wc[w];
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double gt[D], gB[6][D], divT[D];
    if (p1) {
        double rhs[NW][D] = {};
        double visits = 0.0;
        for (int k = 0; k < NV; ++k) {
            const int64_t p = a.c2n[c * NV + k];
            double u[D];
#pragma unroll
            for (int i = 0; i < D; ++i) u[i] = xc[i] - a.x[i * nn + p];
            const AggRef ag(a.agg, nn, p);
            const double n = ag[0];
            visits += n - 1.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int q = i; q < D; ++q)
                    A[midx<D>(i, q)] += ag[Dm::O_SYY + midx<D>(i, q)] - u[i] * ag[Dm::O_SY + q] -
                                        ag[Dm::O_SY + i] * u[q] + n * u[i] * u[q];
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int q = 0; q < D; ++q)
                    rhs[w][q] += ag[Dm::O_SYW + w * D + q] - u[q] * ag[Dm::O_SW + w] - ag[Dm::O_SY + q] * Wc[w] +
                                 n * u[q] * Wc[w];
        }
        double det, tr = 0.0;
        det = D == 3 ? sym_inv3(A, inv) : sym_inv2(A, inv);
#pragma unroll
        for (int i = 0; i < D; ++i) tr += A[midx<D>(i, i)];
        const double scl = tr / D;
        const double scale = D == 3 ? scl * scl * scl : scl * scl;
        ok = (visits >= D) && (tr > 0.0) && (det > 1e-12 * scale);
        if (ok) {
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < D; ++q) s += inv[midx<D>(i, q)] * rhs[w][q];
                    grad[w][i] = s;
                }
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = 0; q < D; ++q) G[i][q] = grad[1 + i][q];
#pragma unroll
        for (int i = 0; i < D; ++i) gt[i] = grad[0][i];
#pragma unroll
        for (int s = 0; s < 6; ++s)
#pragma unroll
            for (int q = 0; q < D; ++q) gB[s][q] = 0.0;
#pragma unroll
        for (int qq = 0; qq < Dm::NB; ++qq)
#pragma unroll
            for (int q = 0; q < D; ++q) gB[slot<D>(qq)][q] = grad[1 + D + qq][q];
        double trG = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) trG += G[i][i];
        divT_fwd<D>(rho0, mu, K, tau, b, gt, gB, divT);
        W0[0] += h * tau * trG;
#pragma unroll
        for (int i = 0; i < D; ++i) W0[1 + i] += h * tau * divT[i];
        double Gd[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = 0; q < D; ++q) Gd[i][q] = G[i][q];
        constexpr int N = D == 3 ? 6 : 3;
        double MG[N][N];
        lie_matrix<D>(Gd, MG);
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double y = 0.0;
#pragma unroll
            for (int s = 0; s < N; ++s) y += MG[r][s] * b[slot<D>(s)];
            W0[1 + D + r] += h * y;
        }
    }
    double S[NMS] = {};
#pragma unroll
    for (int jj = 0; jj < NV; ++jj)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = i; q < D; ++q) S[midx<D>(i, q)] += g.C[jj][i] * g.C[jj][q] / g.cn[jj];

    // ---- reverse over the corners
    for (int e = 0; e < adj_pred_nacc<D>(); ++e) acc[e * ADJ_PB] = 0.0;
    double xcb[D] = {};
    double mub = 0.0, Kb = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double Wk[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            double s = W0[w];
#pragma unroll
            for (int q = 0; q < D; ++q) s += grad[w][q] * dl[k][q];
            Wk[w] = s;
        }
        double bk[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) bk[s] = b[s];
#pragma unroll
        for (int q = 0; q < Dm::NB; ++q) bk[slot<D>(q)] = Wk[1 + D + q];
        double T[6];
        stress6(rho0, mu, K, Wk[0], bk, T);
        const double z = impedance(rho0, mu, K, Wk[0]);
        double N[NMS];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = i; q < D; ++q)
                N[midx<D>(i, q)] = S[midx<D>(i, q)] - g.C[k][i] * g.C[k][q] / g.cn[k];
        double Mk[NMS];
#pragma unroll
        for (int s = 0; s < NMS; ++s) Mk[s] = z * N[s];
        // adjoints of M_k and r_k: corner part (update) + node part (solve)
        const double *cr = j.cadj + (c * NV + k) * AdjArgs::CA;
        const double *nr = j.nadj + nid[k] * AdjArgs::NAD;
        double Mb[NMS], rb[D];
#pragma unroll
        for (int s = 0; s < NMS; ++s) Mb[s] = cr[AdjArgs::O_M + s] + nr[D + s];
#pragma unroll
        for (int i = 0; i < D; ++i) rb[i] = cr[AdjArgs::O_R + i] + nr[i];
        // r = M v - T C
        double vk[D];
#pragma unroll
        for (int i = 0; i < D; ++i) vk[i] = Wk[1 + i];
        sym_outer_acc<D>(rb, vk, Mb);
        double vkb[D];
        sym_mul<D>(Mk, rb, vkb);
        double Tb[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = i; q < D; ++q)
                Tb[sidx(i, q)] -= (i == q) ? rb[i] * g.C[k][i] : rb[i] * g.C[k][q] + rb[q] * g.C[k][i];
#pragma unroll
        for (int q = 0; q < D; ++q) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) s += rb[i] * T[sidx(i, q)];
            Cb(k, q) -= s;
        }
        // M = z N
        double zb = 0.0, Nb[NMS];
#pragma unroll
        for (int s = 0; s < NMS; ++s) {
            zb += Mb[s] * N[s];
            Nb[s] = z * Mb[s];
        }
        // N_k = sum_{jj != k} C_jj C_jj^T / |C_jj|
#pragma unroll
        for (int jj = 0; jj < NV; ++jj) {
            if (jj == k) continue;
            double cbj[D];
#pragma unroll
            for (int q = 0; q < D; ++q) cbj[q] = Cb(jj, q);
            outer_norm_vjp<D>(g.C[jj], Nb, cbj);
#pragma unroll
            for (int q = 0; q < D; ++q) Cb(jj, q) = cbj[q];
        }
        double taub = 0.0, bkb[6] = {0, 0, 0, 0, 0, 0};
        impedance_vjp(rho0, mu, K, Wk[0], zb, taub, mub, Kb);
        stress6_vjp(rho0, mu, K, Wk[0], bk, Tb, taub, bkb, mub, Kb);
        double Wkb[NW];
        Wkb[0] = taub;
#pragma unroll
        for (int i = 0; i < D; ++i) Wkb[1 + i] = vkb[i];
#pragma unroll
        for (int q = 0; q < Dm::NB; ++q) Wkb[1 + D + q] = bkb[slot<D>(q)];
#pragma unroll
        for (int w = 0; w < NW; ++w) W0b(w) += Wkb[w];
        if (p1) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    gradb(w, q) += Wkb[w] * dl[k][q];
                    s += grad[w][q] * Wkb[w];
                }
                Xb(k, q) += s;
                xcb[q] -= s;
            }
        }
    }

    // ---- half step W0 = Wc + h dW/dt and the least-squares solve
    double Wcb[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) Wcb[w] = W0b(w);
    double bbar[NW][D] = {}, Ahat[NMS] = {};
    if (p1) {
        double trG = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) trG += G[i][i];
        double Gb[D][D] = {};
        // tau: W0[0] = tau + h tau tr G
        Wcb[0] += W0b(0) * h * trG;
#pragma unroll
        for (int i = 0; i < D; ++i) Gb[i][i] += W0b(0) * h * tau;
        // v: W0[1+i] = v_i + h tau divT_i
        double dvb[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            Wcb[0] += W0b(1 + i) * h * divT[i];
            dvb[i] = W0b(1 + i) * h * tau;
        }
        double taub = 0.0, bb6[6] = {0, 0, 0, 0, 0, 0}, gtb[D] = {}, gBb[6][D] = {};
        divT_vjp<D>(rho0, mu, K, tau, b, gt, gB, dvb, taub, bb6, gtb, gBb, mub, Kb);
        Wcb[0] += taub;
        // B: W0_B = b + h Mat(G) b
        constexpr int N = D == 3 ? 6 : 3;
        double Gd[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = 0; q < D; ++q) Gd[i][q] = G[i][q];
        double MG[N][N], MGb[N][N];
        lie_matrix<D>(Gd, MG);
#pragma unroll
        for (int s = 0; s < N; ++s) {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < N; ++r) t += h * MG[r][s] * W0b(1 + D + r);
            bb6[slot<D>(s)] += t;
#pragma unroll
            for (int r = 0; r < N; ++r) MGb[r][s] = h * W0b(1 + D + r) * b[slot<D>(s)];
        }
        lie_matrix_T<D>(MGb, Gb);
#pragma unroll
        for (int q = 0; q < Dm::NB; ++q) Wcb[1 + D + q] += bb6[slot<D>(q)];
        // gradients
#pragma unroll
        for (int i = 0; i < D; ++i) {
            gradb(0, i) += gtb[i];
#pragma unroll
            for (int q = 0; q < D; ++q) gradb(1 + i, q) += Gb[i][q];
        }
#pragma unroll
        for (int qq = 0; qq < Dm::NB; ++qq)
#pragma unroll
            for (int q = 0; q < D; ++q) gradb(1 + D + qq, q) += gBb[slot<D>(qq)][q];
        if (ok) {
            // g = A^{-1} b  ->  bbar = A^{-1} gbar, Abar = -sum_w bbar_w g_w^T
            double Ab[D][D] = {};
#pragma unroll
            for (int w = 0; w < NW; ++w) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < D; ++q) s += inv[midx<D>(i, q)] * gradb(w, q);
                    bbar[w][i] = s;
                }
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int q = 0; q < D; ++q) Ab[i][q] -= bbar[w][i] * grad[w][q];
            }
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int q = i; q < D; ++q) Ahat[midx<D>(i, q)] = Ab[i][q] + Ab[q][i];
        }
    }

    // ---- geometry of the corner vectors and the centroid
    double Xg[NV][D] = {};
    double Cbl[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int q = 0; q < D; ++q) Cbl[k][q] = Cb(k, q);
    geom_vjp<D>(X, Cbl, 0.0, Xg);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) xo[k * D + i] = Xb(k, i) + Xg[k][i] + xcb[i] * (1.0 / NV);
    const double *clg = j.cell + c * AdjArgs::CL;
#pragma unroll
    for (int q = 0; q < AdjArgs::CL; ++q) cl[q] = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int i = 0; i < D; ++i) cl[AdjArgs::O_BB + w * D + i] = bbar[w][i];
#pragma unroll
    for (int s = 0; s < NMS; ++s) cl[AdjArgs::O_AH + s] = Ahat[s];
#pragma unroll
    for (int w = 0; w < NW; ++w) cl[AdjArgs::O_WB + w] = clg[AdjArgs::O_WB + w] + Wcb[w];
    // K = lambda + 2 mu / 3
    j.mu_bar[c] += mub + (2.0 / 3.0) * Kb;
}

// The block's cell records and xadj values go out through LDS (the
// accumulators' space, free once every thread is done) in address order,
// 16 bytes per lane, instead of one 368-byte record per lane.
template <int D>
__global__ __launch_bounds__(ADJ_PB) void k_adj_predict(StepArgs a, AdjArgs j) {
    constexpr int NACC = adj_pred_nacc<D>();
    constexpr int CL = AdjArgs::CL, XA = (D + 1) * D;
    constexpr int NST = NACC > CL ? NACC : CL;
    static_assert(CL % 2 == 0 && XA % 2 == 0, "records hold value pairs");
    __shared__ double acc_lds[ADJ_PB * NST];
    const int64_t c0 = (int64_t)blockIdx.x * ADJ_PB, c = c0 + threadIdx.x;
    const bool live = c < a.nc;
    double xo[XA], cl[CL];
    if (live) adj_predict_cell<D>(a, j, c, acc_lds, xo, cl);
    const int ncell = (int)min((int64_t)ADJ_PB, a.nc - c0);
    double2 *st = reinterpret_cast<double2 *>(acc_lds);
    __syncthreads();  // every thread is done with its accumulators
    if (live) {
#pragma unroll
        for (int q = 0; q < CL / 2; ++q) st[threadIdx.x * (CL / 2) + q] = make_double2(cl[2 * q], cl[2 * q + 1]);
    }
    __syncthreads();
    double2 *dcl = reinterpret_cast<double2 *>(j.cell) + c0 * (CL / 2);
    for (int r = threadIdx.x; r < ncell * (CL / 2); r += ADJ_PB) dcl[r] = st[r];
    __syncthreads();
    if (live) {
#pragma unroll
        for (int q = 0; q < XA / 2; ++q) st[threadIdx.x * (XA / 2) + q] = make_double2(xo[2 * q], xo[2 * q + 1]);
    }
    __syncthreads();
    double2 *dx = reinterpret_cast<double2 *>(j.xadj) + c0 * (XA / 2);
    for (int r = threadIdx.x; r < ncell * (XA / 2); r += ADJ_PB) dx[r] = st[r];
}

// ------------------------------------------------------------------ A4
template <int D>
__global__ __launch_bounds__(256) void k_adj_agg(StepArgs a, AdjArgs j) {
    using Dm = Dims<D>;
    constexpr int NV = D + 1;
    constexpr int NMS = Dm::NMS;
    constexpr int NW = Dm::NW;
    const int64_t p = tid() / AG;  // the group's lanes share p: they exit together
    const int l = (int)(threadIdx.x & (AG - 1));
    if (p >= a.nn) return;
    const int64_t nn = a.nn, nc = a.nc;
    double xp[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xp[i] = a.x[i * nn + p];
    // SB[NW][D], SYB[NW], SBW[D], SA[NMS], SAY[D] in one array
    constexpr int OB = 0, OYB = NW * D, OBW = OYB + NW, OA = OBW + D, OAY = OA + NMS, NS = OAY + D;
    static_assert(NS == AdjArgs::NAA || D == 2, "aggregate adjoint record");
    double S[NS] = {};
    const int32_t q0 = a.n2c_off[p], q1 = a.n2c_off[p + 1];
    for (int32_t q = q0 + l; q < q1; q += AG) {
        const int64_t c = a.n2c[q] / NV;
        double y[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) s += a.x[i * nn + a.c2n[c * NV + k]];
            y[i] = s * (1.0 / NV) - xp[i];
        }
        double W[NW];
        W[0] = a.tau[c];
#pragma unroll
        for (int i = 0; i < D; ++i) W[1 + i] = a.v[i * nc + c];
#pragma unroll
        for (int qq = 0; qq < Dm::NB; ++qq) W[1 + D + qq] = a.B[qq * nc + c];
        const double *cl = j.cell + c * AdjArgs::CL;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            double yb = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double bw = cl[AdjArgs::O_BB + w * D + i];
                S[OB + w * D + i] += bw;
                yb += y[i] * bw;
                S[OBW + i] += W[w] * bw;
            }
            S[OYB + w] += yb;
        }
        double Ah[NMS], Ay[D];
#pragma unroll
        for (int s = 0; s < NMS; ++s) {
            Ah[s] = cl[AdjArgs::O_AH + s];
            S[OA + s] += Ah[s];
        }
        sym_mul<D>(Ah, y, Ay);
#pragma unroll
        for (int i = 0; i < D; ++i) S[OAY + i] += Ay[i];
    }
    group_sum(S);
    // same record order as before: SB, SYB, SBW, SA, SAY, stored as pairs
    // of values interleaved over the nodes like the forward aggregates
    // (pair i of node p at i nn + p), so that the cells' gathers of them
    // bring a few cache lines per wave instead of one per lane; lane l
    // writes the values l, l + AG, ...
    double *o = j.agg;
#pragma unroll
    for (int t = 0; t < NS; ++t)
        if ((t & (AG - 1)) == l) o[((int64_t)(t >> 1) * nn + p) * 2 + (t & 1)] = S[t];
}

// ------------------------------------------------------------------ A5
template <int D>
__global__ __launch_bounds__(256) void k_adj_lsq(StepArgs a, AdjArgs j) {
    using Dm = Dims<D>;
    constexpr int NV = D + 1;
    constexpr int NMS = Dm::NMS;
    constexpr int NW = Dm::NW;
    const int64_t c = tid();
    if (c >= a.nc) return;
    const int64_t nn = a.nn, nc = a.nc;
    double X[NV][D], xc[D];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) X[k][i] = a.x[i * nn + a.c2n[c * NV + k]];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) s += X[k][i];
        xc[i] = s * (1.0 / NV);
    }
    double W[NW];
    W[0] = a.tau[c];
#pragma unroll
    for (int i = 0; i < D; ++i) W[1 + i] = a.v[i * nc + c];
#pragma unroll
    for (int qq = 0; qq < Dm::NB; ++qq) W[1 + D + qq] = a.B[qq * nc + c];
    const double *cl = j.cell + c * AdjArgs::CL;
    double Wb[NW], bb[NW][D], Ah[NMS];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        Wb[w] = cl[AdjArgs::O_WB + w];
#pragma unroll
        for (int i = 0; i < D; ++i) bb[w][i] = cl[AdjArgs::O_BB + w * D + i];
    }
#pragma unroll
    for (int s = 0; s < NMS; ++s) Ah[s] = cl[AdjArgs::O_AH + s];
    double xcb[D] = {};
    double sd[D] = {}, sdW[NW] = {};  // sum_j d_kj and sum_j (W_j - W_k) over the stencil
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int64_t p = a.c2n[c * NV + k];
        double y[D];
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = xc[i] - X[k][i];
        const AggRef ad(j.agg, a.nn, p);
        const AggRef fg(a.agg, a.nn, p);
        const double n = fg[0];
        // as a neighbour of the cells around p
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            double s = -ad[NW * D + w];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                s += y[i] * ad[w * D + i];
                xcb[i] += W[w] * ad[w * D + i];
            }
            Wb[w] += s;
        }
        double SA[NMS], SAy[D];
#pragma unroll
        for (int s = 0; s < NMS; ++s) SA[s] = ad[NW * D + NW + D + s];
        sym_mul<D>(SA, y, SAy);
#pragma unroll
        for (int i = 0; i < D; ++i) xcb[i] += -ad[NW * D + NW + i] + SAy[i] - ad[NW * D + NW + D + NMS + i];
        // as the centre: stencil sums from the forward aggregates
#pragma unroll
        for (int i = 0; i < D; ++i) sd[i] += fg[Dm::O_SY + i] - n * y[i];
#pragma unroll
        for (int w = 0; w < NW; ++w) sdW[w] += fg[Dm::O_SW + w] - n * W[w];
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            s += bb[w][i] * sd[i];
            xcb[i] -= bb[w][i] * sdW[w];
        }
        Wb[w] -= s;
    }
    double Asd[D];
    sym_mul<D>(Ah, sd, Asd);
#pragma unroll
    for (int i = 0; i < D; ++i) xcb[i] -= Asd[i];
    // lambda of the cell state at t^n
    j.ltau_out[c] = Wb[0];
#pragma unroll
    for (int i = 0; i < D; ++i) j.lv_out[i * nc + c] = Wb[1 + i];
#pragma unroll
    for (int qq = 0; qq < Dm::NB; ++qq) j.lB_out[qq * nc + c] = Wb[1 + D + qq];
    double *xo = j.xadj + c * NV * D;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) xo[k * D + i] += xcb[i] * (1.0 / NV);
}

// ------------------------------------------------------------------ A6
template <int D>
__global__ __launch_bounds__(256) void k_adj_node2(StepArgs a, AdjArgs j) {
    const int64_t p = tid() / AG;  // the group's lanes share p: they exit together
    const int l = (int)(threadIdx.x & (AG - 1));
    if (p >= a.nn) return;
    const int64_t nn = a.nn;
    double s[D] = {};
    const int32_t q0 = a.n2c_off[p], q1 = a.n2c_off[p + 1];
    for (int32_t q = q0 + l; q < q1; q += AG) {
        const double *xo = j.xadj + (int64_t)a.n2c[q] * D;
#pragma unroll
        for (int i = 0; i < D; ++i) s[i] += xo[i];
    }
    group_sum(s);
#pragma unroll
    for (int i = 0; i < D; ++i)
        if (l == i) j.lx_out[i * nn + p] += s[i];
}

// initial-state adjoint of the node velocity: projection on allowed directions
template <int D>
__global__ void k_adj_project(int64_t nn, const uint8_t *__restrict__ nallow, const double *__restrict__ allow,
                              const double *__restrict__ lvh, double *__restrict__ out /* AoS [nn][D] */) {
    const int64_t p = tid();
    if (p >= nn) return;
    const double *P = allow + p * D * D;
    double o[D] = {};
    for (int t = 0; t < nallow[p]; ++t) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s += P[i * D + t] * lvh[i * nn + p];
#pragma unroll
        for (int i = 0; i < D; ++i) o[i] += s * P[i * D + t];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) out[p * D + i] = o[i];
}

static inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int D>
void launch_adjoint_step(const StepArgs &a, const AdjArgs &j, hipStream_t s) {
    if (a.nc) k_adj_update<D><<<(unsigned)((a.nc + ADJ_UB - 1) / ADJ_UB), ADJ_UB, 0, s>>>(a, j);
    if (a.nn) k_adj_node1<D><<<nb(AG * a.nn), 256, 0, s>>>(a, j);
    if (a.nc) k_adj_predict<D><<<(unsigned)((a.nc + ADJ_PB - 1) / ADJ_PB), ADJ_PB, 0, s>>>(a, j);
    if (a.nn) k_adj_agg<D><<<nb(AG * a.nn), 256, 0, s>>>(a, j);
    if (a.nc) k_adj_lsq<D><<<nb(a.nc), 256, 0, s>>>(a, j);
    if (a.nn) k_adj_node2<D><<<nb(AG * a.nn), 256, 0, s>>>(a, j);
}

template <int D>
void launch_adj_project(int64_t nn, const uint8_t *nallow, const double *allow, const double *lvh, double *out,
                        hipStream_t s) {
    if (nn) k_adj_project<D><<<nb(nn), 256, 0, s>>>(nn, nallow, allow, lvh, out);
}

template void launch_adjoint_step<2>(const StepArgs &, const AdjArgs &, hipStream_t);
template void launch_adjoint_step<3>(const StepArgs &, const AdjArgs &, hipStream_t);
template void launch_adj_project<2>(int64_t, const uint8_t *, const double *, const double *, double *, hipStream_t);
template void launch_adj_project<3>(int64_t, const uint8_t *, const double *, const double *, double *, hipStream_t);

}  // namespace hl
