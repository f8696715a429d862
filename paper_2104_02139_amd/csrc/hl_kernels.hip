// hl_kernels.hip -- HIP kernels of one cell-centred Lagrangian ADER-MOOD
// step (Boscheri, Loubere & Maire, arXiv 2104.02139) for gfx950, FP64.
//
// Data layout in HBM (structure of arrays unless noted):
//   x, vhat, vstar : [D][n_nodes]            node vectors
//   tau, e         : [n_cells]               cell scalars
//   v              : [D][n_cells]            cell velocity
//   B              : [NB][n_cells]           left Cauchy-Green, stored comps
//   c2n            : [n_cells][D+1] int32    cell -> node
//   n2c_off, n2c   : CSR node -> corner id (corner = c*(D+1) + k), corners of
//                    a node in ascending cell order
//   agg            : [n_nodes][NA]           per-node least-squares sums
//   corner         : [n_cells*(D+1)][CW]     per-corner M_cp (sym DxD) and
//                    r_cp = M_cp v*_cp - T*_cp C_cp
// Every sum over a node's corners runs in CSR order and every sum over a
// cell's nodes in local order, so results do not depend on the launch
// shape and there are no floating-point atomics (only an integer-coded
// minimum, which is order independent).
#include "hl_device.h"
#include "hl_kernels.h"

#include <algorithm>

namespace hl {

__device__ __forceinline__ int64_t gtid() {
    return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}

// Block coordinates of a launch, or of one part of a launch that runs the
// stages of two contexts together (k_pair): the block's number within its
// part and the part's block count.  Parts start at a multiple of 8 blocks,
// so id & 7 still names the block's XCD.
struct Blk {
    int64_t id, n;
    __device__ __forceinline__ int64_t tid() const { return id * blockDim.x + threadIdx.x; }
    __device__ __forceinline__ int64_t stride() const { return n * blockDim.x; }
};
__device__ __forceinline__ Blk grid_blk() { return Blk{(int64_t)blockIdx.x, (int64_t)gridDim.x}; }

// Streamed stores: data that the next kernels read only after gigabytes of
// other traffic (corner records, gather records, the new cell state) are
// written with the nontemporal hint, so they do not push reused data (node
// aggregates, node positions) out of the caches.
__device__ __forceinline__ void store_stream(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(double2 *p, double2 v) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<d2 *>(p));
}

// Append `val` to `list` where `want`, one counter atomic per block of 256
// threads; every thread of the block calls it the same number of times.
// sh: 5 words of LDS.  Slots at or beyond `cap` (the list's length) are
// counted but not written.
__device__ __forceinline__ void block_append(int32_t *__restrict__ list, unsigned *__restrict__ counter, bool want,
                                             int32_t val, unsigned cap, unsigned *sh) {
    const int lane = (int)__lane_id(), w = (int)(threadIdx.x >> 6);
    const unsigned long long m = __ballot(want);
    if (lane == 0) sh[w] = (unsigned)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            const unsigned t = sh[i];
            sh[i] = tot;
            tot += t;
        }
        sh[4] = tot ? atomicAdd(counter, tot) : 0u;
    }
    __syncthreads();
    const unsigned slot = sh[4] + sh[w] + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
    if (want && slot < cap) list[slot] = val;
    __syncthreads();
}

// Append `val` to `list` where `want`, one counter atomic per wave: the
// lowest active lane reserves the wave's slots, each lane takes the slot of
// its rank among the wanting lanes.  Callable with a partial wave active.
// Slots at or beyond `cap` are counted but not written.
__device__ __forceinline__ void wave_append(int32_t *__restrict__ list, unsigned *__restrict__ counter, bool want,
                                            int32_t val, unsigned cap) {
    const unsigned long long act = __ballot(1);
    const unsigned long long m = __ballot(want);
    if (!m) return;
    const int lane = (int)__lane_id();
    const int leader = __ffsll((unsigned long long)act) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned)__popcll(m));
    base = __shfl(base, leader, 64);
    const unsigned slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
    if (want && slot < cap) list[slot] = val;
}

// Walk the items of a work list (see WorkList); f(entity) for each entity.
template <class F>
__device__ __forceinline__ void walk_items(const WorkList &w, const Blk b, F f) {
    const int64_t nslot = b.n >> 3;
    const int64_t per = (w.n_items + 7) >> 3;
    const int64_t i0 = (b.id & 7) * per;
    const int64_t i1 = i0 + per < w.n_items ? i0 + per : w.n_items;
    for (int64_t i = i0 + (b.id >> 3); i < i1; i += nslot) {
        const int64_t s0 = w.start[i];
        const int n = w.len[i];
        for (int j = threadIdx.x; j < n; j += blockDim.x) f(s0 + j);
    }
}

// One block per item (grid >= 8 * ceil(n_items / 8)) and items no longer
// than a block: the same XCD grouping without a loop around the body, which
// keeps the body's register allocation as low as a plain launch's.
template <class F>
__device__ __forceinline__ void one_item(const WorkList &w, const Blk b, F f) {
    const int64_t per = (w.n_items + 7) >> 3;
    const int64_t slot = b.id >> 3;
    const int64_t i = (b.id & 7) * per + slot;
    if (slot >= per || i >= w.n_items) return;
    if ((int)threadIdx.x < w.len[i]) f(w.start[i] + threadIdx.x);
}

template <bool LOOP, class F>
__device__ __forceinline__ void for_items(const WorkList &w, const Blk b, F f) {
    if (LOOP)
        walk_items(w, b, f);
    else
        one_item(w, b, f);
}

__device__ __forceinline__ double mesh_dt(const double *dtm, const int32_t *mesh_id, int64_t i) {
    return dtm[mesh_id ? mesh_id[i] : 0];
}

// ------------------------------------------------------- gather record
// Per cell, one 128-byte record {W = (tau, v, B stored comps), centroid}
// read by the node-aggregate gather (one cache line per neighbour instead
// of one per scalar array).
template <int D>
__device__ __forceinline__ void pack_cell(const StepArgs &a, const int64_t c) {
    using Dm = Dims<D>;
    const int64_t nc = a.nc, nn = a.nn;
    double s[D] = {};
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        int64_t p = a.c2n[c * (D + 1) + k];
#pragma unroll
        for (int i = 0; i < D; ++i) s[i] += a.x[i * nn + p];
    }
    double r[Dm::GR];
    r[0] = a.tau[c];
    double k2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        r[1 + i] = a.v[i * nc + c];
        k2 += r[1 + i] * r[1 + i];
    }
#pragma unroll
    for (int q = 0; q < Dm::NB; ++q) r[1 + D + q] = a.B[q * nc + c];
#pragma unroll
    for (int i = 0; i < D; ++i) r[Dm::NW + i] = s[i] * (1.0 / (D + 1));
#pragma unroll
    for (int q = Dm::NW + D; q < Dm::GR; ++q) r[q] = 0.0;
    if (a.eos) r[Dm::G_EPS] = a.e[c] - 0.5 * k2;
    double2 *o = reinterpret_cast<double2 *>(a.xc + c * Dm::GR);
#pragma unroll
    for (int q = 0; q < Dm::GR / 2; ++q) o[q] = make_double2(r[2 * q], r[2 * q + 1]);
}

template <int D, bool LOOP>
__global__ __launch_bounds__(256) void k_pack(StepArgs a, WorkList w) {
    for_items<LOOP>(w, grid_blk(), [&](int64_t c) { pack_cell<D>(a, c); });
}

// ------------------------------------------------ node aggregates (R8)
// For node p and every cell j around it, with y = x_j - x_p (centroid
// relative to the node): n, sum y, sum y y^T, sum W_j, sum y W_j^T, and the
// min / max of rho_j = 1 / tau_j.  A cell c then assembles its
// least-squares normal equations over all cells sharing a node with it
// (one visit per shared node) from the aggregates of its own nodes.
// Cooperative gather: AGG_G lanes per node, lane l holding values
// (2l, 2l+1) of each cell's gather record, so one wave-wide 16-byte load
// brings whole records (8 cache lines for 8 nodes) instead of one line per
// lane.  Each lane keeps, over the node's cells in CSR order, the sums of
// its two values and of their products with y; y reaches every lane of the
// group by shuffles from the lanes holding the centroid.  The products and
// the summation order are the per-node loop's, so the sums are bitwise
// those of one thread per node.
constexpr int AGG_G = 8;

template <int D>
__device__ __forceinline__ void node_agg_group(const StepArgs &a, const int64_t p, const int l,
                                               double *__restrict__ o) {
    using Dm = Dims<D>;
    constexpr int NW = Dm::NW;
    const int64_t nn = a.nn;
    const int v0 = 2 * l, v1 = 2 * l + 1;   // record values held by this lane
    const bool has = v0 < Dm::GR;           // 2D records have 5 pairs
    double xp[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xp[i] = a.x[i * nn + p];
    // centroid values become y = x_c - x_p
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        s0 = v0 == NW + i ? xp[i] : s0;
        s1 = v1 == NW + i ? xp[i] : s1;
    }
    double n = 0.0, Sa = 0.0, Sb = 0.0, Sya[D] = {}, Syb[D] = {};
    double tmin = __builtin_huge_val(), tmax = -__builtin_huge_val();
    double lo0 = __builtin_huge_val(), hi0 = -__builtin_huge_val();  // W bounds (limiter)
    double lo1 = lo0, hi1 = hi0;
    const double2 *rec = reinterpret_cast<const double2 *>(a.xc);
    const int32_t q0 = a.n2c_off[p], q1 = a.n2c_off[p + 1];
    // corners in chunks of AGG_G: lane l reads the cell of corner qb + l
    // (the next chunk's while this one is summed), then all AGG_G record
    // loads are issued before the sums, which run in CSR order
    int jl = q0 + l < q1 ? a.n2c[q0 + l] / (D + 1) : 0;
    for (int32_t qb = q0; qb < q1; qb += AGG_G) {
        const int32_t qn = qb + AGG_G + l;
        const int jn = qn < q1 ? a.n2c[qn] / (D + 1) : 0;
        double2 t[AGG_G];
#pragma unroll
        for (int m = 0; m < AGG_G; ++m) {
            const int jm = __shfl(jl, m, AGG_G);
            t[m] = (has && qb + m < q1) ? rec[(int64_t)jm * (Dm::GR / 2) + l] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int m = 0; m < AGG_G; ++m) {
            if (qb + m >= q1) break;
            const double va = t[m].x - s0, vb = t[m].y - s1;
            double y[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int v = NW + i;
                y[i] = __shfl((v & 1) ? vb : va, v >> 1, AGG_G);
            }
            n += 1.0;
            Sa += va;
            Sb += vb;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                Sya[i] += y[i] * va;
                Syb[i] += y[i] * vb;
            }
            tmin = fmin(tmin, va);  // tau of the cell in lane 0
            tmax = fmax(tmax, va);
            lo0 = fmin(lo0, va);
            hi0 = fmax(hi0, va);
            lo1 = fmin(lo1, vb);
            hi1 = fmax(hi1, vb);
        }
        jl = jn;
    }
    // rho = 1/tau: a correctly rounded reciprocal is monotone on tau > 0, so
    // these equal the min / max of the cells' 1/tau bitwise
    const double rmin = 1.0 / tmax, rmax = 1.0 / tmin;
    // this lane's share of the aggregate record
    auto put = [&](int v, double S, const double (&Sy)[D]) {
        if (v < NW) {
            o[Dm::O_SW + v] = S;
#pragma unroll
            for (int i = 0; i < D; ++i) o[Dm::O_SYW + v * D + i] = Sy[i];
        } else if (v < NW + D) {
            const int k = v - NW;
            o[Dm::O_SY + k] = S;
#pragma unroll
            for (int i = 0; i < D; ++i)
                if (i <= k) o[Dm::O_SYY + midx<D>(i, k)] = Sy[i];
        } else if (v == Dm::G_EPS && a.eos) {
            o[Dm::O_SE] = S;
#pragma unroll
            for (int i = 0; i < D; ++i) o[Dm::O_SYE + i] = Sy[i];
        }
    };
    put(v0, Sa, Sya);
    put(v1, Sb, Syb);
    if (a.limited) {
        if (v0 < NW) {
            o[Dm::O_WMIN + v0] = lo0;
            o[Dm::O_WMAX + v0] = hi0;
        }
        if (v1 < NW) {
            o[Dm::O_WMIN + v1] = lo1;
            o[Dm::O_WMAX + v1] = hi1;
        }
    }
    if (l == 0) {
        o[0] = n;
        o[Dm::O_RMM] = rmin;
        o[Dm::O_RMM + 1] = rmax;
        if (a.eos && Dm::NA_SG > Dm::O_SYE + D) o[Dm::NA_SG - 1] = 0.0;  // pad to a whole pair
    }
}

// LDS of the aggregate stage: one record of NA + 1 doubles per node group
template <int D>
constexpr int agg_lds_doubles() {
    return (256 / AGG_G) * (Dims<D>::NA + 1);
}

template <int D, bool LOOP>
__device__ __forceinline__ void node_agg_body(const StepArgs &a, const WorkList &w, const Blk bk, double *sh_all) {
    using Dm = Dims<D>;
    const int l = threadIdx.x & (AGG_G - 1);
    const int g = threadIdx.x / AGG_G;
    const int per_pass = blockDim.x / AGG_G;
    const int64_t nn = a.nn;
    double *sh = sh_all + g * (Dm::NA + 1);
    // items as in walk_items; every thread of the block runs the same passes
    const int64_t nslot = bk.n >> 3;
    const int64_t per = (w.n_items + 7) >> 3;
    const int64_t i0 = (bk.id & 7) * per;
    const int64_t i1 = i0 + per < w.n_items ? i0 + per : w.n_items;
    for (int64_t it = i0 + (bk.id >> 3); it < i1; it += nslot) {
        const int64_t s0 = w.start[it];
        const int len = w.len[it];
        for (int base = 0; base < len; base += per_pass) {
            const bool act = base + g < len;
            const int64_t p = s0 + base + g;
            if (act) node_agg_group<D>(a, p, l, sh);
            __syncthreads();
            if (act) {
                double2 *b = reinterpret_cast<double2 *>(a.agg) + p;
                const int np = (a.limited ? Dm::NA : (a.eos ? Dm::NA_SG : Dm::NA_BASE)) / 2;
                for (int j = l; j < np; j += AGG_G)
                    b[(int64_t)j * nn] = make_double2(sh[2 * j], sh[2 * j + 1]);
            }
            __syncthreads();
        }
        if (!LOOP) break;
    }
}

template <int D, bool LOOP>
__global__ __launch_bounds__(256) void k_node_agg(StepArgs a, WorkList w) {
    __shared__ double sh[agg_lds_doubles<D>()];
    node_agg_body<D, LOOP>(a, w, grid_blk(), sh);
}

// ---------------------------------------------------------- helpers
template <int D>
__device__ __forceinline__ void load_B6(const double *__restrict__ B, int64_t nc, int64_t c, double b[6]) {
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

template <int D>
__device__ __forceinline__ void store_B6(double *__restrict__ B, int64_t nc, int64_t c, const double b[6]) {
    if (D == 3) {
#pragma unroll
        for (int s = 0; s < 6; ++s) store_stream(&B[s * nc + c], b[s]);
    } else {
        store_stream(&B[c], b[0]);
        store_stream(&B[nc + c], b[1]);
        store_stream(&B[2 * nc + c], b[3]);
    }
}

// 6-vector slot of stored B component s (W index 1 + D + s)
template <int D>
__device__ __forceinline__ constexpr int bslot(int s) {
    return D == 3 ? s : (s == 2 ? 3 : s);
}

// ------------------------------------------ predictor + corner records
// Reconstruction (R8), ADER midpoint predictor (Section 3.4, reading R7),
// corner stress and impedance (R5), corner matrix M_cp (eq. Mcp, R4) and
// r_cp = M_cp v*_cp - T*_cp C_cp (eq. nodal_solver^n).  SG: the stiffened
// gas (R31) also reconstructs eps = e - |v|^2 / 2, advances it with
// d eps/dt = tau T : grad v and carries it through div T.
// STAGE: the corner records go to LDS, record k at lrec + k * lstride (NMS +
// D values), for the block to copy out (k_predict_staged).
// TILE (with STAGE): the node positions and aggregates come from the block's
// node tile in LDS (tile_pairs<D>() pairs per node at ta, the node of corner
// k at place (loc >> 8k) & 255), which the record stage then overwrites:
// every thread of the block calls this, and the block meets at a barrier
// once the tile is read.
template <int D>
struct TileRef {   // one node of a node tile, read like AggRef
    const double2 *b;
    __device__ __forceinline__ TileRef(const double2 *ta, int l) : b(ta + l * tile_pairs<D>()) {}
    __device__ __forceinline__ double operator[](int j) const {
        const double2 t = b[j >> 1];
        return (j & 1) ? t.y : t.x;
    }
    __device__ __forceinline__ double pos(int i) const { return (*this)[2 * ((Dims<D>::O_RMM + 1) / 2) + i]; }
};
// A cell's own inputs to the predictor, loaded by the tiled block before
// its node tile so that the two loads' latencies overlap.
template <int D>
struct PredIn {
    double tau, b[6], v[D], rho0, mu, K, dt;
    int level;
    __device__ __forceinline__ void load(const StepArgs &a, int64_t c) {
        tau = a.tau[c];
        load_B6<D>(a.B, a.nc, c, b);
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = a.v[i * a.nc + c];
        rho0 = a.rho0[c];
        mu = a.mu[c];
        K = a.K[c];
        dt = mesh_dt(a.dt, a.cell_mesh, c);
        level = a.mask[c];
    }
};
template <int D, bool LIM, bool FAM, bool SG, bool STAGE = false, bool TILE = false>
__device__ __forceinline__ void predict_cell(const StepArgs &a, const int64_t c, double *lrec = nullptr,
                                             const int lstride = 0, const double2 *ta = nullptr,
                                             const uint32_t loc = 0, const PredIn<D> *pin = nullptr) {
    static_assert((STAGE || !TILE) && !(TILE && SG), "node tiles: staged records, base aggregates");
    using Dm = Dims<D>;
    constexpr int NV = D + 1;
    const int64_t nc = a.nc, nn = a.nn;
    double X[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        if (TILE) {
            const TileRef<D> tr(ta, (loc >> (8 * k)) & 255);
#pragma unroll
            for (int i = 0; i < D; ++i) X[k][i] = tr.pos(i);
        } else {
            const int64_t p = a.c2n[c * NV + k];
#pragma unroll
            for (int i = 0; i < D; ++i) X[k][i] = a.x[i * nn + p];
        }
    }
    if (STAGE && !TILE) {
        // the node positions wait in this thread's record slots (filled
        // with the records only after the assembly loop) for that loop to
        // read them back: LDS reads instead of gathers from x
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int i = 0; i < D; ++i) lrec[k * lstride + i] = X[k][i];
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
    // corner offsets from the centroid
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) X[k][i] -= xc[i];

    PredIn<D> q;
    if (TILE)
        q = *pin;
    else
        q.load(a, c);
    const double tau = q.tau;
    double b[6];
#pragma unroll
    for (int s6 = 0; s6 < 6; ++s6) b[s6] = q.b[s6];
    const double rho0 = q.rho0, mu = q.mu, K = q.K;
    const int level = q.level;   // cascade level: 0 unlimited, 1 limited, 2 first order
    const bool p1 = level < 2;

    // W0 = W_c + (dt/2) dW/dt at the centroid; corner value W0 + grad W . delta
    double W0[Dm::NW];
    W0[0] = tau;
#pragma unroll
    for (int i = 0; i < D; ++i) W0[1 + i] = q.v[i];
#pragma unroll
    for (int q = 0; q < Dm::NB; ++q) W0[1 + D + q] = b[bslot<D>(q)];
    double grad[Dm::NW][D];
#pragma unroll
    for (int w = 0; w < Dm::NW; ++w)
#pragma unroll
        for (int i = 0; i < D; ++i) grad[w][i] = 0.0;
    // stiffened gas: eps at the centroid (advanced by dt/2 below) and its slope
    double eps0 = 0.0, geps[D] = {};
    if (SG) {
        double k2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) k2 += W0[1 + i] * W0[1 + i];
        eps0 = a.e[c] - 0.5 * k2;
    }
    double eps_mid = eps0;

    // ---- least-squares normal equations from the node aggregates (R8)
    double A[Dm::NMS] = {};
    double rhs[Dm::NW][D] = {};
    double rhs_e[D] = {};
    double visits = 0.0;  // neighbour visits: sum over nodes of (n - 1)
    // the sums of one node's aggregates (ag: AggRef or TileRef) with u =
    // the centroid minus the node's position
    auto add_node = [&](const auto &ag, const double (&u)[D]) {
        const double n = ag[0];
        visits += n - 1.0;
        double Sy[D];
#pragma unroll
        for (int i = 0; i < D; ++i) Sy[i] = ag[Dm::O_SY + i];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = i; j < D; ++j)
                A[midx<D>(i, j)] += ag[Dm::O_SYY + midx<D>(i, j)] - u[i] * Sy[j] - Sy[i] * u[j] + n * u[i] * u[j];
#pragma unroll
        for (int w = 0; w < Dm::NW; ++w) {
            const double sw = ag[Dm::O_SW + w];
#pragma unroll
            for (int j = 0; j < D; ++j)
                rhs[w][j] += ag[Dm::O_SYW + w * D + j] - u[j] * sw - Sy[j] * W0[w] + n * u[j] * W0[w];
        }
        if (SG) {
            const double se = ag[Dm::O_SE];
#pragma unroll
            for (int j = 0; j < D; ++j)
                rhs_e[j] += ag[Dm::O_SYE + j] - u[j] * se - Sy[j] * eps0 + n * u[j] * eps0;
        }
    };
    if (p1) {
#pragma unroll 1
        for (int k = 0; k < NV; ++k) {
            double u[D];
            if (TILE) {
                const TileRef<D> tr(ta, (loc >> (8 * k)) & 255);
#pragma unroll
                for (int i = 0; i < D; ++i) u[i] = xc[i] - tr.pos(i);
                add_node(tr, u);
            } else {
                const int64_t p = a.c2n[c * NV + k];
#pragma unroll
                for (int i = 0; i < D; ++i) u[i] = xc[i] - (STAGE ? lrec[k * lstride + i] : a.x[i * nn + p]);
                add_node(AggRef(a.agg, nn, p), u);
            }
        }
    }
    // the node tile has been read: its LDS becomes the block's record stage.
    // The other variants meet a no-op wave barrier here instead, so that
    // every variant keeps the sums and the solve apart in the same way and
    // the compiler forms the same fused multiply-adds (bitwise the same
    // records whatever the schedule)
    if (TILE)
        __syncthreads();
    else
        __builtin_amdgcn_wave_barrier();
    if (p1) {
        double inv[Dm::NMS];
        double det, tr = 0.0;
        if (D == 3)
            det = sym_inv3(A, inv);
        else
            det = sym_inv2(A, inv);
#pragma unroll
        for (int i = 0; i < D; ++i) tr += A[midx<D>(i, i)];
        const double scl = tr / D;
        const double scale = D == 3 ? scl * scl * scl : scl * scl;
        const bool ok = (visits >= D) && (tr > 0.0) && (det > 1e-12 * scale);
#pragma unroll
        for (int w = 0; w < Dm::NW; ++w)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) s += inv[midx<D>(i, j)] * rhs[w][j];
                grad[w][i] = ok ? s : 0.0;
            }
        if (SG) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) s += inv[midx<D>(i, j)] * rhs_e[j];
                geps[i] = ok ? s : 0.0;
            }
        }

        // ---- Barth-Jespersen limiter (the cascade's second scheme, Section
        // 3.5; reading R26): per scalar, bounds over {c} and its stencil from
        // the node aggregates, ratio at the vertices, slope scaled by phi
        if (LIM && level == 1) {
#pragma unroll
            for (int w = 0; w < Dm::NW; ++w) {
                double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const AggRef ag(a.agg, nn, a.c2n[c * NV + k]);
                    lo = fmin(lo, ag[Dm::O_WMIN + w]);
                    hi = fmax(hi, ag[Dm::O_WMAX + w]);
                }
                double phi = 1.0;
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    double Dk = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) Dk += grad[w][j] * X[k][j];
                    double r = 1.0;
                    if (Dk > 0.0)
                        r = fmin(1.0, (hi - W0[w]) / Dk);
                    else if (Dk < 0.0)
                        r = fmin(1.0, (lo - W0[w]) / Dk);
                    phi = fmin(phi, r);
                }
#pragma unroll
                for (int j = 0; j < D; ++j) grad[w][j] *= phi;
            }
        }

        // ---- time derivatives at the cell centre (reading R7)
        double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) G[i][j] = grad[1 + i][j];
        auto gB = [&](int s6, int j) -> double {  // d b_s6 / d x_j (6-vector order)
            if (D == 3) return grad[1 + D + s6][j];
            return s6 == 0 ? grad[1 + D][j] : (s6 == 1 ? grad[2 + D][j] : (s6 == 3 ? grad[3 + D][j] : 0.0));
        };
        double trG = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) trG += G[i][i];
        const double h = 0.5 * q.dt;
        const double B3[3][3] = {{b[0], b[3], b[4]}, {b[3], b[1], b[5]}, {b[4], b[5], b[2]}};
        // dB/dt = G B + B G^T, stored components only
#pragma unroll
        for (int q = 0; q < Dm::NB; ++q) {
            const int s6 = bslot<D>(q);
            const int i = s6 < 3 ? s6 : (s6 == 5 ? 1 : 0);
            const int j = s6 < 3 ? s6 : (s6 == 3 ? 1 : 2);
            double y = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) y += G[i][k] * B3[k][j] + B3[i][k] * G[j][k];
            W0[1 + D + q] += h * y;
        }
        // div T by the chain rule through T(tau, B) (and eps for the gas)
        if (SG) {
            double divT[D] = {}, Tc[6];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double db[6], dT[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) db[q] = gB(q, j);
                stress6_dir_sg(rho0, mu, a.shear_a, a.sg_gamma, a.sg_pinf, tau, b, eps0, grad[0][j], db, geps[j],
                               dT);
#pragma unroll
                for (int i = 0; i < D; ++i) divT[i] += dT[sidx(i, j)];
            }
#pragma unroll
            for (int i = 0; i < D; ++i) W0[1 + i] += h * tau * divT[i];
            // d eps / dt = tau T : G
            stress6_sg(rho0, mu, a.shear_a, a.sg_gamma, a.sg_pinf, tau, b, eps0, Tc);
            double TG = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) TG += Tc[sidx(i, j)] * G[i][j];
            eps_mid = eps0 + h * tau * TG;
        } else if (FAM) {
            // shear energy family: column j of grad T from the derivative of
            // T along (d tau / d x_j, d B / d x_j)
            double divT[D] = {};
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double db[6], dT[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) db[q] = gB(q, j);
                stress6_dir_family(rho0, mu, K, a.shear_a, tau, b, grad[0][j], db, dT);
#pragma unroll
                for (int i = 0; i < D; ++i) divT[i] += dT[sidx(i, j)];
            }
#pragma unroll
            for (int i = 0; i < D; ++i) W0[1 + i] += h * tau * divT[i];
        } else {
            const double J = rho0 * tau;
            const double rJ = 1.0 / J;
            const double lj = log(J);
            const double cJ = cbrt(J);
            const double J53 = cJ * rJ * rJ;          // J^{-5/3}
            const double J83 = J53 * rJ;              // J^{-8/3}
            const double mdpdJ = 0.5 * K * (1.0 + (1.0 - lj) * rJ * rJ);  // -dp/dJ
            const double trB3 = (b[0] + b[1] + b[2]) * (1.0 / 3.0);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double devB = B3[i][j] - (i == j ? trB3 : 0.0);
                    s1 += devB * grad[0][j];
                    s2 += gB(sidx(i, j), j);
                }
                const double dtr = gB(0, i) + gB(1, i) + gB(2, i);
                const double divT = rho0 * (mdpdJ * grad[0][i] - (5.0 / 3.0) * mu * J83 * s1) +
                                    mu * J53 * (s2 - dtr * (1.0 / 3.0));
                W0[1 + i] += h * tau * divT;
            }
        }
        W0[0] += h * tau * trG;
    }

    // S = sum_j C_j C_j^T / |C_j|; corner shape N_k = S - C_k C_k^T / |C_k|
    double S[Dm::NMS] = {};
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double r = 1.0 / g.cn[j];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int k = i; k < D; ++k) S[midx<D>(i, k)] += g.C[j][i] * g.C[j][k] * r;
    }

    // ---- corner records: predicted state, stress, impedance, M_cp, r_cp
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double Wk[Dm::NW];
#pragma unroll
        for (int w = 0; w < Dm::NW; ++w) {
            double s = W0[w];
#pragma unroll
            for (int j = 0; j < D; ++j) s += grad[w][j] * X[k][j];
            Wk[w] = s;
        }
        double bk[6];
        if (D == 3) {
#pragma unroll
            for (int q = 0; q < 6; ++q) bk[q] = Wk[1 + D + q];
        } else {
            bk[0] = Wk[1 + D];
            bk[1] = Wk[2 + D];
            bk[2] = 1.0;
            bk[3] = Wk[3 + D];
            bk[4] = 0.0;
            bk[5] = 0.0;
        }
        double T[6], z;
        if (SG) {
            double ek = eps_mid;
#pragma unroll
            for (int j = 0; j < D; ++j) ek += geps[j] * X[k][j];
            stress6_sg(rho0, mu, a.shear_a, a.sg_gamma, a.sg_pinf, Wk[0], bk, ek, T);
            z = sound_sg(rho0, mu, a.shear_a, a.sg_gamma, a.sg_pinf, Wk[0], bk, ek) / Wk[0];
        } else {
            if (FAM)
                stress6_family(rho0, mu, K, a.shear_a, Wk[0], bk, T);
            else
                stress6(rho0, mu, K, Wk[0], bk, T);
            z = impedance(rho0, mu, K, Wk[0]);
        }
        const double rk = 1.0 / g.cn[k];
        double M[Dm::NMS];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = i; j < D; ++j)
                M[midx<D>(i, j)] = z * (S[midx<D>(i, j)] - g.C[k][i] * g.C[k][j] * rk);
        double *o = STAGE ? lrec + k * lstride : a.corner + corner_slot<D>(c, k) * Dm::CW;
#pragma unroll
        for (int q = 0; q < Dm::NMS; ++q) o[q] = M[q];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += M[midx<D>(i, j)] * Wk[1 + j] - T[sidx(i, j)] * g.C[k][j];
            o[Dm::NMS + i] = s;
        }
    }
}

template <int D, bool LOOP, bool LIM, bool FAM, bool SG>
__device__ __forceinline__ void predict_body(const StepArgs &a, const WorkList &w, const Blk b) {
    for_items<LOOP>(w, b, [&](int64_t c) { predict_cell<D, LIM, FAM, SG>(a, c); });
}
template <int D, bool LOOP, bool LIM, bool FAM, bool SG>
__global__ __launch_bounds__(256) void k_predict(StepArgs a, WorkList w) {
    predict_body<D, LOOP, LIM, FAM, SG>(a, w, grid_blk());
}

// One block per item (the one_item mapping), corner records staged in LDS
// ([corner][cell][NMS + D], dynamic, NV * blockDim * (NMS + D) doubles):
// after a barrier the block copies them out in address order, so each wave
// store covers 512 consecutive bytes instead of 64 records 72 bytes apart.
// TILE: the block first loads its item's node tile into the same LDS (the
// aggregate pairs its cells' least-squares sums read and the positions of
// each of the item's distinct nodes, tile_pairs<D>() pairs per node), so
// that a node's values are fetched once per item instead of once per corner
// that uses it; threads past the item's end repeat its last cell and keep
// the records to themselves.  Same values as k_predict.
template <int D, bool LIM, bool FAM, bool SG, bool TILE = false>
__device__ __forceinline__ void predict_staged_body(const StepArgs &a, const WorkList &w, const Blk b, double *cs) {
    using Dm = Dims<D>;
    constexpr int NV = D + 1, RW = Dm::CW;
    static_assert(Dm::CW == Dm::NMS + D, "corner records hold M_cp and r_cp only");
    const int64_t per = (w.n_items + 7) >> 3;
    const int64_t slot = b.id >> 3;
    const int64_t it = (b.id & 7) * per + slot;
    if (slot >= per || it >= w.n_items) return;  // the whole block
    const int64_t s0 = w.start[it];
    const int len = w.len[it];
    const int bs = blockDim.x;
    if constexpr (TILE) {
        constexpr int NP = (Dm::O_RMM + 1) / 2, NT = tile_pairs<D>();
        const int o0 = w.tn_off[it], cnt = w.tn_off[it + 1] - o0;
        double2 *ta = reinterpret_cast<double2 *>(cs);
        const double2 *ag2 = reinterpret_cast<const double2 *>(a.agg);
        const int64_t nn = a.nn;
        const int64_t c = s0 + min((int)threadIdx.x, len - 1);
        const uint32_t loc = w.tloc[c];
        PredIn<D> pin;
        pin.load(a, c);
        // one node per thread, all of its loads in flight together;
        // consecutive threads on consecutive nodes of each aggregate plane
        for (int u = threadIdx.x; u < cnt; u += bs) {
            const int64_t p = w.tn[o0 + u];
            double2 v[NT];
#pragma unroll
            for (int j = 0; j < NP; ++j) v[j] = ag2[(int64_t)j * nn + p];
#pragma unroll
            for (int j = NP; j < NT; ++j) {
                const int i0 = 2 * (j - NP);
                v[j].x = a.x[i0 * nn + p];
                v[j].y = i0 + 1 < D ? a.x[(i0 + 1) * nn + p] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) ta[u * NT + j] = v[j];
        }
        __syncthreads();
        predict_cell<D, LIM, FAM, SG, true, true>(a, c, cs + threadIdx.x * RW, bs * RW, ta, loc, &pin);
    } else if ((int)threadIdx.x < len) {
        predict_cell<D, LIM, FAM, SG, true>(a, s0 + threadIdx.x, cs + threadIdx.x * RW, bs * RW);
    }
    __syncthreads();
    // the item's records of corner k are one run within a tile (two runs
    // if the item crosses a tile boundary); a single run that starts on a
    // 16-byte boundary and holds an even number of values goes out in
    // 16-byte stores
    const int tot = len * RW;
    const bool one_run = (int)(s0 & 255) + len <= 256 && (tot & 1) == 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double *run = a.corner + corner_slot<D>(s0, k) * RW;
        if (one_run && ((reinterpret_cast<uintptr_t>(run) | reinterpret_cast<uintptr_t>(cs + k * bs * RW)) & 15) == 0) {
            const double2 *src = reinterpret_cast<const double2 *>(cs + k * bs * RW);
            double2 *dst = reinterpret_cast<double2 *>(run);
            for (int r = threadIdx.x; r < tot / 2; r += bs) store_stream(&dst[r], src[r]);
        } else {
            for (int r = threadIdx.x; r < tot; r += bs) {
                const int ci = r / RW, j = r - ci * RW;
                store_stream(&a.corner[corner_slot<D>(s0 + ci, k) * RW + j], cs[k * bs * RW + r]);
            }
        }
    }
}
template <int D, bool LIM, bool FAM, bool SG, bool TILE = false>
__global__ __launch_bounds__(256) void k_predict_staged(StepArgs a, WorkList w) {
    extern __shared__ double cs[];
    predict_staged_body<D, LIM, FAM, SG, TILE>(a, w, grid_blk(), cs);
}

// x^{n+1} = x^n + dt v* (reading R13) and vhat^{n+1} = 2 v* - vhat^n (R9),
// as one fused multiply-add and one exact doubling.  The staged cell update
// applies the same two functions to the v* it gathers for its forces, which
// gives the node solve's bits without gathering x^{n+1} and vhat^{n+1}.
__device__ __forceinline__ double next_position(double x, double dt, double vs) { return __fma_rn(dt, vs, x); }
__device__ __forceinline__ double next_vhat(double vs, double vh) { return 2.0 * vs - vh; }

// ---------------------------------------------------------- node solve
// M_p v*_p = sum_c (M_cp v*_cp - T*_cp C_cp) (eq. nodal_solver^n, readings
// R14, R15); slip walls by Galerkin projection onto the allowed directions
// (Appendix B eq. sBC1, reading R22); boundary loads of the faces through
// the node (Appendix B, readings R28, R29).  Then x^{n+1} = x^n + dt v*_p
// and vhat^{n+1} = 2 v*_p - vhat^n (Section 3.4, reading R9).
template <int D, bool LD>
__device__ __forceinline__ void node_solve_finish(const StepArgs &a, const int64_t p, const bool any,
                                                  const double (&M)[Dims<D>::NMS], const double (&r)[D],
                                                  const int comp);

// Symmetric tensor from its components (11, 22, 33, 12, 13, 23); the
// leading D x D block.
template <int D>
__device__ __forceinline__ void sym6_unpack(const double *v, double (&T)[D][D]) {
    constexpr int row[6] = {0, 1, 2, 0, 0, 1}, col[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (row[q] < D && col[q] < D) T[row[q]][col[q]] = T[col[q]][row[q]] = v[q];
}

// M_p and the corner part of r_p, summed over the node's corners in CSR
// order by one thread; returns whether the node has corners
template <int D>
__device__ __forceinline__ bool node_gather(const StepArgs &a, const int64_t p, double (&M)[Dims<D>::NMS],
                                            double (&r)[D]) {
    using Dm = Dims<D>;
#pragma unroll
    for (int s = 0; s < Dm::NMS; ++s) M[s] = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) r[i] = 0.0;
    const int32_t q0 = a.n2c_off[p], q1 = a.n2c_off[p + 1];
    for (int32_t q = q0; q < q1; ++q) {
        const double *rec = a.corner + corner_slot_of<D>(a.n2c[q]) * Dm::CW;
#pragma unroll
        for (int s = 0; s < Dm::NMS; ++s) M[s] += rec[s];
#pragma unroll
        for (int i = 0; i < D; ++i) r[i] += rec[Dm::NMS + i];
    }
    return q1 > q0;
}

// Cooperative corner gather (as for the node aggregates): lane l of a group
// of AGG_G sums values 2l and 2l + 1 of the node's corner records in CSR
// order, each read with one 16-byte load, so a wave-wide load brings whole
// records (the last pair's second value lies past the record: the next
// record's first, or the two doubles of pad after the corner array); the
// sums then meet in every lane of the group, which all run the solve.
// Lane i < D writes component i.
template <int D, bool LD>
__device__ __forceinline__ void node_solve_group(const StepArgs &a, const int64_t p, const int l) {
    using Dm = Dims<D>;
    constexpr int CW = Dm::CW;           // values per corner record
    constexpr int NPAIR = (CW + 1) / 2;  // 16-byte loads per record
    static_assert(NPAIR <= AGG_G, "a lane sums one pair of a record");
    const bool has = l < NPAIR;
    double Sa = 0.0, Sb = 0.0;
    const int32_t q0 = a.n2c_off[p], q1 = a.n2c_off[p + 1];
    for (int32_t qb = q0; qb < q1; qb += AGG_G) {
        const int32_t ql = qb + l;
        const int kl = ql < q1 ? a.n2c[ql] : 0;
        double2 t[AGG_G];
#pragma unroll
        for (int m = 0; m < AGG_G; ++m) {
            const int km = __shfl(kl, m, AGG_G);
            const double *rec = a.corner + corner_slot_of<D>(km) * CW;
            const bool in = qb + m < q1;
            t[m] = (has && in) ? *reinterpret_cast<const double2 *>(rec + 2 * l) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int m = 0; m < AGG_G; ++m) {
            if (qb + m >= q1) break;
            Sa += t[m].x;
            Sb += t[m].y;
        }
    }
    double v[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) v[j] = __shfl((j & 1) ? Sb : Sa, j >> 1, AGG_G);
    double M[Dm::NMS], r[D];
#pragma unroll
    for (int s = 0; s < Dm::NMS; ++s) M[s] = v[s];
#pragma unroll
    for (int i = 0; i < D; ++i) r[i] = v[Dm::NMS + i];
    node_solve_finish<D, LD>(a, p, q1 > q0, M, r, l);
}

// Node velocity from the summed corner matrices and right-hand sides, with
// na allowed directions P (na == D: free).  LD: the mesh has boundary loads
// (a separate instantiation keeps the plain solve's register budget).
template <int D, bool LD>
__device__ __forceinline__ void node_velocity(const StepArgs &a, const int64_t p, const bool any,
                                              const double (&M)[Dims<D>::NMS], const double (&r)[D], const int na,
                                              const double *P, double (&vs)[D]) {
    using Dm = Dims<D>;
    const int64_t nn = a.nn;
#pragma unroll
    for (int i = 0; i < D; ++i) vs[i] = 0.0;
    double rl[D], dl[D] = {}, vn = 0.0;
    bool has_v = false;
#pragma unroll
    for (int i = 0; i < D; ++i) rl[i] = r[i];
    if (LD) {
        // face vector (|f|/d) n_f = -C_k of the face opposite node k, from
        // the positions at t^n: a traction adds T^BC (|f|/d) n_f to the
        // right-hand side (R28); a normal velocity adds to d_p and to the
        // target sum_f v_n |f|/d (R29)
        const int32_t l0 = a.ld_off[p], l1 = a.ld_off[p + 1];
        for (int32_t q = l0; q < l1; ++q) {
            const int64_t c = a.ld_cell[q];
            const int code = a.ld_fk[q], k = code & 3;
            double X[D + 1][D];
#pragma unroll
            for (int j = 0; j <= D; ++j) {
                const int64_t pj = a.c2n[c * (D + 1) + j];
#pragma unroll
                for (int i = 0; i < D; ++i) X[j][i] = a.x[i * nn + pj];
            }
            Geo<D> g;
            geom<D>(X, g);
            double Ck[D] = {}, ck = 0.0;  // row k by selects (no indexed registers)
#pragma unroll
            for (int j = 0; j <= D; ++j) {
#pragma unroll
                for (int i = 0; i < D; ++i) Ck[i] = j == k ? g.C[j][i] : Ck[i];
                ck = j == k ? g.cn[j] : ck;
            }
            const double *val = a.ld_val + 6 * (int64_t)q;
            if ((code >> 2) == 1) {
                double T[D][D];
                sym6_unpack<D>(val, T);
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) rl[i] -= T[i][j] * Ck[j];
            } else {
                has_v = true;
#pragma unroll
                for (int i = 0; i < D; ++i) dl[i] -= Ck[i];
                vn += val[0] * ck;
            }
        }
    }
    if (any && na == D) {
        double inv[Dm::NMS];
        if (D == 3)
            sym_inv3(M, inv);
        else
            sym_inv2(M, inv);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += inv[midx<D>(i, j)] * rl[j];
            vs[i] = s;
        }
        if (has_v) {
            // v = M^-1 (r - pi d) with pi such that v . d = sum_f v_n |f|/d
            double z[D], yd = 0.0, zd = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) s += inv[midx<D>(i, j)] * dl[j];
                z[i] = s;
                yd += vs[i] * dl[i];
                zd += s * dl[i];
            }
            const double pi = (yd - vn) / zd;
#pragma unroll
            for (int i = 0; i < D; ++i) vs[i] -= pi * z[i];
        }
    } else if (any && na > 0) {
        // P: D x na orthonormal columns, P[i][t] = P[i*D + t]
        double Mf[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Mf[i][j] = M[midx<D>(i, j)];
        double Ar[D][D], br[D];
#pragma unroll
        for (int s = 0; s < D; ++s) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) t += P[i * D + s] * rl[i];
            br[s] = t;
#pragma unroll
            for (int u = 0; u < D; ++u) {
                double m = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) m += P[i * D + s] * Mf[i][j] * P[j * D + u];
                Ar[s][u] = m;
            }
        }
        double al[D] = {};
        const double det = na == 1 ? Ar[0][0] : Ar[0][0] * Ar[1][1] - Ar[0][1] * Ar[1][0];
        auto solve = [&](const double (&b)[D], double (&x)[D]) {
            if (na == 1) {
                x[0] = b[0] / Ar[0][0];
            } else {  // na == 2 < D == 3
                x[0] = (Ar[1][1] * b[0] - Ar[0][1] * b[1]) / det;
                x[1] = (Ar[0][0] * b[1] - Ar[1][0] * b[0]) / det;
            }
        };
        solve(br, al);
        if (LD && has_v) {
            // the velocity load within the allowed directions: a = y - pi z,
            // z = (P^T M P)^-1 P^T d, a . P^T d = sum_f v_n |f|/d; dropped
            // where P^T d vanishes (walls and symmetry come first)
            double e[D] = {}, z[D] = {}, ee = 0.0, dd = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                double u = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) u += P[i * D + t] * dl[i];
                e[t] = t < na ? u : 0.0;
                ee += e[t] * e[t];
                dd += dl[t] * dl[t];
            }
            if (ee > 1e-20 * dd) {
                solve(e, z);
                double ye = 0.0, ze = 0.0;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    ye += t < na ? al[t] * e[t] : 0.0;
                    ze += t < na ? z[t] * e[t] : 0.0;
                }
                const double pi = (ye - vn) / ze;
#pragma unroll
                for (int t = 0; t < D; ++t) al[t] -= t < na ? pi * z[t] : 0.0;
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) s += (t < na) ? P[i * D + t] * al[t] : 0.0;
            vs[i] = s;
        }
    }
}

// v* of node p under its current constraints, then x^{n+1} and vhat^{n+1};
// comp < 0 writes every component, otherwise only component comp (if < D)
template <int D, bool LD>
__device__ __forceinline__ void node_solve_finish(const StepArgs &a, const int64_t p, const bool any,
                                                  const double (&M)[Dims<D>::NMS], const double (&r)[D],
                                                  const int comp) {
    const int64_t nn = a.nn;
    double vs[D];
    node_velocity<D, LD>(a, p, any, M, r, a.nallow[p], a.allow + p * D * D, vs);
    const double dt = mesh_dt(a.dt, a.node_mesh, p);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (comp >= 0 && comp != i) continue;
        a.vstar[i * nn + p] = vs[i];
        a.x1[i * nn + p] = next_position(a.x[i * nn + p], dt, vs[i]);
        a.vhat1[i * nn + p] = next_vhat(vs[i], a.vhat[i * nn + p]);
    }
}

template <int D, bool LOOP, bool LD>
__device__ __forceinline__ void node_solve_body(const StepArgs &a, const WorkList &w, const Blk b) {
    const int l = threadIdx.x & (AGG_G - 1);
    const int g = threadIdx.x / AGG_G;
    const int per_pass = blockDim.x / AGG_G;
    const int64_t nslot = b.n >> 3;
    const int64_t per = (w.n_items + 7) >> 3;
    const int64_t i0 = (b.id & 7) * per;
    const int64_t i1 = i0 + per < w.n_items ? i0 + per : w.n_items;
    for (int64_t it = i0 + (b.id >> 3); it < i1; it += nslot) {
        const int64_t s0 = w.start[it];
        const int len = w.len[it];
        for (int base = g; base < len; base += per_pass) node_solve_group<D, LD>(a, s0 + base, l);
        if (!LOOP) break;
    }
}
template <int D, bool LOOP, bool LD>
__global__ __launch_bounds__(256) void k_node_solve(StepArgs a, WorkList w) {
    node_solve_body<D, LOOP, LD>(a, w, grid_blk());
}


// ------------------------------------------------------------ contact
// Candidate i of a rigid-plane contact takes constraint set state[i]: 0 its
// own walls, 1 its own walls and the plane (Section 3.8, reading R30).
__global__ void k_contact_apply(ContactArgs k, int dd) {
    const int64_t i = gtid();
    if (i >= k.n) return;
    const int s = k.state[i] ? 1 : 0;
    const int64_t p = k.node[i];
    k.nallow[p] = k.nal[s][i];
    for (int j = 0; j < dd; ++j) k.allow[p * dd + j] = k.alw[s][i * dd + j];
}

// After a trial step: for a free candidate the fraction of the step at
// which it reaches the plane, s = g0 / (g0 - g1) with the gaps
// g = (x - x_T) . n at t^n and at the trial's t^{n+1} (0 if g0 <= 0; 2 when
// it stays above the plane); for a candidate in contact the normal
// component of its free velocity (its own walls only, same corner values).
template <int D, bool LD>
__global__ __launch_bounds__(256) void k_contact_eval(StepArgs a, ContactArgs k) {
    const int64_t i = gtid();
    if (i >= k.n) return;
    const int64_t p = k.node[i];
    const int64_t nn = a.nn;
    if (k.state[i]) {
        double M[Dims<D>::NMS], r[D], vs[D];
        const bool any = node_gather<D>(a, p, M, r);
        node_velocity<D, LD>(a, p, any, M, r, k.nal[0][i], k.alw[0] + i * D * D, vs);
        double vn = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) vn += vs[j] * k.nrm[j];
        k.out_s[i] = 2.0;
        k.out_vn[i] = vn;
    } else {
        double g0 = 0.0, g1 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            g0 += (a.x[j * nn + p] - k.xT[j]) * k.nrm[j];
            g1 += (a.x1[j * nn + p] - k.xT[j]) * k.nrm[j];
        }
        k.out_s[i] = g1 < 0.0 ? (g0 > 0.0 ? g0 / (g0 - g1) : 0.0) : 2.0;
        k.out_vn[i] = 0.0;
    }
}

// -------------------------------------------------------- cell update
// Subcell forces f_cp = M_cp v*_p - r_cp (eq. subforce^n), momentum and
// total energy (eqs. v_c^n, e_c^n), tau = V(x^{n+1}) / m (reading R12), B by
// Crank-Nicolson (P1) or Euler (P0) (eqs. CN_B, firstB; R10, R11), then
// detection (eqs. PAD, RDMP; R16, R17) and the per-cell time-step bounds.
// SG: the stiffened gas (R31) -- eps in the gather record, p + p_inf > 0 in
// the admissibility test, its sound speed in the time-step bound.
// STAGE: the gather record goes to LDS at lrec (16-byte aligned) for the
// block to copy out (k_update_staged).
// VS: the v* gathered for the forces waits in the thread's LDS slots vsl
// (NV * D doubles) and gives x^{n+1} and vhat^{n+1} with the node solve's
// own formulas instead of further gathers (the same bits).
template <int D, bool SG, bool STAGE = false, bool VS = STAGE>
__device__ __forceinline__ void update_cell(const StepArgs &a, const int64_t c, double *lrec = nullptr,
                                            double *vsl = nullptr) {
    if (STAGE && VS) vsl = lrec;
    using Dm = Dims<D>;
    constexpr int NV = D + 1;
    const int64_t nc = a.nc, nn = a.nn;
    const double m = a.mass[c];
    const double dt = mesh_dt(a.dt, a.cell_mesh, c);
    const double dtm = dt / m;
    // the cell's own values, loaded ahead of the force loop's gathers
    double v0[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v0[i] = a.v[i * nc + c];
    const double e0 = a.e[c];
    const int lev = a.mask[c];

    // ---- subcell forces and the compatible momentum / energy update
    double F[D] = {}, Wk = 0.0;
#pragma unroll 1
    for (int k = 0; k < NV; ++k) {
        const int64_t p = a.c2n[c * NV + k];
        double vs[D];
#pragma unroll
        for (int i = 0; i < D; ++i) vs[i] = a.vstar[i * nn + p];
        if (VS) {
            // kept in this thread's LDS slots (for the staged kernel its
            // record slots: the gather record goes there only at the end)
#pragma unroll
            for (int i = 0; i < D; ++i) vsl[k * D + i] = vs[i];
        }
        const double *rec = a.corner + corner_slot<D>(c, k) * Dm::CW;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double f = -rec[Dm::NMS + i];
#pragma unroll
            for (int j = 0; j < D; ++j) f += rec[midx<D>(i, j)] * vs[j];
            F[i] += f;
            Wk += f * vs[i];
        }
    }
    double v1[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        v1[i] = v0[i] + dtm * F[i];
        store_stream(&a.v1[i * nc + c], v1[i]);
    }
    const double e1 = e0 + dtm * Wk;
    store_stream(&a.e1[c], e1);

    // ---- geometry at t^n and t^{n+1}; velocity gradients
    const bool p1 = lev < 2;   // unlimited or limited second order
    double L0[D][D], L1[D][D];
    double tau1, Lc, xc1[D];
    {
        double X0[NV][D], X1[NV][D];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int64_t p = a.c2n[c * NV + k];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                X0[k][i] = a.x[i * nn + p];
                // the node solve's own x^n + dt v* (the node's mesh is the
                // cell's, so dt is the same value)
                X1[k][i] = VS ? next_position(X0[k][i], dt, vsl[k * D + i]) : a.x1[i * nn + p];
            }
        }
        Geo<D> g0, g1;
        geom<D>(X0, g0);
        geom<D>(X1, g1);
        tau1 = g1.V / m;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double sx = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) sx += X1[k][i];
            xc1[i] = sx * (1.0 / NV);
        }
        double S1 = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) S1 += g1.cn[k];
        Lc = 2.0 * g1.V / S1;
        // P1: L^n from vhat^n on x^n and L^{n+1} from vhat^{n+1} on x^{n+1};
        // P0: L* from v* on x^n (L0 only)
        const double *u0 = p1 ? a.vhat : a.vstar;
        const double r0 = 1.0 / g0.V, r1 = 1.0 / g1.V;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                L0[i][j] = 0.0;
                L1[i][j] = 0.0;
            }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int64_t p = a.c2n[c * NV + k];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double vsk = VS ? vsl[k * D + i] : 0.0;
                const double w0 = (VS && !p1) ? vsk : u0[i * nn + p];
                const double w1 = p1 ? (VS ? next_vhat(vsk, w0) : a.vhat1[i * nn + p]) : 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    L0[i][j] += w0 * g0.C[k][j];
                    L1[i][j] += w1 * g1.C[k][j];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                L0[i][j] *= r0;
                L1[i][j] *= r1;
            }
    }
    store_stream(&a.tau1[c], tau1);

    // ---- B: Crank-Nicolson (P1) or Euler (P0)
    double b[6], b1[6];
    load_B6<D>(a.B, nc, c, b);
    if (p1) {
        cn_update<D>(b, L0, L1, 0.5 * dt, b1);
    } else {
        double L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) L[i][j] = L0[i][j];
        const double B3[3][3] = {{b[0], b[3], b[4]}, {b[3], b[1], b[5]}, {b[4], b[5], b[2]}};
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int i = s < 3 ? s : (s == 5 ? 1 : 0);
            const int j = s < 3 ? s : (s == 3 ? 1 : 2);
            double y = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) y += L[i][k] * B3[k][j] + B3[i][k] * L[j][k];
            b1[s] = b[s] + dt * y;
        }
        if (D == 2) {
            b1[2] = 1.0;
            b1[4] = 0.0;
            b1[5] = 0.0;
        }
    }
    store_B6<D>(a.B1, nc, c, b1);

    // gather record of the candidate for the next step's reconstruction
    {
        double r[Dm::GR];
        r[0] = tau1;
#pragma unroll
        for (int i = 0; i < D; ++i) r[1 + i] = v1[i];
#pragma unroll
        for (int q = 0; q < Dm::NB; ++q) r[1 + D + q] = b1[bslot<D>(q)];
#pragma unroll
        for (int i = 0; i < D; ++i) r[Dm::NW + i] = xc1[i];
#pragma unroll
        for (int q = Dm::NW + D; q < Dm::GR; ++q) r[q] = 0.0;
        if (SG) {
            double kk = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) kk += v1[i] * v1[i];
            r[Dm::G_EPS] = e1 - 0.5 * kk;
        }
        double2 *o = reinterpret_cast<double2 *>(STAGE ? lrec : a.xc + c * Dm::GR);
#pragma unroll
        for (int q = 0; q < Dm::GR / 2; ++q) o[q] = make_double2(r[2 * q], r[2 * q + 1]);
    }

    // ---- detection (eqs. PAD, RDMP; R16, R17)
    bool fin = isfinite(tau1) && isfinite(e1);
#pragma unroll
    for (int i = 0; i < D; ++i) fin = fin && isfinite(v1[i]);
#pragma unroll
    for (int s = 0; s < 6; ++s) fin = fin && isfinite(b1[s]);
    double k2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) k2 += v1[i] * v1[i];
    const double eps = e1 - 0.5 * k2;
    bool pad_bad = !fin || !(tau1 > 0.0) || !(det6(b1) > 0.0) || (eps < -a.eps_tol * (fabs(e1) + 0.5 * k2));
    double p_sg = 0.0;
    if (SG) {
        p_sg = sg_pressure6(a.rho0[c], a.mu[c], a.shear_a, a.sg_gamma, a.sg_pinf, tau1, b1, eps);
        pad_bad = pad_bad || !(p_sg + a.sg_pinf > 0.0);
    }
    if (p1 && a.detect) {
        double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int64_t p = a.c2n[c * NV + k];
            const AggRef ag(a.agg, a.nn, p);
            lo = fmin(lo, ag[Dm::O_RMM]);
            hi = fmax(hi, ag[Dm::O_RMM + 1]);
        }
        const double rho1 = 1.0 / tau1;
        const double delta = fmax(a.delta0, a.delta1 * (hi - lo));
        const bool bad = pad_bad || rho1 < lo - delta || rho1 > hi + delta;
        wave_append(a.flist_out, a.fcount_out, bad, (int32_t)c, (unsigned)a.nc);
    }
    a.pstat[c] = (!p1 && pad_bad) ? 1 : 0;

    // ---- time-step bounds at t^{n+1} (eq. CFL2; R20, R21)
    const double ac = SG ? sqrt(tau1 * (a.sg_gamma * (p_sg + a.sg_pinf) + (4.0 / 3.0) * a.mu[c]))
                         : sound(a.rho0[c], a.mu[c], a.K[c], tau1);
    const double V0 = m * a.tau[c], V1 = m * tau1;
    const double dV = fabs(V1 - V0);
    a.dtc[c] = Lc / ac;
    a.dtc[nc + c] = dV > 0.0 ? V1 / dV : __builtin_huge_val();
}

template <int D, bool LOOP, bool SG>
__device__ __forceinline__ void update_body(const StepArgs &a, const WorkList &w, const Blk b) {
    for_items<LOOP>(w, b, [&](int64_t c) { update_cell<D, SG>(a, c); });
}
template <int D, bool LOOP, bool SG>
__global__ __launch_bounds__(256) void k_update(StepArgs a, WorkList w) {
    update_body<D, LOOP, SG>(a, w, grid_blk());
}

// LDS stride of a staged gather record: 18 doubles in 3D, so that the
// 16-byte LDS writes of 8 consecutive lanes fall in distinct banks
template <int D>
constexpr int staged_gr() {
    return Dims<D>::GR + (D == 3 ? 2 : 0);
}

// One block per item, gather records staged in LDS (dynamic, blockDim *
// staged_gr doubles): the item's records are one contiguous run, copied
// out after a barrier in 16-byte chunks in address order.
template <int D, bool SG>
__device__ __forceinline__ void update_staged_body(const StepArgs &a, const WorkList &w, const Blk b, double *cs) {
    using Dm = Dims<D>;
    constexpr int LS = staged_gr<D>(), NPR = Dm::GR / 2;
    const int64_t per = (w.n_items + 7) >> 3;
    const int64_t slot = b.id >> 3;
    const int64_t it = (b.id & 7) * per + slot;
    if (slot >= per || it >= w.n_items) return;  // the whole block
    const int64_t s0 = w.start[it];
    const int len = w.len[it];
    if ((int)threadIdx.x < len) update_cell<D, SG, true>(a, s0 + threadIdx.x, cs + threadIdx.x * LS);
    __syncthreads();
    const double2 *src = reinterpret_cast<const double2 *>(cs);
    double2 *out = reinterpret_cast<double2 *>(a.xc + s0 * Dm::GR);
    for (int q = threadIdx.x; q < len * NPR; q += blockDim.x) {
        const int ci = q / NPR, j = q - ci * NPR;
        store_stream(&out[q], src[ci * (LS / 2) + j]);
    }
}
// Three waves per SIMD: the kernel needs 178 VGPRs (two waves) unless
// capped; the cap costs a 12-byte spill and is faster on the 8.1M-tet bar
// (1.077 against 1.165 ms).
template <int D, bool SG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_update_staged(StepArgs a, WorkList w) {
    extern __shared__ double cs[];
    update_staged_body<D, SG>(a, w, grid_blk(), cs);
}

// The cells of a MOOD pass's list, strided over the grid.  (A loop-free
// head for the first gridDim * blockDim entries runs at three waves per
// SIMD instead of two, but the tail launch it needs costs every captured
// pass more than the head saves.)
//
// The pass's bookkeeping rides on its kernels, each step after the last
// reader of what it changes: the first thread of k_pass_cells clears the
// output flag count and the cell list, and logs the input count; the first
// thread of k_update_list clears the node list and advances the stamp for
// the next pass.  k_step_begin clears every count before the first pass.
template <int D, bool SG>
__device__ __forceinline__ void update_list_body(const StepArgs &a, const Blk b, double *sh) {
    const int64_t n = min((int64_t)a.counters[CNT_CELLS], a.nc);
    if (b.tid() == 0) {
        a.counters[CNT_NODES] = 0u;
        a.counters[CNT_RECOMP] += (unsigned)n;
        *a.stamp = *a.stamp + 1;
    }
    double *vsl = sh + threadIdx.x * (D + 1) * D;
    for (int64_t i = b.tid(); i < n; i += b.stride()) update_cell<D, SG, false, true>(a, a.clist[i], nullptr, vsl);
}
template <int D, bool SG>
__global__ __launch_bounds__(256) void k_update_list(StepArgs a) {
    __shared__ double sh[256 * (D + 1) * D];
    update_list_body<D, SG>(a, grid_blk(), sh);
}

// ------------------------------------------------------ MOOD bookkeeping
// A sparse MOOD pass (Section 3.7) in three launches: the flagged cells,
// the nodes they touch, the cells around those nodes.  The pass's stamp is
// the device stamp + 1 (k_update_list advances it at the pass's end).
// First: every flagged cell drops to the next scheme of the cascade, its
// corner records are recomputed at that level, and its nodes are listed
// once.  log (may be null): log[log_idx] = the input count.
template <int D, bool LIM, bool FAM, bool SG>
__device__ __forceinline__ void pass_cells_body(const StepArgs &a, const int32_t *__restrict__ list,
                                                const unsigned *__restrict__ count, unsigned *__restrict__ log,
                                                int log_idx, const Blk b) {
    const int64_t n = min((int64_t)*count, a.nc);
    const int32_t st = *a.stamp + 1;
    if (b.tid() == 0) {
        *a.fcount_out = 0u;
        a.counters[CNT_CELLS] = 0u;
        if (log) log[log_idx] = (unsigned)n;
    }
    uint8_t *mask = const_cast<uint8_t *>(a.mask);
    for (int64_t i = b.tid(); i < n; i += b.stride()) {
        const int32_t c = list[i];
        mask[c] = (a.cascade == 3 && mask[c] == 0) ? 1 : 2;
        predict_cell<D, LIM, FAM, SG>(a, c);
        bool fresh[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) fresh[k] = atomicExch(&a.nstamp[a.c2n[(int64_t)c * (D + 1) + k]], st) != st;
#pragma unroll
        for (int k = 0; k <= D; ++k)
            wave_append(a.nlist, &a.counters[CNT_NODES], fresh[k], a.c2n[(int64_t)c * (D + 1) + k], (unsigned)a.nn);
    }
}
template <int D, bool LIM, bool FAM, bool SG>
__global__ __launch_bounds__(256) void k_pass_cells(StepArgs a, const int32_t *__restrict__ list,
                                                    const unsigned *__restrict__ count, unsigned *__restrict__ log,
                                                    int log_idx) {
    pass_cells_body<D, LIM, FAM, SG>(a, list, count, log, log_idx, grid_blk());
}

// Second: every listed node is solved again by a group of AGG_G lanes (the
// cooperative gather of the full node solve, same sums), and the group
// lists the cells around it once.
template <int D, bool LD>
__device__ __forceinline__ void pass_nodes_body(const StepArgs &a, const Blk bk, unsigned *sh) {
    const int64_t n = min((int64_t)a.counters[CNT_NODES], a.nn);
    const int32_t st = *a.stamp + 1;
    const int l = threadIdx.x & (AGG_G - 1);
    const int per_block = blockDim.x / AGG_G;
    // block-uniform loops (block_append synchronises the block)
    for (int64_t b0 = bk.id * per_block; b0 < n; b0 += bk.n * per_block) {
        const int64_t i = b0 + threadIdx.x / AGG_G;
        int32_t q0 = 0, q1 = 0;
        if (i < n) {
            const int32_t p = a.nlist[i];
            node_solve_group<D, LD>(a, p, l);
            q0 = a.n2c_off[p];
            q1 = a.n2c_off[p + 1];
        }
        for (int32_t q = q0 + l; __syncthreads_or(q < q1); q += AGG_G) {
            bool fresh = false;
            int32_t j = 0;
            if (q < q1) {
                j = a.n2c[q] / (D + 1);
                fresh = atomicExch(&a.cstamp[j], st) != st;
            }
            block_append(a.clist, &a.counters[CNT_CELLS], fresh, j, (unsigned)a.nc, sh);
        }
    }
}
template <int D, bool LD>
__global__ __launch_bounds__(256) void k_pass_nodes(StepArgs a) {
    __shared__ unsigned sh[5];
    pass_nodes_body<D, LD>(a, grid_blk(), sh);
}

// Start of a step: clear the counters, take the device-side dt.
__device__ __forceinline__ void step_begin_body(unsigned *__restrict__ counters, double *__restrict__ dt_cur,
                                                const double *__restrict__ dt_next, int n_mesh, int copy_dt,
                                                const Blk b) {
    const int64_t i = b.tid();
    if (i < CNT_N) counters[i] = 0u;
    if (copy_dt)
        for (int64_t m = i; m < n_mesh; m += b.stride()) dt_cur[m] = dt_next[m];
}
__global__ void k_step_begin(unsigned *__restrict__ counters, double *__restrict__ dt_cur,
                             const double *__restrict__ dt_next, int n_mesh, int copy_dt) {
    step_begin_body(counters, dt_cur, dt_next, n_mesh, copy_dt, grid_blk());
}

// blockIdx.y picks the field; blocks stride over its elements
__global__ __launch_bounds__(256) void k_copy_fields(CopyFields f) {
    const int k = blockIdx.y;
    const int64_t n = f.n[k];
    const double *__restrict__ src = f.src[k];
    double *__restrict__ dst = f.dst[k];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__device__ __forceinline__ void fill_u8_body(uint8_t *__restrict__ p, int64_t n, uint8_t v, const Blk b) {
    for (int64_t i = b.tid(); i < n; i += b.stride()) p[i] = v;
}
__global__ void k_fill_u8(uint8_t *__restrict__ p, int64_t n, uint8_t v) { fill_u8_body(p, n, v, grid_blk()); }

// -------------------------------------------------------- reductions
// Per-mesh minimum of non-negative doubles through their ordered bit
// patterns (order independent, hence deterministic).
__device__ __forceinline__ void atomic_min_pos(double *addr, double v) {
    if (!(v >= 0.0)) return;  // NaN / negative: ignored
    atomicMin(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Per-mesh minima of the two time-step bounds and the count of inadmissible
// first-order cells, stage 1.  A block covers DT_TILES tiles of 256 cells
// (one load of each per thread in flight).  A block inside one mesh writes
// its minima to part[block]; otherwise a tile that straddles meshes takes
// per-cell atomics, the other tiles one atomic per mesh, and part[block]
// is +inf.  The minimum runs on the ordered bit patterns of non-negative
// doubles: order independent, hence deterministic.
constexpr int DT_TILES = 8;
__device__ __forceinline__ void dt_reduce_body(int64_t nc, const double *__restrict__ dtc,
                                               const int32_t *__restrict__ cell_mesh,
                                               const uint8_t *__restrict__ pstat,
                                               double *__restrict__ red /* [n_mesh][2] */,
                                               double *__restrict__ part /* [nblocks][2] */,
                                               unsigned *__restrict__ bad_count, const Blk bk) {
    const int64_t bid = bk.id;
    __shared__ double sa[DT_TILES][4], sv[DT_TILES][4];
    __shared__ int sbad[DT_TILES][4];
    __shared__ int smesh[DT_TILES];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double ac[DT_TILES], vol[DT_TILES];
    int bad[DT_TILES];
#pragma unroll
    for (int g = 0; g < DT_TILES; ++g) {
        const int64_t c = (bid * DT_TILES + g) * 256 + threadIdx.x;
        ac[g] = vol[g] = __builtin_huge_val();
        bad[g] = 0;
        if (c < nc) {
            ac[g] = dtc[c];
            vol[g] = dtc[nc + c];
            bad[g] = pstat[c];
        }
    }
    const int64_t cb0 = bid * DT_TILES * 256;
    const int64_t cb1 = min(cb0 + DT_TILES * 256, nc) - 1;
    if (!cell_mesh || cell_mesh[cb0] == cell_mesh[cb1]) {
        // the block lies in one mesh: one minimum over all its cells
        double a = __builtin_huge_val(), v = __builtin_huge_val();
        int nbad = 0;
#pragma unroll
        for (int g = 0; g < DT_TILES; ++g) {
            a = fmin(a, ac[g] >= 0.0 ? ac[g] : __builtin_huge_val());
            v = fmin(v, vol[g] >= 0.0 ? vol[g] : __builtin_huge_val());
            nbad += __popcll(__ballot(bad[g] != 0));
        }
        a = wave_min(a);
        v = wave_min(v);
        if (lane == 0) {
            sa[0][w] = a;
            sv[0][w] = v;
            sbad[0][w] = nbad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            part[2 * bid] = fmin(fmin(sa[0][0], sa[0][1]), fmin(sa[0][2], sa[0][3]));
            part[2 * bid + 1] = fmin(fmin(sv[0][0], sv[0][1]), fmin(sv[0][2], sv[0][3]));
            const int nb = sbad[0][0] + sbad[0][1] + sbad[0][2] + sbad[0][3];
            if (nb) atomicAdd(bad_count, (unsigned)nb);
        }
        return;
    }
#pragma unroll
    for (int g = 0; g < DT_TILES; ++g) {
        const int64_t first = (bid * DT_TILES + g) * 256;
        const int64_t c = first + threadIdx.x;
        double a = ac[g], v = vol[g];
        if (!(a >= 0.0)) a = __builtin_huge_val();
        if (!(v >= 0.0)) v = __builtin_huge_val();
        int mesh = -1;  // -1: empty tile or straddling tile (done here)
        if (first < nc) {
            const int64_t last = min(first + 255, nc - 1);
            mesh = cell_mesh ? cell_mesh[first] : 0;
            if (cell_mesh && cell_mesh[last] != mesh) {
                if (c < nc) {
                    atomic_min_pos(&red[2 * cell_mesh[c]], a);
                    atomic_min_pos(&red[2 * cell_mesh[c] + 1], v);
                }
                a = v = __builtin_huge_val();
                mesh = -1;
            }
        }
        a = wave_min(a);
        v = wave_min(v);
        const unsigned long long bb = __ballot(bad[g] != 0);
        if (lane == 0) {
            sa[g][w] = a;
            sv[g][w] = v;
            sbad[g][w] = __popcll(bb);
        }
        if (threadIdx.x == 0) smesh[g] = mesh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the block spans meshes: one atomic per run of tiles of one mesh
        int nb = 0;
        int cur = -1;
        double am = __builtin_huge_val(), vm = __builtin_huge_val();
        for (int g = 0; g < DT_TILES; ++g) {
            nb += sbad[g][0] + sbad[g][1] + sbad[g][2] + sbad[g][3];
            const int m = smesh[g];
            if (m < 0) continue;
            const double at = fmin(fmin(sa[g][0], sa[g][1]), fmin(sa[g][2], sa[g][3]));
            const double vt = fmin(fmin(sv[g][0], sv[g][1]), fmin(sv[g][2], sv[g][3]));
            if (m != cur) {
                if (cur >= 0) {
                    atomic_min_pos(&red[2 * cur], am);
                    atomic_min_pos(&red[2 * cur + 1], vm);
                }
                cur = m;
                am = vm = __builtin_huge_val();
            }
            am = fmin(am, at);
            vm = fmin(vm, vt);
        }
        if (cur >= 0) {
            atomic_min_pos(&red[2 * cur], am);
            atomic_min_pos(&red[2 * cur + 1], vm);
        }
        part[2 * bid] = __builtin_huge_val();
        part[2 * bid + 1] = __builtin_huge_val();
        if (nb) atomicAdd(bad_count, (unsigned)nb);
    }
}
__global__ __launch_bounds__(256) void k_dt_reduce(int64_t nc, const double *__restrict__ dtc,
                                                   const int32_t *__restrict__ cell_mesh,
                                                   const uint8_t *__restrict__ pstat, double *__restrict__ red,
                                                   double *__restrict__ part, unsigned *__restrict__ bad_count) {
    dt_reduce_body(nc, dtc, cell_mesh, pstat, red, part, bad_count, grid_blk());
}

// Stage 2: one block per mesh reduces the partials of the stage-1 blocks
// that hold its cells (blocks shared with another mesh left +inf).
__device__ __forceinline__ void dt_reduce2_body(int n_mesh, const int64_t *__restrict__ mesh_cell_off,
                                                const double *__restrict__ part, double *__restrict__ red,
                                                const Blk b) {
    __shared__ double sa[4], sv[4];
    const int64_t m = b.id;
    if (m >= n_mesh) return;
    const int64_t c0 = mesh_cell_off[m], c1 = mesh_cell_off[m + 1];
    double ac = __builtin_huge_val(), vol = __builtin_huge_val();
    if (c1 > c0) {
        constexpr int64_t CH = 256 * DT_TILES;
        const int64_t b0 = c0 / CH, b1 = (c1 - 1) / CH;
#pragma unroll 4
        for (int64_t b = b0 + threadIdx.x; b <= b1; b += blockDim.x) {
            ac = fmin(ac, part[2 * b]);
            vol = fmin(vol, part[2 * b + 1]);
        }
    }
    ac = wave_min(ac);
    vol = wave_min(vol);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sa[w] = ac;
        sv[w] = vol;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomic_min_pos(&red[2 * m], fmin(fmin(sa[0], sa[1]), fmin(sa[2], sa[3])));
        atomic_min_pos(&red[2 * m + 1], fmin(fmin(sv[0], sv[1]), fmin(sv[2], sv[3])));
    }
}
__global__ __launch_bounds__(256) void k_dt_reduce2(int n_mesh, const int64_t *__restrict__ mesh_cell_off,
                                                    const double *__restrict__ part, double *__restrict__ red) {
    dt_reduce2_body(n_mesh, mesh_cell_off, part, red, grid_blk());
}

__global__ void k_fill(double *p, int64_t n, double v) {
    int64_t i = gtid();
    if (i < n) p[i] = v;
}

// dt_next = min(C_CFL min L/a, C_v dt min V1/|dV|, (1 + C_i) dt)
__device__ __forceinline__ void dt_finalize_body(int n_mesh, const double *__restrict__ red,
                                                 const double *__restrict__ dt, double c_cfl, double c_v, double c_i,
                                                 int first, double *__restrict__ dt_next,
                                                 double *__restrict__ parts /* [n_mesh][2] */, const Blk b) {
    const int64_t m = b.tid();
    if (m >= n_mesh) return;
    double ac = c_cfl * red[2 * m];
    double vol = c_v * dt[m] * red[2 * m + 1];
    double d = ac;
    if (!first) d = fmin(fmin(ac, vol), (1.0 + c_i) * dt[m]);
    dt_next[m] = d;
    parts[2 * m] = ac;
    parts[2 * m + 1] = first ? __builtin_huge_val() : vol;
}
__global__ void k_dt_finalize(int n_mesh, const double *__restrict__ red, const double *__restrict__ dt,
                              double c_cfl, double c_v, double c_i, int first, double *__restrict__ dt_next,
                              double *__restrict__ parts /* [n_mesh][2]: acoustic, volume */) {
    dt_finalize_body(n_mesh, red, dt, c_cfl, c_v, c_i, first, dt_next, parts, grid_blk());
}

// acoustic bound of the current state (initial time step)
template <int D>
__global__ __launch_bounds__(256) void k_acoustic(StepArgs a) {
    constexpr int NV = D + 1;
    const int64_t nc = a.nc, nn = a.nn;
    const int32_t *__restrict__ c2n = a.c2n;
    const double *__restrict__ x = a.x;
    double *__restrict__ dtc = a.dtc;
    int64_t c = gtid();
    if (c >= nc) return;
    double X[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        int64_t p = c2n[c * NV + k];
#pragma unroll
        for (int i = 0; i < D; ++i) X[k][i] = x[i * nn + p];
    }
    Geo<D> g;
    geom<D>(X, g);
    double S = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) S += g.cn[k];
    double ac;
    if (a.eos) {
        double b[6], k2 = 0.0;
        load_B6<D>(a.B, nc, c, b);
#pragma unroll
        for (int i = 0; i < D; ++i) k2 += a.v[i * nc + c] * a.v[i * nc + c];
        ac = sound_sg(a.rho0[c], a.mu[c], a.shear_a, a.sg_gamma, a.sg_pinf, a.tau[c], b, a.e[c] - 0.5 * k2);
    } else {
        ac = sound(a.rho0[c], a.mu[c], a.K[c], a.tau[c]);
    }
    dtc[c] = 2.0 * g.V / S / ac;
    dtc[nc + c] = __builtin_huge_val();
}

// Diagnostics: per-block partials (fixed order), then one block per
// column combines the partials in block order.  Columns 0..8 and 11 are
// sums (mass, mom[3], m e, kinetic, elastic, n_p0, n_limited, n_detB),
// columns 9 and 10 maxima (GCL defect, det B defect).
constexpr int NDIAG = DIAG_N;
__device__ __forceinline__ bool diag_is_max(int s) { return s == 9 || s == 10; }

// Involution monitors of cell c after the step (Section 3.5): the discrete
// GCL V(x^{n+1}) - V(x^n) = dt sum_k Cbar_k . v*_k with Cbar the Simpson
// average of the corner vectors at t^n, t^{n+1/2}, t^{n+1} (exact for the
// straight node paths x^n + t v*), relative to V(x^n); and
// |sqrt(det B^{n+1}) - J^{n+1}| (eq. test_detB_rho, J = rho0 tau) with the
// in-sphere diameter L_c of t^{n+1}.
template <int D>
__device__ __forceinline__ void involution(const StepArgs &a, int64_t c, const double *__restrict__ x1,
                                           const double b1[6], double tau1, double *gcl, double *dB,
                                           double *Lc3) {
    constexpr int NV = D + 1;
    const int64_t nn = a.nn;
    const double dt = mesh_dt(a.dt, a.cell_mesh, c);
    double X0[NV][D], Xh[NV][D], X1[NV][D], vs[NV][D];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int64_t p = a.c2n[c * NV + k];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            X0[k][i] = a.x[i * nn + p];
            vs[k][i] = a.vstar[i * nn + p];
            Xh[k][i] = X0[k][i] + 0.5 * dt * vs[k][i];
            X1[k][i] = x1[i * nn + p];
        }
    }
    Geo<D> g0, gh, g1;
    geom<D>(X0, g0);
    geom<D>(Xh, gh);
    geom<D>(X1, g1);
    double flux = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int i = 0; i < D; ++i) flux += (g0.C[k][i] + 4.0 * gh.C[k][i] + g1.C[k][i]) * (1.0 / 6.0) * vs[k][i];
    *gcl = fabs(g1.V - g0.V - dt * flux) / g0.V;
    *dB = fabs(sqrt(det6(b1)) - a.rho0[c] * tau1);
    double S = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) S += g1.cn[k];
    const double Lc = 2.0 * g1.V / S;
    *Lc3 = Lc * Lc * Lc;
}

template <int D>
__global__ __launch_bounds__(256) void k_diag(StepArgs a, double *__restrict__ part) {
    __shared__ double sh[NDIAG][256];
    const int64_t nc = a.nc;
    const double *__restrict__ m = a.mass, *__restrict__ tau = a.tau1, *__restrict__ v = a.v1,
                                *__restrict__ e = a.e1, *__restrict__ B = a.B1, *__restrict__ rho0 = a.rho0,
                                *__restrict__ mu = a.mu, *__restrict__ K = a.K;
    const uint8_t *__restrict__ mask = a.mask;
    const double shear_a = a.shear_a;
    const int eos = a.eos;
    int64_t c = gtid();
    double q[NDIAG] = {};
    if (c < nc) {
        double mc = m[c];
        double k2 = 0.0;
        q[0] = mc;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double vi = v[i * nc + c];
            q[1 + i] = mc * vi;
            k2 += vi * vi;
        }
        q[4] = mc * e[c];
        q[5] = 0.5 * mc * k2;
        double b[6];
        load_B6<D>(B, nc, c, b);
        double J = rho0[c] * tau[c];
        double lj = log(J);
        double cJ = cbrt(J);
        double I1b = (b[0] + b[1] + b[2]) / (cJ * cJ);
        double psi = eos ? shear_energy6(rho0[c], mu[c], shear_a, tau[c], b)   // stiffened gas: Psi_s
                     : shear_a == -1.0
                         ? K[c] / (4.0 * rho0[c]) * ((J - 1.0) * (J - 1.0) + lj * lj) +
                               mu[c] / (2.0 * rho0[c]) * (I1b - 3.0)
                         : free_energy_family(rho0[c], mu[c], K[c], shear_a, tau[c], b);
        q[6] = mc * psi;
        q[7] = mask[c] >= 2 ? 1.0 : 0.0;   // first order
        q[8] = mask[c] == 1 ? 1.0 : 0.0;   // limited slopes
        double gcl, dB, Lc3;
        involution<D>(a, c, a.x1, b, tau[c], &gcl, &dB, &Lc3);
        q[9] = gcl;
        q[10] = dB;
        q[11] = dB >= Lc3 ? 1.0 : 0.0;
    }
#pragma unroll
    for (int s = 0; s < NDIAG; ++s) sh[s][threadIdx.x] = q[s];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int s = 0; s < NDIAG; ++s)
                sh[s][threadIdx.x] = diag_is_max(s) ? fmax(sh[s][threadIdx.x], sh[s][threadIdx.x + w])
                                                    : sh[s][threadIdx.x] + sh[s][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NDIAG; ++s) part[blockIdx.x * NDIAG + s] = sh[s][0];
    }
}

// one block per sum; fixed strided order then a fixed tree: deterministic
__global__ __launch_bounds__(256) void k_diag_finalize(int64_t nblocks, const double *__restrict__ part,
                                                       double *__restrict__ out) {
    __shared__ double sh[256];
    const int s = blockIdx.x;
    const bool mx = diag_is_max(s);
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x)
        acc = mx ? fmax(acc, part[b * NDIAG + s]) : acc + part[b * NDIAG + s];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + w]) : sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = sh[0];
}

// AoS [n][w] (the caller's numbering) <-> SoA [w][n] (the internal one)
// copies for the ABI; row i of the AoS side is entity idx[i] of the SoA
// side (idx null: entity i).
__global__ void k_aos_to_soa(int64_t n, int w, const double *__restrict__ in, const int32_t *__restrict__ idx,
                             double *__restrict__ out) {
    int64_t i = gtid();
    if (i >= n) return;
    const int64_t j = idx ? idx[i] : i;
    for (int k = 0; k < w; ++k) out[k * n + j] = in[i * w + k];
}

__global__ void k_soa_to_aos(int64_t n, int w, const double *__restrict__ in, const int32_t *__restrict__ idx,
                             double *__restrict__ out) {
    int64_t i = gtid();
    if (i >= n) return;
    const int64_t j = idx ? idx[i] : i;
    for (int k = 0; k < w; ++k) out[i * w + k] = in[k * n + j];
}

// out row i = in row idx[i] (AoS, w values per row)
__global__ void k_gather_rows(int64_t n, int w, const double *__restrict__ in, const int32_t *__restrict__ idx,
                              double *__restrict__ out) {
    int64_t i = gtid();
    if (i >= n) return;
    const int64_t j = idx[i];
    for (int k = 0; k < w; ++k) out[i * w + k] = in[j * w + k];
}

__global__ void k_gather_u8(int64_t n, const uint8_t *__restrict__ in, const int32_t *__restrict__ idx,
                            uint8_t *__restrict__ out) {
    int64_t i = gtid();
    if (i < n) out[i] = in[idx[i]];
}

// stress of the current state for queries: 3D (11,22,33,12,13,23),
// 2D (11,22,12,33), AoS; row i is cell idx[i] (idx null: cell i)
template <int D>
__global__ void k_stress_query(StepArgs a, const int32_t *__restrict__ idx, double *__restrict__ out) {
    const int64_t nc = a.nc;
    const double *__restrict__ tau = a.tau, *__restrict__ rho0 = a.rho0, *__restrict__ mu = a.mu,
                                *__restrict__ K = a.K;
    const double shear_a = a.shear_a;
    const int64_t i = gtid();
    if (i >= nc) return;
    const int64_t c = idx ? idx[i] : i;
    double b[6], t[6];
    load_B6<D>(a.B, nc, c, b);
    if (a.eos) {
        double k2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) k2 += a.v[i * nc + c] * a.v[i * nc + c];
        stress6_sg(rho0[c], mu[c], shear_a, a.sg_gamma, a.sg_pinf, tau[c], b, a.e[c] - 0.5 * k2, t);
    } else if (shear_a == -1.0)
        stress6(rho0[c], mu[c], K[c], tau[c], b, t);
    else
        stress6_family(rho0[c], mu[c], K[c], shear_a, tau[c], b, t);
    if (D == 3) {
        for (int s = 0; s < 6; ++s) out[i * 6 + s] = t[s];
    } else {
        out[i * 4 + 0] = t[0];
        out[i * 4 + 1] = t[1];
        out[i * 4 + 2] = t[3];
        out[i * 4 + 3] = t[2];
    }
}

// ---------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int D>
void launch_centroids(const StepArgs &a, const Sched &k, hipStream_t s) {
    if (!k.w.n_items) return;
    if (k.loop)
        k_pack<D, true><<<k.grid, k.block, 0, s>>>(a, k.w);
    else
        k_pack<D, false><<<k.grid, k.block, 0, s>>>(a, k.w);
}
template <int D>
void launch_node_agg(const StepArgs &a, const Sched &k, hipStream_t s) {
    if (!k.w.n_items) return;
    if (k.loop)
        k_node_agg<D, true><<<k.grid, k.block, 0, s>>>(a, k.w);
    else
        k_node_agg<D, false><<<k.grid, k.block, 0, s>>>(a, k.w);
}
// LDS of a staged predictor launch: its record stage, or its node tiles if
// they are larger (the two share the memory)
template <int D>
size_t predict_lds_bytes(const Sched &k) {
    const size_t rec = sizeof(double) * (size_t)(D + 1) * k.block * (Dims<D>::NMS + D);
    const size_t tile = k.w.tn_off ? sizeof(double2) * (size_t)k.w.tn_max * tile_pairs<D>() : 0;
    return std::max(rec, tile);
}
template <int D>
void launch_predict(const StepArgs &a, const Sched &k, hipStream_t s) {
    if (!k.w.n_items) return;
    const bool lim = a.limited == 2, fam = a.shear_a != -1.0;
#define HL_PREDICT_LAUNCH(L, M, F) k_predict<D, L, M, F, false><<<k.grid, k.block, 0, s>>>(a, k.w)
    if (a.eos) {  // stiffened gas: never with the limited level
        if (k.loop)
            k_predict<D, true, false, false, true><<<k.grid, k.block, 0, s>>>(a, k.w);
        else
            k_predict_staged<D, false, false, true>
                <<<k.grid, k.block, sizeof(double) * (size_t)(D + 1) * k.block * (Dims<D>::NMS + D), s>>>(a, k.w);
    } else if (k.loop) {
        if (fam)
            lim ? HL_PREDICT_LAUNCH(true, true, true) : HL_PREDICT_LAUNCH(true, false, true);
        else
            lim ? HL_PREDICT_LAUNCH(true, true, false) : HL_PREDICT_LAUNCH(true, false, false);
    } else {
        // one block per item: corner records staged through LDS (not for the
        // shear family, whose staged body no longer fits two waves per SIMD),
        // node values from the item's node tile when the list has them
        const size_t lds = predict_lds_bytes<D>(k);
        if (fam)
            lim ? HL_PREDICT_LAUNCH(false, true, true) : HL_PREDICT_LAUNCH(false, false, true);
        else if (k.w.tn_off)
            lim ? k_predict_staged<D, true, false, false, true><<<k.grid, k.block, lds, s>>>(a, k.w)
                : k_predict_staged<D, false, false, false, true><<<k.grid, k.block, lds, s>>>(a, k.w);
        else if (lim)
            k_predict_staged<D, true, false, false><<<k.grid, k.block, lds, s>>>(a, k.w);
        else
            k_predict_staged<D, false, false, false><<<k.grid, k.block, lds, s>>>(a, k.w);
    }
#undef HL_PREDICT_LAUNCH
}
template <int D>
void launch_node_solve(const StepArgs &a, const Sched &k, hipStream_t s) {
    if (!k.w.n_items) return;
    const bool ld = a.ld_off != nullptr;
    if (k.loop)
        ld ? k_node_solve<D, true, true><<<k.grid, k.block, 0, s>>>(a, k.w)
           : k_node_solve<D, true, false><<<k.grid, k.block, 0, s>>>(a, k.w);
    else
        ld ? k_node_solve<D, false, true><<<k.grid, k.block, 0, s>>>(a, k.w)
           : k_node_solve<D, false, false><<<k.grid, k.block, 0, s>>>(a, k.w);
}
void launch_contact_apply(const ContactArgs &k, int dim, hipStream_t s) {
    if (k.n) k_contact_apply<<<nblk(k.n), 256, 0, s>>>(k, dim * dim);
}
template <int D>
void launch_contact_eval(const StepArgs &a, const ContactArgs &k, hipStream_t s) {
    if (!k.n) return;
    if (a.ld_off)
        k_contact_eval<D, true><<<nblk(k.n), 256, 0, s>>>(a, k);
    else
        k_contact_eval<D, false><<<nblk(k.n), 256, 0, s>>>(a, k);
}
template <int D>
void launch_update(const StepArgs &a, const Sched &k, hipStream_t s) {
    if (!k.w.n_items) return;
    if (k.loop)
        a.eos ? k_update<D, true, true><<<k.grid, k.block, 0, s>>>(a, k.w)
              : k_update<D, true, false><<<k.grid, k.block, 0, s>>>(a, k.w);
    else {
        const size_t lds = sizeof(double) * (size_t)k.block * staged_gr<D>();
        a.eos ? k_update_staged<D, true><<<k.grid, k.block, lds, s>>>(a, k.w)
              : k_update_staged<D, false><<<k.grid, k.block, lds, s>>>(a, k.w);
    }
}
template <int D>
void launch_mood_sparse(const StepArgs &a, const int32_t *flist, const unsigned *fcount, int64_t nflag,
                        int64_t max_deg, bool fixed_grid, unsigned *log, int log_idx, hipStream_t s) {
    // fixed grids (graph capture) are capped at 1024 blocks: the kernels
    // stride over their lists, and an empty pass then launches few blocks
    const int64_t gmax = fixed_grid ? 1024 : 16384;
    auto grid = [gmax](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, gmax)); };
    if (fixed_grid) nflag = std::min<int64_t>(a.nc, 256 * 1024);
    const int64_t nnodes = std::min<int64_t>(a.nn, (D + 1) * nflag);
    const int64_t ncells = std::min<int64_t>(a.nc, nnodes * max_deg);
    const bool fam = a.shear_a != -1.0;
    if (a.eos)
        k_pass_cells<D, false, false, true><<<grid(nflag), 256, 0, s>>>(a, flist, fcount, log, log_idx);
    else if (a.limited)
        fam ? k_pass_cells<D, true, true, false><<<grid(nflag), 256, 0, s>>>(a, flist, fcount, log, log_idx)
            : k_pass_cells<D, true, false, false><<<grid(nflag), 256, 0, s>>>(a, flist, fcount, log, log_idx);
    else
        fam ? k_pass_cells<D, false, true, false><<<grid(nflag), 256, 0, s>>>(a, flist, fcount, log, log_idx)
            : k_pass_cells<D, false, false, false><<<grid(nflag), 256, 0, s>>>(a, flist, fcount, log, log_idx);
    if (a.ld_off)
        k_pass_nodes<D, true><<<grid(AGG_G * nnodes), 256, 0, s>>>(a);
    else
        k_pass_nodes<D, false><<<grid(AGG_G * nnodes), 256, 0, s>>>(a);
    if (a.eos)
        k_update_list<D, true><<<grid(ncells), 256, 0, s>>>(a);
    else
        k_update_list<D, false><<<grid(ncells), 256, 0, s>>>(a);
}
void launch_step_begin(unsigned *counters, double *dt_cur, const double *dt_next, int n_mesh, int copy_dt,
                       hipStream_t s) {
    k_step_begin<<<std::max(1, (n_mesh + 255) / 256), 256, 0, s>>>(counters, dt_cur, dt_next, n_mesh, copy_dt);
}
void launch_copy_fields(const CopyFields &f, hipStream_t s) {
    int64_t m = 0;
    for (int k = 0; k < 6; ++k) m = std::max<int64_t>(m, f.n[k]);
    if (m) k_copy_fields<<<dim3((unsigned)std::min<int64_t>((m + 255) / 256, 2048), 6), 256, 0, s>>>(f);
}
void launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
    if (n) k_fill_u8<<<std::min<unsigned>(nblk(n), 4096), 256, 0, s>>>(p, n, v);
}
// Start of a CFL reduction: per-mesh minima to +inf, the inadmissible
// count to 0 (a reduction repeated after further MOOD passes counts afresh).
__device__ __forceinline__ void reduce_begin_body(double *__restrict__ red, int64_t n, unsigned *__restrict__ bad_count,
                                                  const Blk b) {
    const int64_t i = b.tid();
    if (i < n) red[i] = __builtin_huge_val();
    if (i == 0) *bad_count = 0u;
}
__global__ void k_reduce_begin(double *__restrict__ red, int64_t n, unsigned *__restrict__ bad_count) {
    reduce_begin_body(red, n, bad_count, grid_blk());
}

void launch_dt_reduce(int64_t nc, const double *dtc, const int32_t *cell_mesh, const uint8_t *pstat, double *red,
                      double *part, const int64_t *mesh_cell_off, int n_mesh, unsigned *bad_count, hipStream_t s) {
    k_reduce_begin<<<nblk(2 * n_mesh), 256, 0, s>>>(red, 2 * n_mesh, bad_count);
    if (nc) {
        const int64_t nb = (nc + 256 * DT_TILES - 1) / (256 * DT_TILES);
        k_dt_reduce<<<(unsigned)nb, 256, 0, s>>>(nc, dtc, cell_mesh, pstat, red, part, bad_count);
        k_dt_reduce2<<<n_mesh, 256, 0, s>>>(n_mesh, mesh_cell_off, part, red);
    }
}
void launch_dt_finalize(int n_mesh, const double *red, const double *dt, const hl_params &p, int first,
                        double *dt_next, double *parts, hipStream_t s) {
    k_dt_finalize<<<nblk(n_mesh), 256, 0, s>>>(n_mesh, red, dt, p.c_cfl, p.c_v, p.c_i, first, dt_next, parts);
}
template <int D>
void launch_acoustic(const StepArgs &a, hipStream_t s) {
    if (a.nc) k_acoustic<D><<<nblk(a.nc), 256, 0, s>>>(a);
}
template <int D>
int64_t launch_diag(const StepArgs &a, double *part, double *out, hipStream_t s) {
    int64_t nb = nblk(a.nc);
    if (a.nc) k_diag<D><<<nb, 256, 0, s>>>(a, part);
    k_diag_finalize<<<NDIAG, 256, 0, s>>>(a.nc ? nb : 0, part, out);
    return nb;
}
void launch_fill(double *p, int64_t n, double v, hipStream_t s) {
    if (n) k_fill<<<nblk(n), 256, 0, s>>>(p, n, v);
}
void launch_aos_to_soa(int64_t n, int w, const double *in, double *out, hipStream_t s, const int32_t *idx) {
    if (n) k_aos_to_soa<<<nblk(n), 256, 0, s>>>(n, w, in, idx, out);
}
void launch_soa_to_aos(int64_t n, int w, const double *in, double *out, hipStream_t s, const int32_t *idx) {
    if (n) k_soa_to_aos<<<nblk(n), 256, 0, s>>>(n, w, in, idx, out);
}
void launch_gather_rows(int64_t n, int w, const double *in, const int32_t *idx, double *out, hipStream_t s) {
    if (n) k_gather_rows<<<nblk(n), 256, 0, s>>>(n, w, in, idx, out);
}
void launch_gather_u8(int64_t n, const uint8_t *in, const int32_t *idx, uint8_t *out, hipStream_t s) {
    if (n) k_gather_u8<<<nblk(n), 256, 0, s>>>(n, in, idx, out);
}
template <int D>
void launch_stress_query(const StepArgs &a, const int32_t *idx, double *out, hipStream_t s) {
    if (a.nc) k_stress_query<D><<<nblk(a.nc), 256, 0, s>>>(a, idx, out);
}

// ------------------------------------------------- paired launches
// The stages of a 2D and a 3D context in one launch (hl_group_step): blocks
// [0, g0) run the first part, the rest the second, each on its own arguments
// and work list exactly as its own launch would.  Every body is the one the
// single-context kernels run, so the results are bitwise theirs.  Parts run
// the base configuration: neo-Hookean law, two-level cascade, no boundary
// loads (the host checks this).
template <class F0, class F1>
__global__ __launch_bounds__(256) void k_pair(F0 f0, int64_t g0, F1 f1) {
    extern __shared__ double dyn[];
    if ((int64_t)blockIdx.x < g0)
        f0(Blk{(int64_t)blockIdx.x, g0}, dyn);
    else
        f1(Blk{(int64_t)blockIdx.x - g0, (int64_t)gridDim.x - g0}, dyn);
}

namespace {
template <int D, bool LOOP>
struct FNodeAgg {
    StepArgs a;
    WorkList w;
    __device__ void operator()(Blk b, double *sh) const { node_agg_body<D, LOOP>(a, w, b, sh); }
};
template <int D, bool LOOP>
struct FPredict {
    StepArgs a;
    WorkList w;
    __device__ void operator()(Blk b, double *sh) const {
        // one-item predictor lists of a group always carry node tiles
        if (LOOP)
            predict_body<D, true, false, false, false>(a, w, b);
        else
            predict_staged_body<D, false, false, false, true>(a, w, b, sh);
    }
};
template <int D, bool LOOP>
struct FNodeSolve {
    StepArgs a;
    WorkList w;
    __device__ void operator()(Blk b, double *) const { node_solve_body<D, LOOP, false>(a, w, b); }
};
template <int D, bool LOOP>
struct FUpdate {
    StepArgs a;
    WorkList w;
    __device__ void operator()(Blk b, double *sh) const {
        if (LOOP)
            update_body<D, true, false>(a, w, b);
        else
            update_staged_body<D, false>(a, w, b, sh);
    }
};
template <int D>
struct FPassCells {
    StepArgs a;
    const int32_t *list;
    const unsigned *count;
    unsigned *log;
    int log_idx;
    __device__ void operator()(Blk b, double *) const {
        pass_cells_body<D, false, false, false>(a, list, count, log, log_idx, b);
    }
};
template <int D>
struct FPassNodes {
    StepArgs a;
    __device__ void operator()(Blk b, double *sh) const {
        pass_nodes_body<D, false>(a, b, reinterpret_cast<unsigned *>(sh));
    }
};
template <int D>
struct FUpdateList {
    StepArgs a;
    __device__ void operator()(Blk b, double *sh) const { update_list_body<D, false>(a, b, sh); }
};
// start of a step: counters, device dt, and the cascade levels to 0
struct FBegin {
    PairBook k;
    __device__ void operator()(Blk b, double *) const {
        step_begin_body(k.counters, k.dt_cur, k.dt_next, k.n_mesh, k.copy_dt, b);
        fill_u8_body(k.mask, k.nc, 0, b);
    }
};
struct FReduceBegin {
    PairBook k;
    __device__ void operator()(Blk b, double *) const { reduce_begin_body(k.red, 2 * k.n_mesh, k.bad_count, b); }
};
struct FDtReduce {
    PairBook k;
    __device__ void operator()(Blk b, double *) const {
        dt_reduce_body(k.nc, k.dtc, k.cell_mesh, k.pstat, k.red, k.part, k.bad_count, b);
    }
};
struct FDtReduce2 {
    PairBook k;
    __device__ void operator()(Blk b, double *) const { dt_reduce2_body(k.n_mesh, k.mesh_cell_off, k.part, k.red, b); }
};
struct FDtFinalize {
    PairBook k;
    __device__ void operator()(Blk b, double *) const {
        dt_finalize_body(k.n_mesh, k.red, k.dt_cur, k.c_cfl, k.c_v, k.c_i, 0, k.dt_next, k.parts, b);
    }
};

unsigned round8(int64_t n) { return (unsigned)((n + 7) & ~(int64_t)7); }

// one paired launch: part grids g0, g1 (either may be 0), one block size
template <class F0, class F1>
void pair_launch(const F0 &f0, unsigned g0, const F1 &f1, unsigned g1, unsigned block, size_t lds, hipStream_t s) {
    if (g0 + g1 == 0) return;
    k_pair<F0, F1><<<g0 + g1, block, lds, s>>>(f0, (int64_t)g0, f1);
}

// a cell or node stage whose body is F<D, LOOP> on each part's schedule
template <template <int, bool> class F>
void pair_stage(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, size_t lds,
                hipStream_t s) {
    const unsigned g2 = k2.w.n_items ? k2.grid : 0, g3 = k3.w.n_items ? k3.grid : 0;
    const unsigned block = g2 ? k2.block : k3.block;
    if (k2.loop) {
        if (k3.loop)
            pair_launch(F<2, true>{a2, k2.w}, g2, F<3, true>{a3, k3.w}, g3, block, lds, s);
        else
            pair_launch(F<2, true>{a2, k2.w}, g2, F<3, false>{a3, k3.w}, g3, block, lds, s);
    } else {
        if (k3.loop)
            pair_launch(F<2, false>{a2, k2.w}, g2, F<3, true>{a3, k3.w}, g3, block, lds, s);
        else
            pair_launch(F<2, false>{a2, k2.w}, g2, F<3, false>{a3, k3.w}, g3, block, lds, s);
    }
}
}  // namespace

void launch_node_agg_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)std::max(agg_lds_doubles<2>(), agg_lds_doubles<3>());
    pair_stage<FNodeAgg>(a2, k2, a3, k3, lds, s);
}
void launch_predict_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, hipStream_t s) {
    const size_t lds = std::max(predict_lds_bytes<2>(k2), predict_lds_bytes<3>(k3));
    pair_stage<FPredict>(a2, k2, a3, k3, lds, s);
}
void launch_node_solve_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3,
                            hipStream_t s) {
    pair_stage<FNodeSolve>(a2, k2, a3, k3, 0, s);
}
void launch_update_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)std::max(k2.block, k3.block) * std::max(staged_gr<2>(), staged_gr<3>());
    pair_stage<FUpdate>(a2, k2, a3, k3, lds, s);
}
void launch_mood_sparse_pair(const StepArgs &a2, const PairPass &p2, const StepArgs &a3, const PairPass &p3,
                             bool fixed_grid, int log_idx, hipStream_t s) {
    // the grids of launch_mood_sparse, per part
    const int64_t gmax = fixed_grid ? 1024 : 16384;
    auto grid = [gmax](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, gmax)); };
    auto shape = [&](const StepArgs &a, const PairPass &p, int d, unsigned g[3]) {
        const int64_t nflag = fixed_grid ? std::min<int64_t>(a.nc, 256 * 1024) : p.nflag;
        const int64_t nnodes = std::min<int64_t>(a.nn, (d + 1) * nflag);
        const int64_t ncells = std::min<int64_t>(a.nc, nnodes * p.max_deg);
        g[0] = round8(grid(nflag));
        g[1] = round8(grid(AGG_G * nnodes));
        g[2] = round8(grid(ncells));
    };
    unsigned g2[3], g3[3];
    shape(a2, p2, 2, g2);
    shape(a3, p3, 3, g3);
    pair_launch(FPassCells<2>{a2, p2.flist, p2.fcount, p2.log, log_idx}, g2[0],
                FPassCells<3>{a3, p3.flist, p3.fcount, p3.log, log_idx}, g3[0], 256, 0, s);
    pair_launch(FPassNodes<2>{a2}, g2[1], FPassNodes<3>{a3}, g3[1], 256, sizeof(double) * 4, s);
    pair_launch(FUpdateList<2>{a2}, g2[2], FUpdateList<3>{a3}, g3[2], 256, sizeof(double) * 256 * 4 * 3, s);
}
void launch_step_begin_pair(const PairBook &b2, const PairBook &b3, hipStream_t s) {
    auto g = [](const PairBook &b) {
        return round8(std::min<int64_t>(std::max<int64_t>(nblk(std::max<int64_t>(b.nc, b.n_mesh)), 1), 4096));
    };
    pair_launch(FBegin{b2}, g(b2), FBegin{b3}, g(b3), 256, 0, s);
}
void launch_dt_reduce_pair(const PairBook &b2, const PairBook &b3, hipStream_t s) {
    auto gb = [](const PairBook &b) { return round8(nblk(2 * b.n_mesh)); };
    pair_launch(FReduceBegin{b2}, gb(b2), FReduceBegin{b3}, gb(b3), 256, 0, s);
    // exact grids: a block past the cells would read past them (the
    // reduction does not use the XCD grouping)
    auto gr = [](const PairBook &b) { return (unsigned)((b.nc + 256 * DT_TILES - 1) / (256 * DT_TILES)); };
    pair_launch(FDtReduce{b2}, gr(b2), FDtReduce{b3}, gr(b3), 256, 0, s);
    auto g2 = [](const PairBook &b) { return b.nc ? (unsigned)b.n_mesh : 0u; };
    pair_launch(FDtReduce2{b2}, g2(b2), FDtReduce2{b3}, g2(b3), 256, 0, s);
    auto gf = [](const PairBook &b) { return round8(nblk(b.n_mesh)); };
    pair_launch(FDtFinalize{b2}, gf(b2), FDtFinalize{b3}, gf(b3), 256, 0, s);
}

template void launch_centroids<2>(const StepArgs &, const Sched &, hipStream_t);
template void launch_centroids<3>(const StepArgs &, const Sched &, hipStream_t);
template void launch_node_agg<2>(const StepArgs &, const Sched &, hipStream_t);
template void launch_node_agg<3>(const StepArgs &, const Sched &, hipStream_t);
template void launch_predict<2>(const StepArgs &, const Sched &, hipStream_t);
template void launch_predict<3>(const StepArgs &, const Sched &, hipStream_t);
template void launch_contact_eval<2>(const StepArgs &, const ContactArgs &, hipStream_t);
template void launch_contact_eval<3>(const StepArgs &, const ContactArgs &, hipStream_t);
template void launch_node_solve<2>(const StepArgs &, const Sched &, hipStream_t);
template void launch_node_solve<3>(const StepArgs &, const Sched &, hipStream_t);
template void launch_update<2>(const StepArgs &, const Sched &, hipStream_t);
template void launch_update<3>(const StepArgs &, const Sched &, hipStream_t);
template void launch_mood_sparse<2>(const StepArgs &, const int32_t *, const unsigned *, int64_t, int64_t, bool,
                                    unsigned *, int, hipStream_t);
template void launch_mood_sparse<3>(const StepArgs &, const int32_t *, const unsigned *, int64_t, int64_t, bool,
                                    unsigned *, int, hipStream_t);
template void launch_acoustic<2>(const StepArgs &, hipStream_t);
template void launch_acoustic<3>(const StepArgs &, hipStream_t);
template int64_t launch_diag<2>(const StepArgs &, double *, double *, hipStream_t);
template int64_t launch_diag<3>(const StepArgs &, double *, double *, hipStream_t);
template void launch_stress_query<2>(const StepArgs &, const int32_t *, double *, hipStream_t);
template void launch_stress_query<3>(const StepArgs &, const int32_t *, double *, hipStream_t);

}  // namespace hl
