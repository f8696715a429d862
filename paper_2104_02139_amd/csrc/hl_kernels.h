// hl_kernels.h -- launch interface between the host side of libhyperlag
// (hl_api.hip) and its HIP kernels (hl_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "hl_device.h"
#include "hyperlag.h"

namespace hl {

// Device pointers of one step (state n -> candidate n+1).
struct StepArgs {
    int64_t nc, nn;
    const int32_t *c2n, *n2c_off, *n2c;
    const uint8_t *nallow;
    const double *allow;
    const double *mass, *rho0, *mu, *K;
    const int32_t *cell_mesh, *node_mesh;  // may be null (one mesh)
    const double *dt;                      // [n_mesh]
    // state n
    const double *x, *vhat, *tau, *v, *e, *B;
    // candidate n+1
    double *x1, *vhat1, *tau1, *v1, *e1, *B1;
    double *vstar;
    // work
    double *xc, *agg, *corner, *dtc;
    const uint8_t *mask;
    uint8_t *pstat;            // 1: first-order cell whose candidate is not admissible
    // MOOD lists: flagged cells appended to flist_out (count fcount_out);
    // re-solved nodes and recomputed cells, deduplicated by stamps
    int32_t *flist_out;
    unsigned *fcount_out;
    int32_t *nlist, *clist;
    int32_t *nstamp, *cstamp;
    int32_t *stamp;            // device: stamp of the last MOOD pass; a pass stamps with *stamp + 1
    unsigned int *counters;    // [CNT_NODES], [CNT_CELLS], [CNT_BAD]
    double delta0, delta1, eps_tol;
    int detect;
    int cascade;   // 2: a flagged cell goes to first order; 3: to limited first
    double shear_a;  // shear energy family parameter; -1: neo-Hookean
    int eos;       // 1: stiffened gas (gamma, p_inf) for the volumetric part
    double sg_gamma, sg_pinf;
    int limited;   // 0: no limited cells; 1: they appear in the MOOD passes
                   // (node W bounds, limiter in the pass kernels); 2: also in
                   // the full-mesh pass (replayed levels)
    // Boundary loads grouped by node (all null when there are none): the
    // entries of node p are ld_off[p] .. ld_off[p+1]-1; entry q is the face
    // opposite local node (ld_fk[q] & 3) of cell ld_cell[q], of kind
    // ld_fk[q] >> 2 (1 traction, 2 normal velocity), with values
    // ld_val[6q .. 6q+5].
    const int32_t *ld_off, *ld_cell;
    const uint8_t *ld_fk;
    const double *ld_val;
};

// device counters of a step: flag counts of the two flag lists, nodes and
// cells listed by the current MOOD pass, inadmissible first-order cells,
// cell updates redone by the MOOD passes of the step
enum { CNT_F0 = 0, CNT_F1 = 1, CNT_NODES = 2, CNT_CELLS = 3, CNT_BAD = 4, CNT_RECOMP = 5, CNT_N = 8 };

// Corner records are stored corner-major within tiles of 256 cells: the
// record of corner k of cell c is number ((c / 256) (D + 1) + k) 256 +
// c % 256.  Lanes of consecutive cells then write and read consecutive
// records, while each record stays contiguous for the nodes that gather it.
// The array holds whole tiles: ceil(n_cells / 256) 256 (D + 1) records.
template <int D>
__host__ __device__ __forceinline__ int64_t corner_slot(int64_t c, int k) {
    return ((((c >> 8) * (D + 1)) + k) << 8) + (c & 255);
}
template <int D>
__host__ __device__ __forceinline__ int64_t corner_slot_of(int64_t corner_id) {
    return corner_slot<D>(corner_id / (D + 1), (int)(corner_id % (D + 1)));
}

// Node aggregates are stored pair-interleaved over nodes: values (2j, 2j+1)
// of node p form the double2 at index j * nn + p.  A cell gathers the same
// values of its nodes in every lane, and the nodes of neighbouring cells are
// close in number, so one wave-wide load touches a few cache lines instead of
// one line per lane.
struct AggRef {
    const double2 *b;
    int64_t nn;
    __device__ __forceinline__ AggRef(const double *agg, int64_t nn_, int64_t p)
        : b(reinterpret_cast<const double2 *>(agg) + p), nn(nn_) {}
    __device__ __forceinline__ double operator[](int j) const {
        const double2 t = b[(int64_t)(j >> 1) * nn];
        return (j & 1) ? t.y : t.x;
    }
};

template <int N>
__device__ __forceinline__ void agg_store(double *agg, int64_t nn, int64_t p, const double (&o)[N]) {
    static_assert(N % 2 == 0, "aggregate records hold value pairs");
    double2 *b = reinterpret_cast<double2 *>(agg) + p;
#pragma unroll
    for (int j = 0; j < N / 2; ++j) b[(int64_t)j * nn] = make_double2(o[2 * j], o[2 * j + 1]);
}

// Adjoint of one step (frozen dt and cascade choice).  Layouts are sized for
// 3D; 2D uses the leading components of each slot.
struct AdjArgs {
    // lambda after the step (in) and before it (out), laid out like the state
    const double *lx_in, *lvh_in, *ltau_in, *lv_in, *lB_in;
    double *lx_out, *lvh_out, *ltau_out, *lv_out, *lB_out;
    double *cadj;    // [corners][CA]  update^T contributions per corner
    double *nadj;    // [nodes][NAD]   nodal-solve^T: rbar_p, Mbar_p
    double *cell;    // [cells][CL]    least-squares adjoint, W adjoint
    double *agg;     // [nodes][NAA]   aggregates of the least-squares adjoint
    double *xadj;    // [corners][3]   position adjoint per corner
    double *mu_bar;  // [cells]        accumulated adjoint of mu
    static constexpr int O_X0 = 0, O_X1 = 3, O_VH0 = 6, O_VS = 9, O_VH1 = 12, O_M = 15, O_R = 21, CA = 24;
    static constexpr int NAD = 9;
    static constexpr int O_BB = 0, O_AH = 30, O_WB = 36, CL = 46;
    static constexpr int NAA = 52;
};

template <int D> void launch_adjoint_step(const StepArgs &a, const AdjArgs &j, hipStream_t s);
template <int D>
void launch_adj_project(int64_t nn, const uint8_t *nallow, const double *allow, const double *lvh, double *out,
                        hipStream_t s);

// Work list of one stage launch.  An item is a run of at most `tile`
// consecutive entities (cells or nodes) of one mesh; the items of the largest
// mesh come first.  The launch has a multiple of 8 blocks and blocks are dealt
// to the 8 XCDs round robin: the blocks on XCD x walk the x-th eighth of the
// list in order (block slot s takes items s, s + nslot, ...), so the items one
// L2 serves are neighbours in the mesh.  With fewer blocks than items the
// blocks are persistent.
//
// Node tiles (cell items of the predictor, one item per block; all null
// otherwise): item i uses the distinct nodes tn[tn_off[i] .. tn_off[i+1]),
// ascending, at most tn_max of them; tloc[c] gives the places in that list
// of cell c's nodes, 8 bits per corner, corner k in bits 8k .. 8k+7.
struct WorkList {
    const int64_t *start;  // first entity of each item
    const int32_t *len;    // entities in each item
    int64_t n_items;
    const int32_t *tn_off, *tn;
    const uint32_t *tloc;
    int tn_max;
};

// Pairs of doubles per node in a node tile held in LDS: the aggregate values
// the least-squares sums read (count, sum y, sum y y^T, sum W, sum y W^T),
// then the node position (padded to a whole pair).
template <int D>
__host__ __device__ constexpr int tile_pairs() {
    return (Dims<D>::O_RMM + 1) / 2 + (D + 1) / 2;
}
// the most nodes a node tile may hold with blocks of `block` threads:
// 20 KB of LDS per 64 threads, so that two waves per SIMD still fit, and
// no more than an 8-bit place can name
template <int D>
__host__ __device__ constexpr int tile_max_nodes(int block) {
    return (block / 64) * 20480 / (16 * tile_pairs<D>()) < 255 ? (block / 64) * 20480 / (16 * tile_pairs<D>())
                                                                 : 255;
}
struct Sched {
    WorkList w;
    unsigned grid, block;  // grid: multiple of 8; block: multiple of 64, <= 256
    bool loop;             // false: one block per item and item <= block, so
                           // each thread has at most one entity (no loop)
};

// Rigid-plane contact (evolving boundary condition): candidate i is node
// node[i] in constraint set state[i] (0 its own walls, 1 its own walls and
// the plane), whose allowed-direction counts and bases (D x D, row-major,
// columns) are nal[set][i] and alw[set][i D D ..].  The evaluation writes
// out_s (fraction of the step at which a free candidate reaches the plane,
// 2 if it does not) and out_vn (free normal velocity of a held candidate).
struct ContactArgs {
    int64_t n;
    const int32_t *node;
    const uint8_t *state;
    const uint8_t *nal[2];
    const double *alw[2];
    uint8_t *nallow;   // the mesh's per-node constraint arrays (apply)
    double *allow;
    double xT[3], nrm[3];
    double *out_s, *out_vn;
};
void launch_contact_apply(const ContactArgs &k, int dim, hipStream_t s);
template <int D> void launch_contact_eval(const StepArgs &a, const ContactArgs &k, hipStream_t s);

// One level of conforming red refinement on the device (hl_refine.hip):
// positions [nn][D] and cells [nc][D+1] from the host, the refined mesh and
// the node pair (min << 32 | max) of every new edge-midpoint node back.
template <int D>
hipError_t refine_once(int64_t nn, int64_t nc, const double *x_host, const int32_t *cells_host, hipStream_t s,
                       std::vector<double> &x_out, std::vector<int32_t> &cells_out,
                       std::vector<uint64_t> &edges_out);

template <int D> void launch_centroids(const StepArgs &a, const Sched &k, hipStream_t s);
template <int D> void launch_node_agg(const StepArgs &a, const Sched &k, hipStream_t s);
template <int D> void launch_predict(const StepArgs &a, const Sched &k, hipStream_t s);
template <int D> void launch_node_solve(const StepArgs &a, const Sched &k, hipStream_t s);
template <int D> void launch_update(const StepArgs &a, const Sched &k, hipStream_t s);
template <int D> void launch_acoustic(const StepArgs &a, hipStream_t s);
// Diagnostics of the step just taken (a: the step's arguments, state n ->
// candidate n+1): out[0..8] = mass, mom[3], sum m e, kinetic, elastic,
// first-order and limited cell counts; out[9] = max relative GCL defect,
// out[10] = max |sqrt(det B) - J|, out[11] = cells with that >= L_c^3.
// part: [blocks][DIAG_N] partials.
constexpr int DIAG_N = 12;
template <int D>
int64_t launch_diag(const StepArgs &a, double *part, double *out, hipStream_t s);
// stress query, AoS rows in the order idx (row i = cell idx[i]; null: i)
template <int D> void launch_stress_query(const StepArgs &a, const int32_t *idx, double *out, hipStream_t s);
// One sparse MOOD pass: flagged list `fb` in, newly flagged list written to
// a.flist_out.  fixed_grid: launch shapes independent of the flag count
// (for graph capture); kernels then read every count from device memory.
// The pass clears its own lists and advances a.stamp; log (may be null):
// log[log_idx] = the input flag count.
template <int D>
void launch_mood_sparse(const StepArgs &a, const int32_t *flist, const unsigned *fcount, int64_t nflag,
                        int64_t max_deg, bool fixed_grid, unsigned *log, int log_idx, hipStream_t s);
void launch_step_begin(unsigned *counters, double *dt_cur, const double *dt_next, int n_mesh, int copy_dt,
                       hipStream_t s);

// Paired launches: the stage of a 2D context (a2, k2) and of a 3D context
// (a3, k3) as one kernel launch, each part as its own launch would run it.
// Both contexts run the base configuration (neo-Hookean law, two-level
// cascade, no boundary loads) and, where both have work, one block size.
void launch_node_agg_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, hipStream_t s);
void launch_predict_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, hipStream_t s);
void launch_node_solve_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3,
                            hipStream_t s);
void launch_update_pair(const StepArgs &a2, const Sched &k2, const StepArgs &a3, const Sched &k3, hipStream_t s);
// one sparse MOOD pass of each part (see launch_mood_sparse)
struct PairPass {
    const int32_t *flist;
    const unsigned *fcount;
    int64_t nflag, max_deg;
    unsigned *log;   // may be null
};
void launch_mood_sparse_pair(const StepArgs &a2, const PairPass &p2, const StepArgs &a3, const PairPass &p3,
                             bool fixed_grid, int log_idx, hipStream_t s);
// per-context buffers of the step's start (counters, dt, cascade levels)
// and of the CFL reduction
struct PairBook {
    unsigned *counters;
    double *dt_cur, *dt_next;
    int n_mesh;
    int copy_dt;
    uint8_t *mask;
    int64_t nc;
    const double *dtc;
    const int32_t *cell_mesh;
    const uint8_t *pstat;
    double *red, *part, *parts;
    const int64_t *mesh_cell_off;
    unsigned *bad_count;
    double c_cfl, c_v, c_i;
};
// step start: counters cleared, dt_cur = dt_next if copy_dt, mask = 0
void launch_step_begin_pair(const PairBook &b2, const PairBook &b3, hipStream_t s);
// the CFL reduction of launch_dt_reduce + launch_dt_finalize (first = 0)
void launch_dt_reduce_pair(const PairBook &b2, const PairBook &b3, hipStream_t s);
void launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);
void launch_dt_reduce(int64_t nc, const double *dtc, const int32_t *cell_mesh, const uint8_t *pstat, double *red,
                      double *part, const int64_t *mesh_cell_off, int n_mesh, unsigned *bad_count, hipStream_t s);
void launch_dt_finalize(int n_mesh, const double *red, const double *dt, const hl_params &p, int first,
                        double *dt_next, double *parts, hipStream_t s);
void launch_fill(double *p, int64_t n, double v, hipStream_t s);
// AoS [n][w] rows <-> SoA [w][n] entities; row i is entity idx[i] (idx null:
// entity i)
void launch_aos_to_soa(int64_t n, int w, const double *in, double *out, hipStream_t s, const int32_t *idx = nullptr);
// out row i = in row idx[i]
void launch_gather_rows(int64_t n, int w, const double *in, const int32_t *idx, double *out, hipStream_t s);
void launch_gather_u8(int64_t n, const uint8_t *in, const int32_t *idx, uint8_t *out, hipStream_t s);
// up to six device-to-device copies of doubles in one launch
struct CopyFields {
    const double *src[6];
    double *dst[6];
    int64_t n[6];
};
void launch_copy_fields(const CopyFields &f, hipStream_t s);
void launch_soa_to_aos(int64_t n, int w, const double *in, double *out, hipStream_t s, const int32_t *idx = nullptr);

}  // namespace hl
