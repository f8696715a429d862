// hl_api.hip -- host side of libhyperlag: the C-ABI declared in
// include/hyperlag.h (context, mesh upload, state init, step, MOOD loop,
// queries, kernel timing).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "hl_device.h"
#include "hl_kernels.h"
#include "hl_mesh.h"
#include "hyperlag.h"

namespace {

enum { PK_CENTROIDS = 0, PK_NODE_AGG, PK_PREDICT, PK_NODE_SOLVE, PK_UPDATE, PK_MOOD, PK_REDUCE, PK_COUNT };
const char *kProfNames[PK_COUNT] = {"pack", "node_agg", "predict", "node_solve", "update", "mood_sparse",
                                    "reduce"};

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> pending_kind;  // kernel kind of pending pair i
    size_t used = 0;                // pairs in use
    double total_ms[PK_COUNT] = {};
    int64_t count[PK_COUNT] = {};
};

// Launch schedule of one stage: entities per work item, threads per block,
// blocks per compute unit (0: one block per item).
struct StageCfg {
    int tile = 256, block = 256, blocks_per_cu = 0;
};
// entity kind of each stage (HL_STAGE_* order): 0 cells, 1 nodes
constexpr int kStageKind[HL_STAGE_COUNT] = {0, 1, 0, 1, 0};
struct DevList {
    int64_t *start = nullptr;
    int32_t *len = nullptr;
    int64_t n = 0;
    // node tiles of the items (predictor lists only; see hl::WorkList)
    int32_t *tn_off = nullptr, *tn = nullptr;
    uint32_t *tloc = nullptr;
    int tn_max = 0;
};

}  // namespace

struct hl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int dim = 0;
    int64_t nn = 0, nc = 0;
    int n_mesh = 1;
    // mesh
    int32_t *c2n = nullptr, *n2c_off = nullptr, *n2c = nullptr;
    uint8_t *nallow = nullptr;
    double *allow = nullptr;
    std::vector<double> x0_host, nrm_host;
    std::vector<int32_t> c2n_host;
    std::vector<uint8_t> nw_host;
    std::vector<int64_t> cell_off_host, node_off_host;
    int32_t *cell_mesh = nullptr, *node_mesh = nullptr;
    // Internal numbering: the host mesh arrays above and every device array
    // use it; everything at the boundary uses the caller's.  x_i2u[i] is the
    // caller's id of internal entity i, x_u2i the inverse (empty and null
    // when the two numberings coincide).
    int numbering = HL_NUMBERING_SPATIAL;  // for the next upload
    bool permuted = false;
    std::vector<int32_t> c_i2u, c_u2i, n_i2u, n_u2i;
    int32_t *d_c_i2u = nullptr, *d_c_u2i = nullptr, *d_n_u2i = nullptr;
    uint8_t *mask_in = nullptr;  // a replayed cascade choice, internal order
    uint64_t mesh_hash = 0;      // identifies the held mesh in state snapshots
    // material
    double *mass = nullptr, *rho0 = nullptr, *mu = nullptr, *K = nullptr;
    // state, double buffered
    double *x[2] = {}, *vhat[2] = {}, *tau[2] = {}, *v[2] = {}, *e[2] = {}, *B[2] = {};
    int cur = 0;
    // work
    double *vstar = nullptr, *xc = nullptr, *agg = nullptr, *corner = nullptr, *dtc = nullptr;
    uint8_t *mask = nullptr, *pstat = nullptr;
    int32_t *flist[2] = {}, *nlist = nullptr, *clist = nullptr, *nstamp = nullptr, *cstamp = nullptr;
    int32_t *stamp_dev = nullptr;   // device stamp of the current MOOD pass
    int64_t stamp_host = 0;         // passes since the stamps were last cleared
    unsigned *pass_log = nullptr;   // input flag count of each pass (graph mode)
    int64_t max_deg = 0;
    // captured step, one per buffer parity
    uint64_t gen = 0;     // advanced whenever captured graphs are dropped (groups re-capture then)
    bool graph_on = false;
    int graph_passes = 6;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    // continuation: CONT_PASSES more sparse MOOD passes, per buffer parity
    // and parity of the input flag list
    hipGraph_t gcont_g[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t gcont[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int64_t *mesh_cell_off = nullptr;
    double *dt_part = nullptr;
    unsigned *counters = nullptr;
    unsigned *counters_host = nullptr;  // pinned: CNT_N counters, then 128 pass-log entries
    double *dt_cur = nullptr, *dt_next = nullptr, *dt_red = nullptr, *dt_parts = nullptr;
    double *diag_part = nullptr, *diag_out = nullptr;
    double *scratch = nullptr;
    size_t scratch_bytes = 0;
    bool have_mesh = false, have_state = false;
    bool rec_valid = false;  // gather records hold the current state
    hl_params prm{};
    std::vector<void *> allocs;
    Prof prof;
    // stage schedules and their work lists (device memory in allocs)
    int n_cu = 0;
    // default schedules (the autotuner's choice on the 8.1M-tet bar): pack,
    // predict and update one 256-cell item per block (the predictor's node
    // tile, about 130 nodes of the bar, and then its corner records in the
    // same 80 KB of LDS); the node stages (AGG_G lanes per node) one pass of
    // 64 (aggregates) or 32 (solve) nodes per 256-thread block, which keeps
    // each XCD's nodes in flight, and the cell records they share, in its L2
    // A predictor schedule the caller has not set follows the mesh
    // (predict_default): 256-cell items while they still give 8 blocks per
    // CU, else 128 or 64 (a small mesh would leave CUs idle).
    StageCfg cfg[HL_STAGE_COUNT] = {{256, 256, 0}, {64, 256, 0}, {256, 256, 0}, {32, 256, 0}, {256, 256, 0}};
    bool cfg_set[HL_STAGE_COUNT] = {};  // set by hl_set_schedule or hl_autotune
    hl::Sched sk[HL_STAGE_COUNT] = {};
    bool sched_ready = false;
    // (entity kind, tile, most nodes per node tile or 0) -> list
    std::map<std::tuple<int, int, int>, DevList> wlists;
    // boundary loads grouped by node (own allocations, freed with the mesh)
    struct {
        int64_t n = 0;  // loads set by the caller
        int32_t *off = nullptr, *cell = nullptr;
        uint8_t *fk = nullptr;
        double *val = nullptr;
        std::vector<void *> mem;
    } ld;
    // rigid-plane contact (own allocations, freed with the mesh)
    struct {
        int64_t n = 0;
        int32_t *node = nullptr;
        uint8_t *state = nullptr;           // device copy of state_h
        uint8_t *nal[2] = {nullptr, nullptr};
        double *alw[2] = {nullptr, nullptr};
        double *out = nullptr;              // [2n]: s, then vn
        std::vector<uint8_t> state_h;
        double xT[3] = {0, 0, 0}, nrm[3] = {0, 0, 0};
        std::vector<void *> mem;
    } ct;
    // statistics of the last step's MOOD loop
    int64_t last_first = 0;
    int last_iters = 0;
    unsigned last_inadm = 0;
    int64_t last_recomp = 0;
    // adjoint tapes (own allocations, freed with the mesh)
    struct {
        int nsteps = 0, every = 0, nckpt = 0;
        size_t state_sz = 0;  // doubles per state snapshot
        double *ckpt = nullptr, *seg = nullptr, *dts = nullptr;
        uint8_t *masks = nullptr;
        double *lam[2] = {nullptr, nullptr};
        double *cadj = nullptr, *nadj = nullptr, *cell = nullptr, *agg = nullptr, *xadj = nullptr;
        double *mu_bar = nullptr, *out = nullptr;
        double *dtn = nullptr;  // dt_next after the last recorded step [n_mesh]
        // forward intermediates of the steps of one segment (node
        // aggregates, corner records, v*), inter_sz doubles per step, kept
        // by the segment's replay for its reverse steps; null when they do
        // not fit the budget (the reverse steps then recompute them)
        double *inter = nullptr;
        size_t inter_sz = 0;
        std::vector<void *> mem;
    } tape;
};

namespace {

// text of the last failed HIP call, for hl_last_error()
thread_local char g_last_error[256] = "";

hl_status hip_fail(hipError_t e, const char *what, int line) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s (line %d): %s", what, line, hipGetErrorString(e));
    return HL_E_HIP;
}

#define HIPCHK(call)                                               \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return hip_fail(_e, #call, __LINE__); \
    } while (0)

hl_params default_params(int dim) {
    hl_params p;
    p.c_cfl = dim == 2 ? 0.4 : 0.25;
    p.c_v = 0.2;
    p.c_i = 0.1;
    p.delta0 = 1e-4;
    p.delta1 = 1e-3;
    p.eps_tol = 1e-12;
    p.detect = 1;
    p.cascade = 2;
    p.shear_a = -1.0;
    p.eos = 0;
    p.reserved = 0;
    p.sg_gamma = 2.2;
    p.sg_pinf = 1e6;
    return p;
}

bool params_valid(const hl_params &p) {
    const bool sg_ok = p.eos == 0 || (p.eos == 1 && p.sg_gamma > 1.0 && std::isfinite(p.sg_gamma) &&
                                      p.sg_pinf >= 0.0 && std::isfinite(p.sg_pinf) && p.cascade != 3);
    return p.c_cfl > 0 && p.c_v > 0 && p.c_i >= 0 && p.delta0 >= 0 && p.delta1 >= 0 && p.eps_tol >= 0 &&
           (p.cascade == 0 || p.cascade == 2 || p.cascade == 3) && p.shear_a >= -1.0 && p.shear_a <= 0.5 && sg_ok;
}

void drop_graphs(hl_ctx *c) {
    ++c->gen;
    for (int b = 0; b < 2; ++b) {
        if (c->gexec[b]) (void)hipGraphExecDestroy(c->gexec[b]);
        for (int f = 0; f < 2; ++f) {
            if (c->gcont[b][f]) (void)hipGraphExecDestroy(c->gcont[b][f]);
            if (c->gcont_g[b][f]) (void)hipGraphDestroy(c->gcont_g[b][f]);
            c->gcont[b][f] = nullptr;
            c->gcont_g[b][f] = nullptr;
        }
        if (c->graph[b]) (void)hipGraphDestroy(c->graph[b]);
        c->gexec[b] = nullptr;
        c->graph[b] = nullptr;
    }
}

void free_tape(hl_ctx *c) {
    for (void *p : c->tape.mem) (void)hipFree(p);
    c->tape.mem.clear();
    c->tape.nsteps = c->tape.every = c->tape.nckpt = 0;
    c->tape.ckpt = c->tape.seg = c->tape.dts = nullptr;
    c->tape.masks = nullptr;
    c->tape.lam[0] = c->tape.lam[1] = nullptr;
    c->tape.cadj = c->tape.nadj = c->tape.cell = c->tape.agg = c->tape.xadj = c->tape.mu_bar = c->tape.out = nullptr;
    c->tape.dtn = nullptr;
    c->tape.inter = nullptr;
    c->tape.inter_sz = 0;
}

void free_loads(hl_ctx *c) {
    for (void *p : c->ld.mem) (void)hipFree(p);
    c->ld.mem.clear();
    c->ld.n = 0;
    c->ld.off = c->ld.cell = nullptr;
    c->ld.fk = nullptr;
    c->ld.val = nullptr;
}

void free_contact(hl_ctx *c) {
    for (void *p : c->ct.mem) (void)hipFree(p);
    c->ct.mem.clear();
    c->ct.n = 0;
    c->ct.node = nullptr;
    c->ct.state = nullptr;
    c->ct.nal[0] = c->ct.nal[1] = nullptr;
    c->ct.alw[0] = c->ct.alw[1] = nullptr;
    c->ct.out = nullptr;
    c->ct.state_h.clear();
}

void free_all(hl_ctx *c) {
    drop_graphs(c);
    free_tape(c);
    free_loads(c);
    free_contact(c);
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->counters_host) (void)hipHostFree(c->counters_host);
    c->counters_host = nullptr;
    c->c2n = c->n2c_off = c->n2c = nullptr;
    c->nallow = nullptr;
    c->allow = c->mass = c->rho0 = c->mu = c->K = nullptr;
    for (int b = 0; b < 2; ++b) c->x[b] = c->vhat[b] = c->tau[b] = c->v[b] = c->e[b] = c->B[b] = nullptr;
    c->vstar = c->xc = c->agg = c->corner = c->dtc = nullptr;
    c->mask = c->pstat = nullptr;
    c->flist[0] = c->flist[1] = c->nlist = c->clist = c->nstamp = c->cstamp = nullptr;
    c->mesh_cell_off = nullptr;
    c->cell_mesh = c->node_mesh = nullptr;
    c->permuted = false;
    c->c_i2u.clear();
    c->c_u2i.clear();
    c->n_i2u.clear();
    c->n_u2i.clear();
    c->d_c_i2u = c->d_c_u2i = c->d_n_u2i = nullptr;
    c->mask_in = nullptr;
    c->mesh_hash = 0;
    c->dt_part = nullptr;
    c->stamp_dev = nullptr;
    c->pass_log = nullptr;
    c->stamp_host = 0;
    c->counters = nullptr;
    c->dt_cur = c->dt_next = c->dt_red = c->dt_parts = c->diag_part = c->diag_out = c->scratch = nullptr;
    c->have_mesh = c->have_state = false;
    c->rec_valid = false;
    c->wlists.clear();
    c->sched_ready = false;
}

template <class T>
hl_status dalloc(hl_ctx *c, T **p, size_t n) {
    void *q = nullptr;
    size_t bytes = std::max<size_t>(n * sizeof(T), 256);
    if (hipMalloc(&q, bytes) != hipSuccess) return HL_E_OOM;
    c->allocs.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return HL_OK;
}

// Work list of entity kind `kind` cut into items of at most `tile`
// entities, items of the largest mesh first (ties in mesh order).  Node
// items of a mesh go in the order of the first cell that uses their first
// node: the node numbering of a generated grid already follows its cells,
// while after a refinement the edge midpoints (numbered after the old
// nodes) are interleaved with the old nodes around them, so the cells
// both gather are fetched once.
//
// With tile_nodes > 0 (cell lists of the one-item predictor) every item also
// gets its node tile: its cells' distinct nodes, ascending, and for each
// cell the places of its nodes in that list.  An item with more than
// tile_nodes distinct nodes is cut in halves until each part fits.
hl_status work_list(hl_ctx *c, int kind, int tile, int tile_nodes, DevList *out) {
    const auto key = std::make_tuple(kind, tile, tile_nodes);
    auto it = c->wlists.find(key);
    if (it != c->wlists.end()) {
        *out = it->second;
        return HL_OK;
    }
    const std::vector<int64_t> &off = kind == 0 ? c->cell_off_host : c->node_off_host;
    std::vector<int> order((size_t)c->n_mesh);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
    std::vector<int64_t> first_use;
    if (kind == 1) {
        const int nv = c->dim + 1;
        first_use.assign((size_t)c->nn, INT64_MAX);
        for (int64_t q = 0; q < c->nc * nv; ++q) {
            int64_t &f = first_use[(size_t)c->c2n_host[(size_t)q]];
            f = std::min<int64_t>(f, q / nv);
        }
    }
    std::vector<int64_t> st;
    std::vector<int32_t> ln;
    std::vector<std::pair<int64_t, int64_t>> items;  // (key, start)
    for (int m : order) {
        items.clear();
        for (int64_t b = off[m]; b < off[m + 1]; b += tile) items.emplace_back(kind == 1 ? first_use[b] : b, b);
        if (kind == 1) std::stable_sort(items.begin(), items.end(), [](const auto &x, const auto &y) {
            return x.first < y.first;
        });
        for (const auto &t : items) {
            st.push_back(t.second);
            ln.push_back((int32_t)std::min<int64_t>(tile, off[m + 1] - t.second));
        }
    }
    std::vector<int32_t> tn_off, tn;
    std::vector<uint32_t> tloc;
    if (tile_nodes > 0 && kind == 0) {
        const int nv = c->dim + 1;
        std::vector<int64_t> st2;
        std::vector<int32_t> ln2;
        std::vector<int32_t> u;
        tn_off.push_back(0);
        tloc.assign((size_t)c->nc, 0u);
        // items still to place, last first
        std::vector<std::pair<int64_t, int32_t>> todo;
        for (size_t i = 0; i < st.size(); ++i) {
            todo.assign(1, {st[i], ln[i]});
            while (!todo.empty()) {
                const auto [s0, n0] = todo.back();
                todo.pop_back();
                u.assign(c->c2n_host.begin() + s0 * nv, c->c2n_host.begin() + (s0 + n0) * nv);
                std::sort(u.begin(), u.end());
                u.erase(std::unique(u.begin(), u.end()), u.end());
                if ((int)u.size() > tile_nodes) {
                    todo.push_back({s0 + n0 / 2, n0 - n0 / 2});
                    todo.push_back({s0, n0 / 2});
                    continue;
                }
                if ((int64_t)tn.size() + (int64_t)u.size() > INT32_MAX) return HL_E_INVALID;
                for (int64_t cc = s0; cc < s0 + n0; ++cc) {
                    uint32_t w = 0;
                    for (int k = 0; k < nv; ++k) {
                        const int32_t p = c->c2n_host[(size_t)(cc * nv + k)];
                        w |= (uint32_t)(std::lower_bound(u.begin(), u.end(), p) - u.begin()) << (8 * k);
                    }
                    tloc[(size_t)cc] = w;
                }
                tn.insert(tn.end(), u.begin(), u.end());
                tn_off.push_back((int32_t)tn.size());
                st2.push_back(s0);
                ln2.push_back(n0);
            }
        }
        st.swap(st2);
        ln.swap(ln2);
    }
    DevList d;
    d.n = (int64_t)st.size();
    hl_status r;
    if ((r = dalloc(c, &d.start, st.size())) != HL_OK) return r;
    if ((r = dalloc(c, &d.len, ln.size())) != HL_OK) return r;
    if (d.n) {
        HIPCHK(hipMemcpy(d.start, st.data(), sizeof(int64_t) * st.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d.len, ln.data(), sizeof(int32_t) * ln.size(), hipMemcpyHostToDevice));
    }
    if (!tn_off.empty()) {
        if ((r = dalloc(c, &d.tn_off, tn_off.size())) != HL_OK) return r;
        if ((r = dalloc(c, &d.tn, tn.size())) != HL_OK) return r;
        if ((r = dalloc(c, &d.tloc, tloc.size())) != HL_OK) return r;
        HIPCHK(hipMemcpy(d.tn_off, tn_off.data(), sizeof(int32_t) * tn_off.size(), hipMemcpyHostToDevice));
        if (!tn.empty()) HIPCHK(hipMemcpy(d.tn, tn.data(), sizeof(int32_t) * tn.size(), hipMemcpyHostToDevice));
        if (!tloc.empty())
            HIPCHK(hipMemcpy(d.tloc, tloc.data(), sizeof(uint32_t) * tloc.size(), hipMemcpyHostToDevice));
        d.tn_max = tile_nodes;
    }
    c->wlists.emplace(key, d);
    *out = d;
    return HL_OK;
}

hl_status build_sched(hl_ctx *c, int stage, const StageCfg &g, hl::Sched *k) {
    DevList d;
    // the one-item predictor reads node values from node tiles
    const bool one_item = g.blocks_per_cu == 0 && g.tile <= g.block;
    const int tn = stage == HL_STAGE_PREDICT && one_item
                       ? (c->dim == 3 ? hl::tile_max_nodes<3>(g.block) : hl::tile_max_nodes<2>(g.block))
                       : 0;
    hl_status r = work_list(c, kStageKind[stage], g.tile, tn, &d);
    if (r != HL_OK) return r;
    k->w.start = d.start;
    k->w.len = d.len;
    k->w.n_items = d.n;
    k->w.tn_off = d.tn_off;
    k->w.tn = d.tn;
    k->w.tloc = d.tloc;
    k->w.tn_max = d.tn_max;
    int64_t grid = (d.n + 7) / 8 * 8;
    if (g.blocks_per_cu > 0) grid = std::min<int64_t>(grid, ((int64_t)g.blocks_per_cu * c->n_cu + 7) / 8 * 8);
    k->grid = (unsigned)std::max<int64_t>(8, grid);
    k->block = (unsigned)g.block;
    k->loop = g.blocks_per_cu > 0 || g.tile > g.block;
    return HL_OK;
}

// Device work lists are built before any launch that may be captured.
// The predictor's default schedule for the uploaded meshes (and those of
// `peer`, the other context of a group, whose launches are shared): one
// item of T cells per T-thread block with T the largest of 256, 128, 64
// whose items number at least 8 per CU (node tiles of 256 cells hold about
// 130 nodes against about 48 for 64 cells, but a launch of few large blocks
// leaves CUs idle at its end).
StageCfg predict_default(const hl_ctx *c, const hl_ctx *peer = nullptr) {
    for (int t : {256, 128}) {
        int64_t items = 0;
        for (const hl_ctx *x : {c, peer})
            if (x)
                for (size_t m = 0; m + 1 < x->cell_off_host.size(); ++m)
                    items += (x->cell_off_host[m + 1] - x->cell_off_host[m] + t - 1) / t;
        if (items >= 8 * (int64_t)c->n_cu) return StageCfg{t, t, 0};
    }
    return StageCfg{64, 64, 0};
}

hl_status ensure_scheds(hl_ctx *c, const hl_ctx *peer = nullptr) {
    if (!c->cfg_set[HL_STAGE_PREDICT]) {
        const StageCfg want = predict_default(c, peer);
        StageCfg &have = c->cfg[HL_STAGE_PREDICT];
        if (want.tile != have.tile || want.block != have.block || want.blocks_per_cu != have.blocks_per_cu) {
            have = want;
            if (c->sched_ready) {
                c->sched_ready = false;
                drop_graphs(c);
            }
        }
    }
    if (c->sched_ready) return HL_OK;
    for (int st = 0; st < HL_STAGE_COUNT; ++st) {
        hl_status r = build_sched(c, st, c->cfg[st], &c->sk[st]);
        if (r != HL_OK) return r;
    }
    c->sched_ready = true;
    return HL_OK;
}

bool cfg_valid(const StageCfg &g) {
    return g.tile >= 1 && g.tile <= (1 << 20) && g.block >= 64 && g.block <= 256 && g.block % 64 == 0 &&
           g.blocks_per_cu >= 0 && g.blocks_per_cu <= 64;
}

// bring a borrowed input array to the host
template <class T>
hl_status to_host(const T *src, size_t n, int on_device, std::vector<T> &dst) {
    dst.resize(n);
    if (n == 0) return HL_OK;
    if (!src) return HL_E_INVALID;
    if (on_device) {
        if (hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) return HL_E_HIP;
    } else {
        std::memcpy(dst.data(), src, n * sizeof(T));
    }
    return HL_OK;
}

// signed simplex measure with the same edge formulas as the device code
double host_volume(int d, const double *X /* (d+1) x d */) {
    if (d == 3) {
        double e1[3], e2[3], e3[3];
        for (int i = 0; i < 3; ++i) {
            e1[i] = X[3 + i] - X[i];
            e2[i] = X[6 + i] - X[i];
            e3[i] = X[9 + i] - X[i];
        }
        const double s = 1.0 / 6.0;
        double c0 = s * (e2[1] * e3[2] - e2[2] * e3[1]);
        double c1 = s * (e2[2] * e3[0] - e2[0] * e3[2]);
        double c2 = s * (e2[0] * e3[1] - e2[1] * e3[0]);
        return e1[0] * c0 + e1[1] * c1 + e1[2] * c2;
    }
    double e1x = X[2] - X[0], e1y = X[3] - X[1];
    double e2x = X[4] - X[0], e2y = X[5] - X[1];
    return e1x * (0.5 * e2y) + e1y * (-0.5 * e2x);
}

// Orthonormal basis of the directions a node with `nw` unit wall normals
// may move in (slip walls, Appendix B).  Returns the number of columns;
// P[i*d + t] is component i of column t.
int wall_basis(int d, int nw, const double *nrm, double *P) {
    for (int i = 0; i < d * d; ++i) P[i] = 0.0;
    // orthonormalise the normals
    double Q[3][3];
    int nq = 0;
    for (int r = 0; r < nw && r < d; ++r) {
        double w[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) w[i] = nrm[r * d + i];
        for (int q = 0; q < nq; ++q) {
            double s = 0;
            for (int i = 0; i < 3; ++i) s += w[i] * Q[q][i];
            for (int i = 0; i < 3; ++i) w[i] -= s * Q[q][i];
        }
        double n = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (n < 1e-8) continue;
        for (int i = 0; i < 3; ++i) Q[nq][i] = w[i] / n;
        ++nq;
    }
    if (nq == 0) {
        for (int i = 0; i < d; ++i) P[i * d + i] = 1.0;
        return d;
    }
    if (nq >= d) return 0;
    if (d == 2) {  // tangent of the one wall
        P[0 * 2 + 0] = -Q[0][1];
        P[1 * 2 + 0] = Q[0][0];
        return 1;
    }
    if (nq == 2) {  // 3D: line along n1 x n2
        double t[3] = {Q[0][1] * Q[1][2] - Q[0][2] * Q[1][1], Q[0][2] * Q[1][0] - Q[0][0] * Q[1][2],
                       Q[0][0] * Q[1][1] - Q[0][1] * Q[1][0]};
        double n = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        for (int i = 0; i < 3; ++i) P[i * 3 + 0] = t[i] / n;
        return 1;
    }
    // 3D, one wall: t1 = n x a (a = axis least aligned with n), t2 = n x t1
    const double *n = Q[0];
    int ax = 0;
    for (int i = 1; i < 3; ++i)
        if (std::fabs(n[i]) < std::fabs(n[ax])) ax = i;
    double a[3] = {0, 0, 0};
    a[ax] = 1.0;
    double t1[3] = {n[1] * a[2] - n[2] * a[1], n[2] * a[0] - n[0] * a[2], n[0] * a[1] - n[1] * a[0]};
    double l = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int i = 0; i < 3; ++i) t1[i] /= l;
    double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    for (int i = 0; i < 3; ++i) {
        P[i * 3 + 0] = t1[i];
        P[i * 3 + 1] = t2[i];
    }
    return 2;
}

hl::StepArgs make_args(hl_ctx *c, int src) {
    hl::StepArgs a{};
    int dst = 1 - src;
    a.nc = c->nc;
    a.nn = c->nn;
    a.c2n = c->c2n;
    a.n2c_off = c->n2c_off;
    a.n2c = c->n2c;
    a.nallow = c->nallow;
    a.allow = c->allow;
    a.mass = c->mass;
    a.rho0 = c->rho0;
    a.mu = c->mu;
    a.K = c->K;
    a.cell_mesh = c->cell_mesh;
    a.node_mesh = c->node_mesh;
    a.dt = c->dt_cur;
    a.x = c->x[src];
    a.vhat = c->vhat[src];
    a.tau = c->tau[src];
    a.v = c->v[src];
    a.e = c->e[src];
    a.B = c->B[src];
    a.x1 = c->x[dst];
    a.vhat1 = c->vhat[dst];
    a.tau1 = c->tau[dst];
    a.v1 = c->v[dst];
    a.e1 = c->e[dst];
    a.B1 = c->B[dst];
    a.vstar = c->vstar;
    a.xc = c->xc;
    a.agg = c->agg;
    a.corner = c->corner;
    a.dtc = c->dtc;
    a.mask = c->mask;
    a.pstat = c->pstat;
    a.flist_out = c->flist[0];
    a.fcount_out = c->counters + hl::CNT_F0;
    a.nlist = c->nlist;
    a.clist = c->clist;
    a.nstamp = c->nstamp;
    a.cstamp = c->cstamp;
    a.stamp = c->stamp_dev;
    a.counters = c->counters;
    a.delta0 = c->prm.delta0;
    a.delta1 = c->prm.delta1;
    a.eps_tol = c->prm.eps_tol;
    a.detect = c->prm.detect;
    a.cascade = c->prm.cascade == 3 ? 3 : 2;
    a.shear_a = c->prm.shear_a;
    a.eos = c->prm.eos;
    a.sg_gamma = c->prm.sg_gamma;
    a.sg_pinf = c->prm.sg_pinf;
    a.limited = a.cascade == 3 ? 1 : 0;
    a.ld_off = c->ld.off;
    a.ld_cell = c->ld.cell;
    a.ld_fk = c->ld.fk;
    a.ld_val = c->ld.val;
    return a;
}

// ------------------------------------------------------------ profiling
void prof_begin(hl_ctx *c, int kind, size_t *slot) {
    if (!c->prof.on) return;
    Prof &P = c->prof;
    if (2 * (P.used + 1) > P.pool.size()) {
        size_t grow = std::max<size_t>(256, P.pool.size());
        for (size_t i = 0; i < grow; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            P.pool.push_back(e);
        }
    }
    *slot = P.used++;
    P.pending_kind.resize(P.used);
    P.pending_kind[*slot] = kind;
    (void)hipEventRecord(P.pool[2 * *slot], c->stream);
}

void prof_end(hl_ctx *c, size_t slot) {
    if (!c->prof.on) return;
    (void)hipEventRecord(c->prof.pool[2 * slot + 1], c->stream);
}

void prof_collect(hl_ctx *c) {
    Prof &P = c->prof;
    if (P.used == 0) return;
    (void)hipStreamSynchronize(c->stream);
    for (size_t i = 0; i < P.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, P.pool[2 * i], P.pool[2 * i + 1]) == hipSuccess) {
            P.total_ms[P.pending_kind[i]] += ms;
            P.count[P.pending_kind[i]] += 1;
        }
    }
    P.used = 0;
}

#define PROF(c, kind, stmt)          \
    do {                             \
        size_t _slot = 0;            \
        prof_begin((c), (kind), &_slot); \
        stmt;                        \
        prof_end((c), _slot);        \
    } while (0)

template <int D>
void enqueue_first(hl_ctx *c, hl::StepArgs &a, bool copy_dt, bool clear_mask, hipStream_t s) {
    hl::launch_step_begin(c->counters, c->dt_cur, c->dt_next, c->n_mesh, copy_dt ? 1 : 0, s);
    if (clear_mask) hl::launch_fill_u8(c->mask, c->nc, 0, s);
    a.flist_out = c->flist[0];
    a.fcount_out = c->counters + hl::CNT_F0;
    PROF(c, PK_NODE_AGG, hl::launch_node_agg<D>(a, c->sk[HL_STAGE_NODE_AGG], s));
    PROF(c, PK_PREDICT, hl::launch_predict<D>(a, c->sk[HL_STAGE_PREDICT], s));
    PROF(c, PK_NODE_SOLVE, hl::launch_node_solve<D>(a, c->sk[HL_STAGE_NODE_SOLVE], s));
    PROF(c, PK_UPDATE, hl::launch_update<D>(a, c->sk[HL_STAGE_UPDATE], s));
}

// MOOD pass reading flag list fb: the flagged cells drop to first order and
// only their corners, their nodes and the cells around those nodes change.
template <int D>
void enqueue_pass(hl_ctx *c, hl::StepArgs a, int fb, int log_index, int64_t nflag, bool fixed, hipStream_t s) {
    const int nb = 1 - fb;
    a.flist_out = c->flist[nb];
    a.fcount_out = c->counters + hl::CNT_F0 + nb;
    PROF(c, PK_MOOD,
         hl::launch_mood_sparse<D>(a, c->flist[fb], c->counters + hl::CNT_F0 + fb, nflag, c->max_deg, fixed,
                                   log_index >= 0 ? c->pass_log : nullptr, log_index >= 0 ? log_index : 0, s));
}

void enqueue_reduce(hl_ctx *c, hipStream_t s) {
    PROF(c, PK_REDUCE, {
        hl::launch_dt_reduce(c->nc, c->dtc, c->cell_mesh, c->pstat, c->dt_red, c->dt_part, c->mesh_cell_off,
                             c->n_mesh, c->counters + hl::CNT_BAD, s);
        hl::launch_dt_finalize(c->n_mesh, c->dt_red, c->dt_cur, c->prm, 0, c->dt_next, c->dt_parts, s);
    });
}

hl_status read_counters(hl_ctx *c, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(c->counters_host, c->counters, hl::CNT_N * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HL_OK;
}

template <int D>
hl_status capture_step(hl_ctx *c, int src) {
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = c->cap_stream;
    hl::StepArgs a = make_args(c, src);
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    enqueue_first<D>(c, a, true, true, cs);
    for (int p = 0; p < c->graph_passes; ++p) enqueue_pass<D>(c, a, p & 1, p, 0, true, cs);
    enqueue_reduce(c, cs);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(cs, &g));
    c->graph[src] = g;
    HIPCHK(hipGraphInstantiate(&c->gexec[src], g, nullptr, nullptr, 0));
    return HL_OK;
}

template <int D>
hl_status fill_info(hl_ctx *c, int src, hl_step_info *info);

// Passes per continuation graph (even, so the input list parity returns).
constexpr int CONT_PASSES = 8;

template <int D>
hl_status capture_cont(hl_ctx *c, int src, int fb) {
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = c->cap_stream;
    hl::StepArgs a = make_args(c, src);
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int p = 0; p < CONT_PASSES; ++p) enqueue_pass<D>(c, a, fb ^ (p & 1), 64 + p, 0, true, cs);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(cs, &g));
    c->gcont_g[src][fb] = g;
    HIPCHK(hipGraphInstantiate(&c->gcont[src][fb], g, nullptr, nullptr, 0));
    return HL_OK;
}

// quick: a replay for the reverse sweep (no MOOD, no report): the step is
// enqueued without waiting for its counters.
template <int D>
hl_status run_step(hl_ctx *c, double dt, const uint8_t *replay_mask, int mask_on_device, hl_step_info *info,
                   bool quick = false, bool reduce = true, double *const *inter = nullptr) {
    hipStream_t s = c->stream;
    const int src = c->cur;
    hl::StepArgs a = make_args(c, src);
    if (quick && inter) {
        // the adjoint's replay writes the step's node aggregates, corner
        // records and v* straight into its tape slot
        a.agg = inter[0];
        a.corner = inter[1];
        a.vstar = inter[2];
    }
    if (c->nc == 0) {
        // nothing moves: copy the node state through
        HIPCHK(hipMemcpyAsync(c->x[1 - src], c->x[src], sizeof(double) * c->nn * D, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(c->vhat[1 - src], c->vhat[src], sizeof(double) * c->nn * D, hipMemcpyDeviceToDevice, s));
        if (c->nn) HIPCHK(hipMemsetAsync(c->vstar, 0, sizeof(double) * c->nn * D, s));
        HIPCHK(hipStreamSynchronize(s));
        c->cur = 1 - src;
        if (info) std::memset(info, 0, sizeof(*info));
        return HL_OK;
    }
    // stamps are 32-bit: clear them long before they could wrap
    if (c->stamp_host > INT32_MAX - 4096) {
        HIPCHK(hipMemsetAsync(c->nstamp, 0, sizeof(int32_t) * c->nn, s));
        HIPCHK(hipMemsetAsync(c->cstamp, 0, sizeof(int32_t) * c->nc, s));
        HIPCHK(hipMemsetAsync(c->stamp_dev, 0, sizeof(int32_t), s));
        c->stamp_host = 0;
    }
    if (replay_mask) {
        HIPCHK(hipMemcpyAsync(c->mask, replay_mask, (size_t)c->nc,
                              mask_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        a.detect = 0;
        // a caller's levels may include the limited one; the adjoint's
        // replays (quick) repeat recorded two-level choices (levels 0 and 2)
        a.limited = quick && c->prm.cascade != 3 ? 0 : 2;
    }
    {
        hl_status st = ensure_scheds(c);
        if (st != HL_OK) return st;
    }
    const bool graph = c->graph_on && !replay_mask && !c->prof.on;
    // the update kernel leaves the gather records of the state it writes;
    // after an upload they are rebuilt here
    if (!c->rec_valid) {
        PROF(c, PK_CENTROIDS, hl::launch_centroids<D>(a, c->sk[HL_STAGE_PACK], s));
        c->rec_valid = true;
    }
    int iters = 1;
    int64_t first = 0, nflag = 0;
    int fb = 0, pass = 0;
    if (graph) {
        if (dt > 0.0) hl::launch_fill(c->dt_next, c->n_mesh, dt, s);
        if (!c->gexec[src]) {
            hl_status st = capture_step<D>(c, src);
            if (st != HL_OK) return st;
        }
        HIPCHK(hipGraphLaunch(c->gexec[src], s));
        c->stamp_host += c->graph_passes;
        // pass log and counters land in pinned memory: one wait for both
        unsigned *log = c->counters_host + hl::CNT_N;
        const int np = std::min(c->graph_passes, 64);
        if (np) HIPCHK(hipMemcpyAsync(log, c->pass_log, sizeof(unsigned) * np, hipMemcpyDeviceToHost, s));
        hl_status st = read_counters(c, s);
        if (st != HL_OK) return st;
        pass = c->graph_passes;
        fb = pass & 1;  // list written by the last pass
        nflag = c->counters_host[hl::CNT_F0 + fb];
        first = np ? log[0] : nflag;
        for (int p = 0; p < np; ++p) iters += log[p] > 0;
        if (a.detect && nflag > 0) {
            // the captured passes did not reach the fixpoint: one more pass
            // eagerly, then captured blocks of CONT_PASSES passes (a pass
            // with no input exits at once) until no cell is flagged
            enqueue_pass<D>(c, a, fb, -1, nflag, false, s);
            c->stamp_host++;
            ++iters;
            ++pass;
            if ((st = read_counters(c, s)) != HL_OK) return st;
            fb = 1 - fb;
            nflag = c->counters_host[hl::CNT_F0 + fb];
            while (nflag > 0) {
                if (!c->gcont[src][fb] && (st = capture_cont<D>(c, src, fb)) != HL_OK) return st;
                HIPCHK(hipGraphLaunch(c->gcont[src][fb], s));
                c->stamp_host += CONT_PASSES;
                unsigned *clog = c->counters_host + hl::CNT_N + 64;
                HIPCHK(hipMemcpyAsync(clog, c->pass_log + 64, sizeof(unsigned) * CONT_PASSES, hipMemcpyDeviceToHost,
                                      s));
                if ((st = read_counters(c, s)) != HL_OK) return st;
                for (int p = 0; p < CONT_PASSES; ++p) iters += clog[p] > 0;
                pass += CONT_PASSES;
                nflag = c->counters_host[hl::CNT_F0 + fb];
            }
            enqueue_reduce(c, s);
            if ((st = read_counters(c, s)) != HL_OK) return st;
        }
    } else if (quick && replay_mask && !info) {
        if (dt > 0.0) hl::launch_fill(c->dt_cur, c->n_mesh, dt, s);
        enqueue_first<D>(c, a, !(dt > 0.0), false, s);
        // the next dt: not wanted when the caller sets it from a record
        if (reduce) enqueue_reduce(c, s);
        c->last_first = 0;
        c->last_iters = 1;
        c->last_inadm = 0;
        c->last_recomp = 0;
        c->cur = 1 - src;
        return HL_OK;
    } else {
        if (dt > 0.0) hl::launch_fill(c->dt_cur, c->n_mesh, dt, s);
        enqueue_first<D>(c, a, !(dt > 0.0), !replay_mask, s);
        hl_status st = read_counters(c, s);
        if (st != HL_OK) return st;
        nflag = c->counters_host[hl::CNT_F0];
        first = nflag;
        while (a.detect && nflag > 0) {
            enqueue_pass<D>(c, a, fb, -1, nflag, false, s);
            c->stamp_host++;
            ++iters;
            ++pass;
            if ((st = read_counters(c, s)) != HL_OK) return st;
            fb = 1 - fb;
            nflag = c->counters_host[hl::CNT_F0 + fb];
        }
        enqueue_reduce(c, s);
        if ((st = read_counters(c, s)) != HL_OK) return st;
    }
    const unsigned inadm = c->counters_host[hl::CNT_BAD];
    c->last_first = first;
    c->last_iters = iters;
    c->last_inadm = inadm;
    c->last_recomp = c->counters_host[hl::CNT_RECOMP];
    c->cur = 1 - src;
    if (info) {
        hl_status st = fill_info<D>(c, src, info);
        if (st != HL_OK) return st;
    }
    return inadm ? HL_WARN_PARACHUTE_INADMISSIBLE : HL_OK;
}

// Step report of the step just taken from buffer src (statistics of its
// MOOD loop from the context).
template <int D>
hl_status fill_info(hl_ctx *c, int src, hl_step_info *info) {
    hipStream_t s = c->stream;
    hl::StepArgs a = make_args(c, src);
    {
        std::memset(info, 0, sizeof(*info));
        hl::launch_diag<D>(a, c->diag_part, c->diag_out, s);
        double d[hl::DIAG_N], dts[4];
        HIPCHK(hipMemcpyAsync(d, c->diag_out, sizeof d, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&dts[0], c->dt_cur, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&dts[1], c->dt_next, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&dts[2], c->dt_parts, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        info->dt_used = dts[0];
        info->dt_next = dts[1];
        info->dt_acoustic = dts[2];
        info->dt_volume = dts[3];
        info->mass = d[0];
        info->mom[0] = d[1];
        info->mom[1] = d[2];
        info->mom[2] = d[3];
        info->energy = d[4];
        info->kinetic = d[5];
        info->elastic = d[6];
        info->n_p0 = (int64_t)llround(d[7]);
        info->n_limited = (int64_t)llround(d[8]);
        info->gcl_defect = d[9];
        info->detB_defect = d[10];
        info->n_detB = (int64_t)llround(d[11]);
        info->n_recomputed = c->last_recomp;
        info->n_flag_first = c->last_first;
        info->mood_iters = c->last_iters;
        info->status = c->last_inadm ? 1 : 0;
        info->trials = 1;
        for (uint8_t v : c->ct.state_h) info->n_contact += v;
    }
    return HL_OK;
}

hl::ContactArgs contact_args(hl_ctx *c) {
    hl::ContactArgs k{};
    k.n = c->ct.n;
    k.node = c->ct.node;
    k.state = c->ct.state;
    k.nal[0] = c->ct.nal[0];
    k.nal[1] = c->ct.nal[1];
    k.alw[0] = c->ct.alw[0];
    k.alw[1] = c->ct.alw[1];
    k.nallow = c->nallow;
    k.allow = c->allow;
    for (int i = 0; i < 3; ++i) {
        k.xT[i] = c->ct.xT[i];
        k.nrm[i] = c->ct.nrm[i];
    }
    k.out_s = c->ct.out;
    k.out_vn = c->ct.out + c->ct.n;
    return k;
}

// upload the host contact states and set the candidates' constraints
hl_status contact_apply(hl_ctx *c) {
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->ct.state, c->ct.state_h.data(), (size_t)c->ct.n, hipMemcpyHostToDevice, s));
    hl::launch_contact_apply(contact_args(c), c->dim, s);
    HIPCHK(hipStreamSynchronize(s));
    return HL_OK;
}

// One step with rigid-plane contact (Section 3.8, reading R30): trial
// steps from t^n until no candidate detaches or crosses the plane; the
// step that reaches the plane is cut to the impact time.
template <int D>
hl_status contact_step(hl_ctx *c, double dt, hl_step_info *info) {
    constexpr double S_EPS = 1e-9, TIE = 1e-9;
    constexpr int MAX_TRIALS = 8;
    hipStream_t s = c->stream;
    const int src = c->cur;
    const int64_t n = c->ct.n;
    if (!(dt > 0.0)) {
        HIPCHK(hipMemcpyAsync(&dt, c->dt_next, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const double dt_req = dt;
    std::vector<uint8_t> pending(n, 0);
    std::vector<double> out(2 * n);
    bool clipped = false;
    hl_status st = contact_apply(c);
    if (st != HL_OK) return st;
    hl_status rs = HL_OK;
    auto evaluate = [&]() -> hl_status {
        hl::launch_contact_eval<D>(make_args(c, src), contact_args(c), s);
        HIPCHK(hipMemcpyAsync(out.data(), c->ct.out, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return HL_OK;
    };
    int trial = 1;
    for (;; ++trial) {
        if (trial > 1) {
            c->cur = src;
            c->rec_valid = false;  // the gather records hold the trial's state
        }
        rs = run_step<D>(c, dt, nullptr, 0, nullptr);
        if (rs < 0) return rs;
        if (trial == MAX_TRIALS) break;
        if ((st = evaluate()) != HL_OK) return st;
        // detachment at t^n
        bool away = false;
        for (int64_t i = 0; i < n; ++i)
            if (c->ct.state_h[i] && out[n + i] > 0.0) {
                c->ct.state_h[i] = 0;
                away = true;
            }
        if (away) {
            if ((st = contact_apply(c)) != HL_OK) return st;
            continue;
        }
        // impact
        double smin = 2.0;
        for (int64_t i = 0; i < n; ++i)
            if (!c->ct.state_h[i] && !pending[i] && out[i] < 2.0) smin = std::min(smin, out[i]);
        if (smin >= 2.0) break;
        if (smin <= S_EPS) {
            for (int64_t i = 0; i < n; ++i)
                if (!c->ct.state_h[i] && !pending[i] && out[i] <= S_EPS) c->ct.state_h[i] = 1;
            if ((st = contact_apply(c)) != HL_OK) return st;
            continue;
        }
        for (int64_t i = 0; i < n; ++i)
            if (!c->ct.state_h[i] && !pending[i] && out[i] <= smin * (1.0 + TIE)) pending[i] = 1;
        dt = smin * dt;
        clipped = true;
    }
    if (trial == MAX_TRIALS) {
        // accepted as is: every free node below the plane goes into contact
        if ((st = evaluate()) != HL_OK) return st;
        for (int64_t i = 0; i < n; ++i)
            if (!c->ct.state_h[i] && out[i] < 2.0) pending[i] = 1;
    }
    for (int64_t i = 0; i < n; ++i)
        if (pending[i]) c->ct.state_h[i] = 1;
    if ((st = contact_apply(c)) != HL_OK) return st;
    if (clipped) {
        // the growth bound continues from the uncut trial dt
        double parts[2];
        HIPCHK(hipMemcpyAsync(parts, c->dt_parts, sizeof parts, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double dn = std::min(std::min(parts[0], parts[1]), (1.0 + c->prm.c_i) * dt_req);
        HIPCHK(hipMemcpyAsync(c->dt_next, &dn, sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (info) {
        if ((st = fill_info<D>(c, src, info)) != HL_OK) return st;
        info->trials = trial;
        info->clipped = clipped ? 1 : 0;
    }
    return rs;
}

// ------------------------------------------------------------- adjoint
template <class T>
hl_status talloc(hl_ctx *c, T **p, size_t n) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n * sizeof(T), 256)) != hipSuccess) return HL_E_OOM;
    c->tape.mem.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return HL_OK;
}

// state snapshot: x, vhat [D][nn], tau [nc], v [D][nc], e [nc], B [nB][nc]
size_t snapshot_size(const hl_ctx *c) {
    const size_t d = c->dim, nn = c->nn, nc = c->nc, nB = d == 3 ? 6 : 3;
    return 2 * d * nn + (2 + d + nB) * nc;
}

hl_status copy_state(hl_ctx *c, int buf, double *dst, bool to_snapshot) {
    const size_t d = c->dim, nn = c->nn, nc = c->nc, nB = d == 3 ? 6 : 3;
    double *parts[6] = {c->x[buf], c->vhat[buf], c->tau[buf], c->v[buf], c->e[buf], c->B[buf]};
    const size_t sz[6] = {d * nn, d * nn, nc, d * nc, nc, nB * nc};
    hl::CopyFields f{};
    size_t off = 0;
    for (int k = 0; k < 6; ++k) {
        f.src[k] = to_snapshot ? parts[k] : dst + off;
        f.dst[k] = to_snapshot ? dst + off : parts[k];
        f.n[k] = (int64_t)sz[k];
        off += sz[k];
    }
    hl::launch_copy_fields(f, c->stream);  // one launch for the six fields
    return HL_OK;
}

// one step with the recorded dt and cascade choice of step n; with reduce
// false the step leaves no next dt (the caller takes it from the record)
template <int D>
hl_status replay_recorded(hl_ctx *c, int n, bool reduce, double *const *inter = nullptr) {
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->dt_next, c->tape.dts + (size_t)n * c->n_mesh, sizeof(double) * c->n_mesh,
                          hipMemcpyDeviceToDevice, s));
    return run_step<D>(c, 0.0, c->tape.masks + (size_t)n * c->nc, 1, nullptr, true, reduce, inter) < 0 ? HL_E_HIP
                                                                                                      : HL_OK;
}

// forward intermediates of step n for the reverse sweep: state n in buffer 0
template <int D>
void recompute_step(hl_ctx *c, int n) {
    hipStream_t s = c->stream;
    (void)hipMemcpyAsync(c->dt_cur, c->tape.dts + (size_t)n * c->n_mesh, sizeof(double) * c->n_mesh,
                         hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(c->mask, c->tape.masks + (size_t)n * c->nc, (size_t)c->nc, hipMemcpyDeviceToDevice, s);
    hl::StepArgs a = make_args(c, 0);
    a.detect = 0;
    hl::launch_step_begin(c->counters, c->dt_cur, c->dt_next, c->n_mesh, 0, s);
    hl::launch_centroids<D>(a, c->sk[HL_STAGE_PACK], s);
    hl::launch_node_agg<D>(a, c->sk[HL_STAGE_NODE_AGG], s);
    hl::launch_predict<D>(a, c->sk[HL_STAGE_PREDICT], s);
    hl::launch_node_solve<D>(a, c->sk[HL_STAGE_NODE_SOLVE], s);
    hl::launch_update<D>(a, c->sk[HL_STAGE_UPDATE], s);
}

hl::AdjArgs adj_args(hl_ctx *c, int in) {
    const size_t d = c->dim, nn = c->nn, nc = c->nc;
    hl::AdjArgs j{};
    const double *li = c->tape.lam[in];
    double *lo = c->tape.lam[1 - in];
    j.lx_in = li;
    j.lvh_in = li + d * nn;
    j.ltau_in = li + 2 * d * nn;
    j.lv_in = li + 2 * d * nn + nc;
    j.lB_in = li + 2 * d * nn + (1 + d) * nc;
    j.lx_out = lo;
    j.lvh_out = lo + d * nn;
    j.ltau_out = lo + 2 * d * nn;
    j.lv_out = lo + 2 * d * nn + nc;
    j.lB_out = lo + 2 * d * nn + (1 + d) * nc;
    j.cadj = c->tape.cadj;
    j.nadj = c->tape.nadj;
    j.cell = c->tape.cell;
    j.agg = c->tape.agg;
    j.xadj = c->tape.xadj;
    j.mu_bar = c->tape.mu_bar;
    return j;
}

// node aggregates the step writes (no limiter bounds, no gas sums: the
// adjoint runs neither)
template <int D>
constexpr size_t kAggBase = hl::Dims<D>::NA_BASE;

// The forward intermediates of step n of the current segment (tape slot
// k): node aggregates [kAggBase][nn] (the pairs a step without limiter
// bounds or gas sums writes), corner records in whole 256-cell tiles, v*.
template <int D>
void inter_slot(hl_ctx *c, int k, double *p[3]) {
    auto &t = c->tape;
    const size_t nn = c->nn, nc = c->nc;
    const size_t na = kAggBase<D> * nn, ncr = (nc + 255) / 256 * 256 * (D + 1) * hl::Dims<D>::CW;
    double *src = t.inter + (size_t)k * t.inter_sz;
    p[0] = src;
    p[1] = src + na;
    p[2] = src + na + ncr;
}

template <int D>
hl_status forward_record(hl_ctx *c, int nsteps, int every) {
    free_tape(c);
    auto &t = c->tape;
    t.nsteps = nsteps;
    t.every = every;
    t.nckpt = (nsteps + every - 1) / every + 1;
    t.state_sz = snapshot_size(c);
    const size_t nn = c->nn, nc = c->nc, ncor = nc * (D + 1), lam_sz = 2 * D * nn + (1 + D + (D == 3 ? 6 : 3)) * nc;
    hl_status st;
    if ((st = talloc(c, &t.ckpt, t.nckpt * t.state_sz)) != HL_OK) return st;
    if ((st = talloc(c, &t.seg, (size_t)every * t.state_sz)) != HL_OK) return st;
    if ((st = talloc(c, &t.dts, (size_t)nsteps * c->n_mesh)) != HL_OK) return st;
    if ((st = talloc(c, &t.masks, (size_t)nsteps * nc)) != HL_OK) return st;
    for (int b = 0; b < 2; ++b)
        if ((st = talloc(c, &t.lam[b], lam_sz)) != HL_OK) return st;
    if ((st = talloc(c, &t.cadj, ncor * hl::AdjArgs::CA)) != HL_OK) return st;
    if ((st = talloc(c, &t.nadj, nn * hl::AdjArgs::NAD)) != HL_OK) return st;
    if ((st = talloc(c, &t.cell, nc * hl::AdjArgs::CL)) != HL_OK) return st;
    if ((st = talloc(c, &t.agg, nn * hl::AdjArgs::NAA)) != HL_OK) return st;
    if ((st = talloc(c, &t.xadj, ncor * 3)) != HL_OK) return st;
    if ((st = talloc(c, &t.mu_bar, nc)) != HL_OK) return st;
    if ((st = talloc(c, &t.out, std::max(nn, nc) * 3)) != HL_OK) return st;
    if ((st = talloc(c, &t.dtn, (size_t)c->n_mesh)) != HL_OK) return st;
    {
        // the segment's forward intermediates, if they fit 8 GiB
        t.inter_sz = kAggBase<D> * nn + (nc + 255) / 256 * 256 * (D + 1) * hl::Dims<D>::CW + D * nn;
        const size_t n_inter = t.inter_sz * (size_t)every;
        void *q = nullptr;
        if (sizeof(double) * n_inter <= (size_t(8) << 30) && hipMalloc(&q, sizeof(double) * n_inter) == hipSuccess) {
            t.mem.push_back(q);
            t.inter = static_cast<double *>(q);
        } else {
            (void)hipGetLastError();  // a refused allocation is not an error here
            t.inter = nullptr;
        }
    }
    for (int n = 0; n < nsteps; ++n) {
        if (n % every == 0) {
            if ((st = copy_state(c, c->cur, t.ckpt + (size_t)(n / every) * t.state_sz, true)) != HL_OK) return st;
        }
        hl_status r = run_step<D>(c, 0.0, nullptr, 0, nullptr);
        if (r < 0) return r;
        HIPCHK(hipMemcpyAsync(t.masks + (size_t)n * nc, c->mask, nc, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(t.dts + (size_t)n * c->n_mesh, c->dt_cur, sizeof(double) * c->n_mesh,
                              hipMemcpyDeviceToDevice, c->stream));
    }
    if ((st = copy_state(c, c->cur, t.ckpt + (size_t)(t.nckpt - 1) * t.state_sz, true)) != HL_OK) return st;
    HIPCHK(hipMemcpyAsync(t.dtn, c->dt_next, sizeof(double) * c->n_mesh, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return HL_OK;
}

template <int D>
hl_status forward_replay(hl_ctx *c) {
    for (int n = 0; n < c->tape.nsteps; ++n) {
        // each replayed step takes its dt from the record: only the last
        // one computes the next dt (that of the replayed state)
        hl_status st = replay_recorded<D>(c, n, n + 1 == c->tape.nsteps);
        if (st != HL_OK) return st;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return HL_OK;
}

template <int D>
hl_status adjoint_run(hl_ctx *c, const double *dLdx, double *dLdmu, double *dLdvc, double *dLdvn, int on_device) {
    auto &t = c->tape;
    hipStream_t s = c->stream;
    const size_t nn = c->nn, nc = c->nc, lam_sz = 2 * D * nn + (1 + D + (D == 3 ? 6 : 3)) * nc;
    const hipMemcpyKind kin = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind kout = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    {
        hl_status st = ensure_scheds(c);
        if (st != HL_OK) return st;
    }
    // lambda at the final time: dL/dx, nothing on the other fields
    HIPCHK(hipMemsetAsync(t.lam[0], 0, sizeof(double) * lam_sz, s));
    HIPCHK(hipMemsetAsync(t.mu_bar, 0, sizeof(double) * nc, s));
    if (nn) {
        HIPCHK(hipMemcpyAsync(t.out, dLdx, sizeof(double) * nn * D, kin, s));
        hl::launch_aos_to_soa(nn, D, t.out, t.lam[0], s, c->permuted ? c->d_n_u2i : nullptr);
    }
    int in = 0;
    const int nseg = (t.nsteps + t.every - 1) / t.every;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * t.every, s1 = std::min(t.nsteps, s0 + t.every);
        // rebuild the segment's states from its checkpoint
        c->cur = 0;
        hl_status st = copy_state(c, 0, t.ckpt + (size_t)seg * t.state_sz, false);
        if (st != HL_OK) return st;
        c->rec_valid = false;
        for (int n = s0; n < s1; ++n) {
            if ((st = copy_state(c, c->cur, t.seg + (size_t)(n - s0) * t.state_sz, true)) != HL_OK) return st;
            // with room for them, the replay also runs the segment's last
            // step and writes every step's intermediates to the tape
            if (t.inter) {
                double *slot[3];
                inter_slot<D>(c, n - s0, slot);
                if ((st = replay_recorded<D>(c, n, false, slot)) != HL_OK) return st;
            } else if (n + 1 < s1) {
                if ((st = replay_recorded<D>(c, n, false)) != HL_OK) return st;
            }
        }
        for (int n = s1 - 1; n >= s0; --n) {
            hl::StepArgs a;
            if (t.inter) {
                // the step's dt and cascade levels read from the record,
                // its intermediates from the replay, state n and the
                // candidate (state n + 1) from the held snapshots
                a = make_args(c, 0);
                a.dt = t.dts + (size_t)n * c->n_mesh;
                a.mask = t.masks + (size_t)n * c->nc;
                double *slot[3];
                inter_slot<D>(c, n - s0, slot);
                a.agg = slot[0];
                a.corner = slot[1];
                a.vstar = slot[2];
                double *cx = t.seg + (size_t)(n - s0) * t.state_sz;
                a.x = cx;
                a.vhat = cx + D * nn;
                a.tau = cx + 2 * D * nn;
                a.v = cx + 2 * D * nn + nc;
                a.e = cx + 2 * D * nn + (1 + D) * nc;
                a.B = cx + 2 * D * nn + (2 + D) * nc;
                const double *next = n + 1 < s1 ? t.seg + (size_t)(n + 1 - s0) * t.state_sz
                                                : t.ckpt + (size_t)(seg + 1) * t.state_sz;
                // the candidate of step n is state n + 1, laid out as in
                // copy_state: x, vhat, tau, v, e, B
                double *nx = const_cast<double *>(next);
                a.x1 = nx;
                a.vhat1 = nx + D * nn;
                a.tau1 = nx + 2 * D * nn;
                a.v1 = nx + 2 * D * nn + nc;
                a.e1 = nx + 2 * D * nn + (1 + D) * nc;
                a.B1 = nx + 2 * D * nn + (2 + D) * nc;
            } else {
                if ((st = copy_state(c, 0, t.seg + (size_t)(n - s0) * t.state_sz, false)) != HL_OK) return st;
                recompute_step<D>(c, n);
                a = make_args(c, 0);
            }
            hl::launch_adjoint_step<D>(a, adj_args(c, in), s);
            in = 1 - in;
        }
    }
    // lambda at t = 0 -> gradients of the inputs
    const double *lam = t.lam[in];
    const int32_t *cidx = c->permuted ? c->d_c_u2i : nullptr, *nidx = c->permuted ? c->d_n_u2i : nullptr;
    if (nc) {
        if (cidx) {
            hl::launch_soa_to_aos(nc, 1, t.mu_bar, t.out, s, cidx);
            HIPCHK(hipMemcpyAsync(dLdmu, t.out, sizeof(double) * nc, kout, s));
        } else {
            HIPCHK(hipMemcpyAsync(dLdmu, t.mu_bar, sizeof(double) * nc, kout, s));
        }
        hl::launch_soa_to_aos(nc, D, lam + 2 * D * nn + nc, t.out, s, cidx);
        HIPCHK(hipMemcpyAsync(dLdvc, t.out, sizeof(double) * nc * D, kout, s));
    }
    if (nn) {
        hl::launch_adj_project<D>(nn, c->nallow, c->allow, lam + D * nn, t.out, s);
        if (nidx) {
            hl::launch_gather_rows(nn, D, t.out, nidx, c->scratch, s);
            HIPCHK(hipMemcpyAsync(dLdvn, c->scratch, sizeof(double) * nn * D, kout, s));
        } else {
            HIPCHK(hipMemcpyAsync(dLdvn, t.out, sizeof(double) * nn * D, kout, s));
        }
    }
    // leave the context at the final forward state, with the next dt and
    // the cascade levels of the last recorded step
    c->cur = 0;
    hl_status st = copy_state(c, 0, t.ckpt + (size_t)(t.nckpt - 1) * t.state_sz, false);
    if (st != HL_OK) return st;
    HIPCHK(hipMemcpyAsync(c->dt_next, t.dtn, sizeof(double) * c->n_mesh, hipMemcpyDeviceToDevice, s));
    if (t.nsteps > 0)
        HIPCHK(hipMemcpyAsync(c->dt_cur, t.dts + (size_t)(t.nsteps - 1) * c->n_mesh, sizeof(double) * c->n_mesh,
                              hipMemcpyDeviceToDevice, s));
    if (nc)
        HIPCHK(hipMemcpyAsync(c->mask, t.masks + (size_t)(t.nsteps - 1) * nc, nc, hipMemcpyDeviceToDevice, s));
    c->rec_valid = false;
    HIPCHK(hipStreamSynchronize(s));
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return hip_fail(le, "adjoint kernel launch", __LINE__);
    return HL_OK;
}

// ------------------------------------------------------------ autotuner
template <int D>
void launch_stage(hl_ctx *c, const hl::StepArgs &a, int stage, const hl::Sched &k, hipStream_t s) {
    switch (stage) {
        case HL_STAGE_PACK: hl::launch_centroids<D>(a, k, s); break;
        case HL_STAGE_NODE_AGG: hl::launch_node_agg<D>(a, k, s); break;
        case HL_STAGE_PREDICT: hl::launch_predict<D>(a, k, s); break;
        case HL_STAGE_NODE_SOLVE: hl::launch_node_solve<D>(a, k, s); break;
        default:
            // the update appends flagged cells: start every run from empty lists
            hl::launch_step_begin(c->counters, c->dt_cur, c->dt_next, c->n_mesh, 0, s);
            hl::launch_update<D>(a, k, s);
            break;
    }
}

// Times every candidate schedule of every stage on the current mesh and
// state (the stages read the state and write only work buffers and the
// candidate buffers) and keeps the fastest.  Results do not depend on the
// schedule: every entity is computed by one thread in a fixed order.
template <int D>
hl_status autotune(hl_ctx *c, int reps, double *best_ms) {
    hipStream_t s = c->stream;
    hl_status st = ensure_scheds(c);
    if (st != HL_OK) return st;
    const bool prof = c->prof.on;
    c->prof.on = false;
    hl::StepArgs a = make_args(c, c->cur);
    hl::launch_step_begin(c->counters, c->dt_cur, c->dt_next, c->n_mesh, 1, s);
    for (int stage = 0; stage < HL_STAGE_COUNT; ++stage) launch_stage<D>(c, a, stage, c->sk[stage], s);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    static const int kBlock[] = {64, 128, 256};
    // tile in eighths of a block: node stages run AGG_G lanes per node, so
    // their one-pass items (block / AGG_G nodes) are candidates too
    static const int kTile8[] = {1, 2, 8, 16, 32};
    static const int kPerCu[] = {0, 2, 4, 8};
    auto sweep = [&](int stage, StageCfg *keep, double *best) -> hl_status {
        for (int b : kBlock)
            for (int m8 : kTile8)
                for (int q : kPerCu) {
                    if (m8 < 8 && kStageKind[stage] == 0) continue;
                    StageCfg g;
                    g.tile = b * m8 / 8;
                    g.block = b;
                    g.blocks_per_cu = q;
                    hl::Sched k;
                    hl_status r = build_sched(c, stage, g, &k);
                    if (r != HL_OK) return r;
                    launch_stage<D>(c, a, stage, k, s);
                    HIPCHK(hipEventRecord(e0, s));
                    for (int i = 0; i < reps; ++i) launch_stage<D>(c, a, stage, k, s);
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < *best) {
                        *best = ms;
                        *keep = g;
                    }
                }
        return HL_OK;
    };
    for (int stage = 0; stage < HL_STAGE_COUNT && st == HL_OK; ++stage) {
        double best = 1e300;
        StageCfg keep = c->cfg[stage];
        st = sweep(stage, &keep, &best);
        if (st != HL_OK) break;
        c->cfg[stage] = keep;
        c->cfg_set[stage] = true;
        if (best_ms) best_ms[stage] = best < 1e300 ? best / reps : 0.0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof.on = prof;
    // leave empty lists behind; the gather records now hold the candidate
    hl::launch_step_begin(c->counters, c->dt_cur, c->dt_next, c->n_mesh, 0, s);
    c->rec_valid = false;
    c->sched_ready = false;
    drop_graphs(c);
    if (st != HL_OK) return st;
    HIPCHK(hipStreamSynchronize(s));
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return hip_fail(le, "autotune launch", __LINE__);
    return ensure_scheds(c);
}

int field_width(const hl_ctx *c, int field, bool *node, bool *is_u8) {
    *node = false;
    *is_u8 = false;
    const int d = c->dim;
    switch (field) {
        case HL_X:
        case HL_VHAT:
        case HL_VSTAR:
            *node = true;
            return d;
        case HL_TAU:
        case HL_E:
        case HL_MASS:
            return 1;
        case HL_V:
            return d;
        case HL_B:
            return d == 3 ? 6 : 3;
        case HL_ORDER:
            *is_u8 = true;
            return 1;
        case HL_T:
            return d == 3 ? 6 : 4;
        default:
            return -1;
    }
}

double *field_ptr(hl_ctx *c, int field) {
    const int b = c->cur;
    switch (field) {
        case HL_X: return c->x[b];
        case HL_VHAT: return c->vhat[b];
        case HL_VSTAR: return c->vstar;
        case HL_TAU: return c->tau[b];
        case HL_E: return c->e[b];
        case HL_MASS: return c->mass;
        case HL_V: return c->v[b];
        case HL_B: return c->B[b];
        default: return nullptr;
    }
}

}  // namespace

extern "C" {

const char *hl_last_error(void) { return g_last_error; }

const char *hl_status_str(hl_status s) {
    switch (s) {
        case HL_OK: return "ok";
        case HL_WARN_PARACHUTE_INADMISSIBLE: return "a first-order (parachute) cell is not admissible";
        case HL_E_INVALID: return "invalid argument";
        case HL_E_DEGENERATE_CELL: return "cell with non-positive volume";
        case HL_E_OOM: return "device allocation failed";
        case HL_E_HIP: return "HIP runtime error";
        case HL_E_STATE: return "call out of order (mesh or state missing)";
        case HL_E_NONCONFORMING: return "the cells do not form a conforming mesh";
        default: return "unknown status";
    }
}

hl_status hl_create(hl_ctx **out, int device, void *hip_stream) {
    if (!out) return HL_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return HL_E_HIP;
    if (device < 0 || device >= n) return HL_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return HL_E_HIP;
    hl_ctx *c = new hl_ctx();
    c->device = device;
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        c->n_cu < 1)
        c->n_cu = 256;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    *out = c;
    return HL_OK;
}

hl_status hl_destroy(hl_ctx *c) {
    if (!c) return HL_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    free_all(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return HL_OK;
}

}  // extern "C"

namespace {

// Mesh inputs brought to the host, cells in global node numbering.
struct HostMesh {
    std::vector<double> x, nrm;
    std::vector<int32_t> cells;
    std::vector<uint8_t> nw;
};

hl_status gather_mesh(int dim, int64_t n_nodes, const double *x0, int64_t n_cells, const int32_t *cells,
                      const uint8_t *nwall, const double *normals, int on_device, HostMesh &h) {
    const int nv = dim + 1;
    hl_status st;
    if ((st = to_host(x0, (size_t)(n_nodes * dim), on_device, h.x)) != HL_OK) return st;
    if ((st = to_host(cells, (size_t)(n_cells * nv), on_device, h.cells)) != HL_OK) return st;
    if (nwall) {
        if ((st = to_host(nwall, (size_t)n_nodes, on_device, h.nw)) != HL_OK) return st;
        if (!normals) return HL_E_INVALID;
        if ((st = to_host(normals, (size_t)(n_nodes * dim * dim), on_device, h.nrm)) != HL_OK) return st;
    } else {
        h.nw.assign((size_t)n_nodes, 0);
        h.nrm.assign((size_t)(n_nodes * dim * dim), 0.0);
    }
    return HL_OK;
}

// The held mesh in the caller's numbering.
void user_mesh(const hl_ctx *c, HostMesh &h) {
    if (!c->permuted) {
        h.x = c->x0_host;
        h.cells = c->c2n_host;
        h.nw = c->nw_host;
        h.nrm = c->nrm_host;
        return;
    }
    const int d = c->dim, nv = d + 1, dd = d * d;
    const size_t nn = (size_t)c->nn, nc = (size_t)c->nc;
    h.x.resize(nn * d);
    h.nrm.resize(nn * dd);
    h.nw.resize(nn);
    h.cells.resize(nc * nv);
    for (size_t u = 0; u < nn; ++u) {
        const size_t i = (size_t)c->n_u2i[u];
        for (int j = 0; j < d; ++j) h.x[u * d + j] = c->x0_host[i * d + j];
        for (int j = 0; j < dd; ++j) h.nrm[u * dd + j] = c->nrm_host[i * dd + j];
        h.nw[u] = c->nw_host[i];
    }
    for (size_t u = 0; u < nc; ++u) {
        const size_t i = (size_t)c->c_u2i[u];
        for (int k = 0; k < nv; ++k) h.cells[u * nv + k] = c->n_i2u[(size_t)c->c2n_host[i * nv + k]];
    }
}

// Validate, build the node -> corner lists and wall bases, allocate the
// device buffers and upload.  node_off / cell_off delimit the meshes of a
// batch (n_mesh >= 1); cells already use global node numbers.
hl_status upload_impl(hl_ctx *c, int dim, int n_mesh, const std::vector<int64_t> &node_off,
                      const std::vector<int64_t> &cell_off, HostMesh &h, bool check_conformity) {
    const int nv = dim + 1;
    const int64_t n_nodes = node_off[n_mesh], n_cells = cell_off[n_mesh];
    std::vector<double> &xh = h.x, &nrm = h.nrm;
    std::vector<int32_t> &ch = h.cells;
    std::vector<uint8_t> &nw = h.nw;
    hl_status st;
    for (int m = 0; m < n_mesh; ++m)
        for (int64_t q = cell_off[m] * nv; q < cell_off[m + 1] * nv; ++q)
            if (ch[q] < node_off[m] || ch[q] >= node_off[m + 1]) return HL_E_INVALID;
    for (int64_t p = 0; p < n_nodes; ++p)
        if (nw[p] > dim) return HL_E_INVALID;
    for (double v : xh)
        if (!std::isfinite(v)) return HL_E_INVALID;
    // positive orientation of every cell
    for (int64_t cc = 0; cc < n_cells; ++cc) {
        double X[12];
        for (int k = 0; k < nv; ++k)
            for (int i = 0; i < dim; ++i) X[k * dim + i] = xh[(size_t)ch[cc * nv + k] * dim + i];
        if (!(host_volume(dim, X) > 0.0)) return HL_E_DEGENERATE_CELL;
    }
    if (check_conformity)
        for (int m = 0; m < n_mesh; ++m)
            if ((st = hl::check_conforming(dim, xh.data(), ch.data(), node_off[m], node_off[m + 1], cell_off[m],
                                           cell_off[m + 1])) != HL_OK)
                return st;
    // internal numbering: cells along a Hilbert curve, nodes by first use
    std::vector<int32_t> ci2u, ni2u, cu2i, nu2i;
    bool perm = c->numbering == HL_NUMBERING_SPATIAL && n_cells > 0;
    if (perm) {
        hl::spatial_numbering(dim, xh.data(), ch.data(), node_off, cell_off, ci2u, ni2u);
        bool ident = true;
        for (int64_t i = 0; i < n_cells && ident; ++i) ident = ci2u[i] == i;
        for (int64_t i = 0; i < n_nodes && ident; ++i) ident = ni2u[i] == i;
        perm = !ident;
    }
    if (perm) {
        cu2i.resize((size_t)n_cells);
        nu2i.resize((size_t)n_nodes);
        for (int64_t i = 0; i < n_cells; ++i) cu2i[ci2u[i]] = (int32_t)i;
        for (int64_t i = 0; i < n_nodes; ++i) nu2i[ni2u[i]] = (int32_t)i;
        std::vector<double> x2((size_t)(n_nodes * dim)), n2((size_t)(n_nodes * dim * dim));
        std::vector<uint8_t> w2((size_t)n_nodes);
        std::vector<int32_t> c2((size_t)(n_cells * nv));
        for (int64_t i = 0; i < n_nodes; ++i) {
            const int64_t u = ni2u[i];
            for (int j = 0; j < dim; ++j) x2[i * dim + j] = xh[u * dim + j];
            for (int j = 0; j < dim * dim; ++j) n2[i * dim * dim + j] = nrm[u * dim * dim + j];
            w2[i] = nw[u];
        }
        for (int64_t i = 0; i < n_cells; ++i)
            for (int k = 0; k < nv; ++k) c2[i * nv + k] = nu2i[ch[(size_t)ci2u[i] * nv + k]];
        xh.swap(x2);
        nrm.swap(n2);
        nw.swap(w2);
        ch.swap(c2);
    } else {
        ci2u.clear();
        ni2u.clear();
    }
    // node -> corner lists in (cell, local node) order
    std::vector<int32_t> off((size_t)n_nodes + 1, 0), lst((size_t)(n_cells * nv));
    for (int64_t q = 0; q < n_cells * nv; ++q) off[(size_t)ch[q] + 1]++;
    for (int64_t p = 0; p < n_nodes; ++p) off[p + 1] += off[p];
    {
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int64_t q = 0; q < n_cells * nv; ++q) lst[fill[ch[q]]++] = (int32_t)q;
    }
    std::vector<uint8_t> nal((size_t)n_nodes);
    std::vector<double> alw((size_t)(n_nodes * dim * dim));
    for (int64_t p = 0; p < n_nodes; ++p)
        nal[p] = (uint8_t)wall_basis(dim, nw[p], nrm.data() + p * dim * dim, alw.data() + p * dim * dim);

    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    c->dim = dim;
    c->nn = n_nodes;
    c->nc = n_cells;
    c->n_mesh = n_mesh;
    const size_t nn = (size_t)n_nodes, ncl = (size_t)n_cells, ncor = ncl * nv;
    const int NA = dim == 3 ? hl::Dims<3>::NA : hl::Dims<2>::NA;
    const int CW = dim == 3 ? hl::Dims<3>::CW : hl::Dims<2>::CW;
    const int nB = dim == 3 ? 6 : 3;
#define A_(p, n)                                  \
    do {                                          \
        if ((st = dalloc(c, &(p), (n))) != HL_OK) { \
            free_all(c);                          \
            return st;                            \
        }                                         \
    } while (0)
    A_(c->c2n, ncor);
    A_(c->n2c_off, nn + 1);
    A_(c->n2c, ncor);
    A_(c->nallow, nn);
    A_(c->allow, nn * dim * dim);
    A_(c->mass, ncl);
    A_(c->rho0, ncl);
    A_(c->mu, ncl);
    A_(c->K, ncl);
    for (int b = 0; b < 2; ++b) {
        A_(c->x[b], nn * dim);
        A_(c->vhat[b], nn * dim);
        A_(c->tau[b], ncl);
        A_(c->v[b], ncl * dim);
        A_(c->e[b], ncl);
        A_(c->B[b], ncl * nB);
    }
    A_(c->vstar, nn * dim);
    A_(c->xc, ncl * (dim == 3 ? hl::Dims<3>::GR : hl::Dims<2>::GR));
    A_(c->agg, nn * NA);
    // whole 256-cell tiles, and two doubles of pad: the node gathers read
    // each record in 16-byte pairs, the last one reaching one double past it
    A_(c->corner, (ncl + 255) / 256 * 256 * nv * CW + 2);
    A_(c->dtc, 2 * ncl);
    A_(c->mask, ncl);
    A_(c->pstat, ncl);
    A_(c->flist[0], ncl);
    A_(c->flist[1], ncl);
    A_(c->nlist, nn);
    A_(c->clist, ncl);
    A_(c->nstamp, nn);
    A_(c->cstamp, ncl);
    A_(c->mesh_cell_off, (size_t)n_mesh + 1);
    if (n_mesh > 1) {
        A_(c->cell_mesh, ncl);
        A_(c->node_mesh, nn);
    }
    A_(c->dt_part, 2 * (ncl / 256 + 2));
    A_(c->counters, hl::CNT_N);
    A_(c->stamp_dev, 1);
    A_(c->pass_log, 128);  // [0, 64): captured step; [64, 128): continuation
    A_(c->dt_cur, (size_t)n_mesh);
    A_(c->dt_next, (size_t)n_mesh);
    A_(c->dt_red, 2 * (size_t)n_mesh);
    A_(c->dt_parts, 2 * (size_t)n_mesh);
    A_(c->diag_part, hl::DIAG_N * (ncl / 256 + 2));
    A_(c->diag_out, 16);
    c->scratch_bytes = std::max<size_t>(sizeof(double) * std::max(nn * dim, ncl * 6), 256);
    A_(c->scratch, c->scratch_bytes / sizeof(double));
    A_(c->mask_in, ncl);
    if (perm) {
        A_(c->d_c_i2u, ncl);
        A_(c->d_c_u2i, ncl);
        A_(c->d_n_u2i, nn);
    }
#undef A_
    if (hipHostMalloc((void **)&c->counters_host, (hl::CNT_N + 128) * sizeof(unsigned), hipHostMallocDefault) !=
        hipSuccess) {
        free_all(c);
        return HL_E_OOM;
    }
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->c2n, ch.data(), sizeof(int32_t) * ncor, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->n2c_off, off.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->n2c, lst.data(), sizeof(int32_t) * ncor, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->nallow, nal.data(), nn, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->allow, alw.data(), sizeof(double) * nn * dim * dim, hipMemcpyHostToDevice, s));
    // positions AoS -> SoA on the host
    std::vector<double> xs(nn * dim);
    for (size_t p = 0; p < nn; ++p)
        for (int i = 0; i < dim; ++i) xs[i * nn + p] = xh[p * dim + i];
    HIPCHK(hipMemcpyAsync(c->x[0], xs.data(), sizeof(double) * nn * dim, hipMemcpyHostToDevice, s));
    if (nn) HIPCHK(hipMemsetAsync(c->nstamp, 0, sizeof(int32_t) * nn, s));
    if (ncl) HIPCHK(hipMemsetAsync(c->cstamp, 0, sizeof(int32_t) * ncl, s));
    if (ncl) HIPCHK(hipMemsetAsync(c->pstat, 0, ncl, s));
    HIPCHK(hipMemcpyAsync(c->mesh_cell_off, cell_off.data(), sizeof(int64_t) * (n_mesh + 1), hipMemcpyHostToDevice,
                          s));
    if (perm) {
        HIPCHK(hipMemcpyAsync(c->d_c_i2u, ci2u.data(), sizeof(int32_t) * ncl, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(c->d_c_u2i, cu2i.data(), sizeof(int32_t) * ncl, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(c->d_n_u2i, nu2i.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, s));
    }
    std::vector<int32_t> cm, nm;
    if (n_mesh > 1) {
        cm.resize(ncl);
        nm.resize(nn);
        for (int m = 0; m < n_mesh; ++m) {
            for (int64_t q = cell_off[m]; q < cell_off[m + 1]; ++q) cm[q] = m;
            for (int64_t q = node_off[m]; q < node_off[m + 1]; ++q) nm[q] = m;
        }
        if (ncl) HIPCHK(hipMemcpyAsync(c->cell_mesh, cm.data(), sizeof(int32_t) * ncl, hipMemcpyHostToDevice, s));
        if (nn) HIPCHK(hipMemcpyAsync(c->node_mesh, nm.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    c->cell_off_host = cell_off;
    c->node_off_host = node_off;
    c->max_deg = 0;
    for (int64_t p = 0; p < n_nodes; ++p) c->max_deg = std::max<int64_t>(c->max_deg, off[p + 1] - off[p]);
    HIPCHK(hipMemsetAsync(c->stamp_dev, 0, sizeof(int32_t), s));
    HIPCHK(hipStreamSynchronize(s));
    c->stamp_host = 0;
    c->x0_host.swap(xh);
    c->c2n_host.swap(ch);
    c->nw_host.swap(nw);
    c->nrm_host.swap(nrm);
    c->permuted = perm;
    c->c_i2u.swap(ci2u);
    c->c_u2i.swap(cu2i);
    c->n_i2u.swap(ni2u);
    c->n_u2i.swap(nu2i);
    {
        // FNV-1a over the sizes and the internal connectivity
        uint64_t hsh = 1469598103934665603ull;
        auto mix = [&](uint64_t v) {
            for (int b = 0; b < 8; ++b) {
                hsh ^= (v >> (8 * b)) & 0xffu;
                hsh *= 1099511628211ull;
            }
        };
        mix((uint64_t)dim);
        mix((uint64_t)n_nodes);
        mix((uint64_t)n_cells);
        mix((uint64_t)n_mesh);
        for (int32_t q : c->c2n_host) mix((uint64_t)(uint32_t)q);
        c->mesh_hash = hsh;
    }
    c->cur = 0;
    c->prm = default_params(dim);
    c->have_mesh = true;
    c->have_state = false;
    return HL_OK;
}

}  // namespace

extern "C" {

hl_status hl_mesh_upload(hl_ctx *c, int dim, int64_t n_nodes, const double *x0, int64_t n_cells,
                         const int32_t *cells, const uint8_t *nwall, const double *normals, int on_device) {
    if (!c || (dim != 2 && dim != 3) || n_nodes < 0 || n_cells < 0) return HL_E_INVALID;
    if (n_cells * (dim + 1) >= (int64_t)INT32_MAX || n_nodes >= (int64_t)INT32_MAX) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    HostMesh h;
    hl_status st = gather_mesh(dim, n_nodes, x0, n_cells, cells, nwall, normals, on_device, h);
    if (st != HL_OK) return st;
    std::vector<int64_t> no = {0, n_nodes}, co = {0, n_cells};
    return upload_impl(c, dim, 1, no, co, h, true);
}

hl_status hl_mesh_upload_batch(hl_ctx *c, int dim, int n_meshes, const int64_t *node_offsets,
                               const int64_t *cell_offsets, const double *x0, const int32_t *cells,
                               const uint8_t *nwall, const double *normals, int on_device) {
    if (!c || (dim != 2 && dim != 3) || n_meshes < 1 || !node_offsets || !cell_offsets) return HL_E_INVALID;
    std::vector<int64_t> no(node_offsets, node_offsets + n_meshes + 1), co(cell_offsets, cell_offsets + n_meshes + 1);
    if (no[0] != 0 || co[0] != 0) return HL_E_INVALID;
    for (int m = 0; m < n_meshes; ++m)
        if (no[m + 1] < no[m] || co[m + 1] < co[m]) return HL_E_INVALID;
    const int64_t n_nodes = no[n_meshes], n_cells = co[n_meshes];
    if (n_cells * (dim + 1) >= (int64_t)INT32_MAX || n_nodes >= (int64_t)INT32_MAX) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    HostMesh h;
    hl_status st = gather_mesh(dim, n_nodes, x0, n_cells, cells, nwall, normals, on_device, h);
    if (st != HL_OK) return st;
    // mesh-local node numbers -> global
    const int nv = dim + 1;
    for (int m = 0; m < n_meshes; ++m)
        for (int64_t q = co[m] * nv; q < co[m + 1] * nv; ++q) {
            const int64_t g = (int64_t)h.cells[q] + no[m];
            if (h.cells[q] < 0 || g >= no[m + 1]) return HL_E_INVALID;
            h.cells[q] = (int32_t)g;
        }
    return upload_impl(c, dim, n_meshes, no, co, h, true);
}

hl_status hl_mesh_refine(hl_ctx *c, int levels) {
    if (!c || levels < 0 || levels > 4) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (c->n_mesh != 1) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    const int d = c->dim, nv = d + 1, dd = d * d;
    {
        // every level multiplies the cells by 2^d; node and corner ids stay int32
        double ncl = (double)c->nc;
        for (int l = 0; l < levels; ++l) ncl *= (d == 3 ? 8.0 : 4.0);
        if (ncl * (nv > 3 ? 6 : 3) >= (double)INT32_MAX) {
            std::snprintf(g_last_error, sizeof g_last_error, "refined mesh too large for 32-bit ids");
            return HL_E_INVALID;
        }
    }
    HostMesh h;
    user_mesh(c, h);
    for (int l = 0; l < levels; ++l) {
        const int64_t nn = (int64_t)h.nw.size(), nc = (int64_t)h.cells.size() / nv;
        std::vector<double> xo;
        std::vector<int32_t> co;
        std::vector<uint64_t> ed;
        hipError_t e = d == 3 ? hl::refine_once<3>(nn, nc, h.x.data(), h.cells.data(), c->stream, xo, co, ed)
                              : hl::refine_once<2>(nn, nc, h.x.data(), h.cells.data(), c->stream, xo, co, ed);
        if (e != hipSuccess) return hip_fail(e, "mesh refinement", __LINE__);
        // a midpoint keeps the wall normals its two end nodes share
        const int64_t ne = (int64_t)ed.size();
        std::vector<uint8_t> nw((size_t)(nn + ne), 0);
        std::vector<double> nrm((size_t)(nn + ne) * dd, 0.0);
        std::copy(h.nw.begin(), h.nw.end(), nw.begin());
        std::copy(h.nrm.begin(), h.nrm.end(), nrm.begin());
        for (int64_t k = 0; k < ne; ++k) {
            const int64_t p = (int64_t)(ed[k] >> 32), q = (int64_t)(ed[k] & 0xffffffffu);
            int cnt = 0;
            for (int r = 0; r < h.nw[p]; ++r) {
                const double *np_ = h.nrm.data() + p * dd + r * d;
                bool shared = false;
                for (int t = 0; t < h.nw[q] && !shared; ++t) {
                    const double *nq = h.nrm.data() + q * dd + t * d;
                    double dot = 0.0;
                    for (int i = 0; i < d; ++i) dot += np_[i] * nq[i];
                    shared = dot >= 1.0 - 1e-12;
                }
                if (shared && cnt < d) {
                    for (int i = 0; i < d; ++i) nrm[(nn + k) * dd + cnt * d + i] = np_[i];
                    ++cnt;
                }
            }
            nw[nn + k] = (uint8_t)cnt;
        }
        h.x.swap(xo);
        h.cells.swap(co);
        h.nw.swap(nw);
        h.nrm.swap(nrm);
    }
    const int64_t nn = (int64_t)h.nw.size(), nc = (int64_t)h.cells.size() / nv;
    std::vector<int64_t> no = {0, nn}, cof = {0, nc};
    // red refinement of a conforming mesh is conforming: no second check
    return upload_impl(c, d, 1, no, cof, h, false);
}

hl_status hl_set_numbering(hl_ctx *c, int numbering) {
    if (!c || (numbering != HL_NUMBERING_KEEP && numbering != HL_NUMBERING_SPATIAL)) return HL_E_INVALID;
    c->numbering = numbering;
    return HL_OK;
}

hl_status hl_mesh_check(int dim, int64_t n_nodes, const double *x0, int64_t n_cells, const int32_t *cells) {
    if ((dim != 2 && dim != 3) || n_nodes < 0 || n_cells < 0) return HL_E_INVALID;
    if ((n_nodes > 0 && !x0) || (n_cells > 0 && !cells)) return HL_E_INVALID;
    if (n_cells * (dim + 1) >= (int64_t)INT32_MAX || n_nodes >= (int64_t)INT32_MAX) return HL_E_INVALID;
    const int nv = dim + 1;
    for (int64_t q = 0; q < n_cells * nv; ++q)
        if (cells[q] < 0 || cells[q] >= n_nodes) return HL_E_INVALID;
    for (int64_t i = 0; i < n_nodes * dim; ++i)
        if (!std::isfinite(x0[i])) return HL_E_INVALID;
    for (int64_t cc = 0; cc < n_cells; ++cc) {
        double X[12];
        for (int k = 0; k < nv; ++k)
            for (int i = 0; i < dim; ++i) X[k * dim + i] = x0[(size_t)cells[cc * nv + k] * dim + i];
        if (!(host_volume(dim, X) > 0.0)) return HL_E_DEGENERATE_CELL;
    }
    return hl::check_conforming(dim, x0, cells, 0, n_nodes, 0, n_cells);
}

hl_status hl_mesh_info(hl_ctx *c, int *dim, int64_t *n_nodes, int64_t *n_cells) {
    if (!c) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (dim) *dim = c->dim;
    if (n_nodes) *n_nodes = c->nn;
    if (n_cells) *n_cells = c->nc;
    return HL_OK;
}

hl_status hl_mesh_get(hl_ctx *c, double *x, int32_t *cells, uint8_t *nwall, double *normals, int on_device) {
    if (!c) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    const hipMemcpyKind k = on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    auto put = [&](void *dst, const void *src, size_t bytes) -> hl_status {
        if (!dst || !bytes) return HL_OK;
        if (on_device) {
            HIPCHK(hipMemcpy(dst, src, bytes, k));
        } else {
            std::memcpy(dst, src, bytes);
        }
        return HL_OK;
    };
    hl_status st;
    HostMesh h;
    user_mesh(c, h);
    if ((st = put(x, h.x.data(), sizeof(double) * h.x.size())) != HL_OK) return st;
    if ((st = put(cells, h.cells.data(), sizeof(int32_t) * h.cells.size())) != HL_OK) return st;
    if ((st = put(nwall, h.nw.data(), h.nw.size())) != HL_OK) return st;
    return put(normals, h.nrm.data(), sizeof(double) * h.nrm.size());
}

hl_status hl_set_params(hl_ctx *c, const hl_params *p) {
    if (!c || !p || !params_valid(*p)) return HL_E_INVALID;
    c->prm = *p;
    drop_graphs(c);
    return HL_OK;
}

hl_status hl_set_boundary_loads(hl_ctx *c, int64_t n, const int32_t *cell, const uint8_t *face, const uint8_t *kind,
                                const double *value, int on_device) {
    if (!c || n < 0) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (n > 0 && (!cell || !face || !kind || !value)) return HL_E_INVALID;
    if (n >= (int64_t)INT32_MAX / 3) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    const int d = c->dim, nv = d + 1;
    std::vector<int32_t> hc(n);
    std::vector<uint8_t> hf(n), hk(n);
    std::vector<double> hv(6 * n);
    if (n > 0 && on_device) {
        HIPCHK(hipMemcpy(hc.data(), cell, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hf.data(), face, n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hk.data(), kind, n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hv.data(), value, sizeof(double) * 6 * n, hipMemcpyDeviceToHost));
    } else if (n > 0) {
        std::memcpy(hc.data(), cell, sizeof(int32_t) * n);
        std::memcpy(hf.data(), face, n);
        std::memcpy(hk.data(), kind, n);
        std::memcpy(hv.data(), value, sizeof(double) * 6 * n);
    }
    for (int64_t l = 0; l < n; ++l) {
        if (hc[l] < 0 || hc[l] >= c->nc || hf[l] > d || (hk[l] != 1 && hk[l] != 2)) return HL_E_INVALID;
        for (int q = 0; q < 6; ++q)
            if (!std::isfinite(hv[6 * l + q])) return HL_E_INVALID;
    }
    if (c->permuted)
        for (int64_t l = 0; l < n; ++l) hc[l] = c->c_u2i[hc[l]];  // the local face index is kept
    // entries grouped by node, each node's in the order of l
    const int64_t nn = c->nn;
    std::vector<int32_t> off(nn + 1, 0);
    for (int64_t l = 0; l < n; ++l)
        for (int j = 0; j < nv; ++j)
            if (j != hf[l]) ++off[c->c2n_host[(size_t)hc[l] * nv + j] + 1];
    for (int64_t p = 0; p < nn; ++p) off[p + 1] += off[p];
    const int64_t ne = off[nn];
    std::vector<int32_t> pos(off.begin(), off.end() - 1), ec(ne);
    std::vector<uint8_t> efk(ne);
    std::vector<double> ev(6 * ne);
    for (int64_t l = 0; l < n; ++l)
        for (int j = 0; j < nv; ++j) {
            if (j == hf[l]) continue;
            const int32_t q = pos[c->c2n_host[(size_t)hc[l] * nv + j]]++;
            ec[q] = hc[l];
            efk[q] = (uint8_t)(hf[l] | (hk[l] << 2));
            for (int t = 0; t < 6; ++t) ev[6 * (size_t)q + t] = hv[6 * l + t];
        }
    drop_graphs(c);
    free_tape(c);
    free_loads(c);
    if (n == 0) return HL_OK;
    auto get = [&](void **p, size_t bytes) -> bool {
        if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
        c->ld.mem.push_back(*p);
        return true;
    };
    if (!get((void **)&c->ld.off, sizeof(int32_t) * (nn + 1)) || !get((void **)&c->ld.cell, sizeof(int32_t) * ne) ||
        !get((void **)&c->ld.fk, ne) || !get((void **)&c->ld.val, sizeof(double) * 6 * ne)) {
        free_loads(c);
        return HL_E_OOM;
    }
    hipStream_t s = c->stream;
    hipError_t e = hipMemcpyAsync(c->ld.off, off.data(), sizeof(int32_t) * (nn + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->ld.cell, ec.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->ld.fk, efk.data(), ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->ld.val, ev.data(), sizeof(double) * 6 * ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_loads(c);
        return hip_fail(e, "boundary load upload", __LINE__);
    }
    c->ld.n = n;
    return HL_OK;
}

hl_status hl_set_contact(hl_ctx *c, int64_t n, const int32_t *nodes, const double *point, const double *normal,
                         int on_device) {
    if (!c || n < 0) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (n > 0 && (!nodes || !point || !normal || c->n_mesh != 1)) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    const int d = c->dim, dd = d * d;
    const int64_t nn = c->nn;
    std::vector<int32_t> nd(n);
    double xT[3] = {0, 0, 0}, nr[3] = {0, 0, 0};
    if (n > 0) {
        if (on_device)
            HIPCHK(hipMemcpy(nd.data(), nodes, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        else
            std::memcpy(nd.data(), nodes, sizeof(int32_t) * n);
        std::vector<char> seen(nn, 0);
        for (int64_t i = 0; i < n; ++i) {
            if (nd[i] < 0 || nd[i] >= nn || seen[nd[i]]) return HL_E_INVALID;
            seen[nd[i]] = 1;
        }
        if (c->permuted)
            for (int64_t i = 0; i < n; ++i) nd[i] = c->n_u2i[nd[i]];
        double l = 0.0;
        for (int i = 0; i < d; ++i) {
            xT[i] = point[i];
            nr[i] = normal[i];
            if (!std::isfinite(xT[i]) || !std::isfinite(nr[i])) return HL_E_INVALID;
            l += nr[i] * nr[i];
        }
        l = std::sqrt(l);
        if (!(l > 0.0)) return HL_E_INVALID;
        for (int i = 0; i < d; ++i) nr[i] /= l;
    }
    // release the previous candidates to their own walls
    if (c->ct.n > 0) {
        std::fill(c->ct.state_h.begin(), c->ct.state_h.end(), 0);
        hl_status st = contact_apply(c);
        if (st != HL_OK) return st;
    }
    drop_graphs(c);
    free_tape(c);
    free_contact(c);
    if (n == 0) return HL_OK;
    // own allowed directions of each candidate, and those left when the
    // plane's normal is added (Gram-Schmidt of the own basis against the
    // normal's projection on it; a projection below 1e-8 adds nothing)
    std::vector<uint8_t> nal_all(nn);
    std::vector<double> alw_all((size_t)nn * dd);
    HIPCHK(hipMemcpy(nal_all.data(), c->nallow, nn, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(alw_all.data(), c->allow, sizeof(double) * nn * dd, hipMemcpyDeviceToHost));
    std::vector<uint8_t> nal0(n), nal1(n);
    std::vector<double> alw0((size_t)n * dd), alw1((size_t)n * dd, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t p = nd[i];
        const int na = nal_all[p];
        const double *P = alw_all.data() + p * dd;
        nal0[i] = (uint8_t)na;
        std::copy(P, P + dd, alw0.begin() + i * dd);
        double u[3] = {0, 0, 0}, lu = 0.0;
        for (int t = 0; t < na; ++t) {
            double s = 0.0;
            for (int j = 0; j < d; ++j) s += P[j * d + t] * nr[j];
            for (int j = 0; j < d; ++j) u[j] += s * P[j * d + t];
        }
        for (int j = 0; j < d; ++j) lu += u[j] * u[j];
        lu = std::sqrt(lu);
        if (lu < 1e-8) {
            nal1[i] = (uint8_t)na;
            std::copy(P, P + dd, alw1.begin() + i * dd);
            continue;
        }
        for (int j = 0; j < d; ++j) u[j] /= lu;
        double Q[3][3];
        int nq = 0;
        for (int t = 0; t < na && nq < na - 1; ++t) {
            double w[3] = {0, 0, 0};
            for (int j = 0; j < d; ++j) w[j] = P[j * d + t];
            double s = 0.0;
            for (int j = 0; j < d; ++j) s += w[j] * u[j];
            for (int j = 0; j < d; ++j) w[j] -= s * u[j];
            for (int q = 0; q < nq; ++q) {
                double r = 0.0;
                for (int j = 0; j < d; ++j) r += w[j] * Q[q][j];
                for (int j = 0; j < d; ++j) w[j] -= r * Q[q][j];
            }
            double lw = 0.0;
            for (int j = 0; j < d; ++j) lw += w[j] * w[j];
            lw = std::sqrt(lw);
            if (lw < 1e-8) continue;
            for (int j = 0; j < d; ++j) Q[nq][j] = w[j] / lw;
            ++nq;
        }
        nal1[i] = (uint8_t)nq;
        for (int q = 0; q < nq; ++q)
            for (int j = 0; j < d; ++j) alw1[i * dd + j * d + q] = Q[q][j];
    }
    auto get = [&](void **p, size_t bytes) -> bool {
        if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
        c->ct.mem.push_back(*p);
        return true;
    };
    auto &ct = c->ct;
    if (!get((void **)&ct.node, sizeof(int32_t) * n) || !get((void **)&ct.state, n) ||
        !get((void **)&ct.nal[0], n) || !get((void **)&ct.nal[1], n) ||
        !get((void **)&ct.alw[0], sizeof(double) * n * dd) || !get((void **)&ct.alw[1], sizeof(double) * n * dd) ||
        !get((void **)&ct.out, sizeof(double) * 2 * n)) {
        free_contact(c);
        return HL_E_OOM;
    }
    hipStream_t s = c->stream;
    hipError_t e = hipMemcpyAsync(ct.node, nd.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ct.nal[0], nal0.data(), n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ct.nal[1], nal1.data(), n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ct.alw[0], alw0.data(), sizeof(double) * n * dd, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ct.alw[1], alw1.data(), sizeof(double) * n * dd, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_contact(c);
        return hip_fail(e, "contact upload", __LINE__);
    }
    ct.n = n;
    ct.state_h.assign(n, 0);
    for (int i = 0; i < 3; ++i) {
        ct.xT[i] = xT[i];
        ct.nrm[i] = nr[i];
    }
    return contact_apply(c);
}

hl_status hl_get_contact(hl_ctx *c, uint8_t *state, int64_t n) {
    if (!c || n != c->ct.n || (n > 0 && !state)) return HL_E_INVALID;
    if (n > 0) std::memcpy(state, c->ct.state_h.data(), n);
    return HL_OK;
}

hl_status hl_state_init(hl_ctx *c, const double *rho0, const double *mu, const double *lam, const double *v_cell,
                        const double *v_node, const hl_params *p, int on_device) {
    if (!c) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    if (c->ct.n > 0) {  // a new state starts with every contact candidate free
        std::fill(c->ct.state_h.begin(), c->ct.state_h.end(), 0);
        hl_status st = contact_apply(c);
        if (st != HL_OK) return st;
    }
    const int d = c->dim, nv = d + 1, nB = d == 3 ? 6 : 3;
    const size_t nc = (size_t)c->nc, nn = (size_t)c->nn;
    std::vector<double> r, m_, l, vc, vn;
    hl_status st;
    if ((st = to_host(rho0, nc, on_device, r)) != HL_OK) return st;
    if ((st = to_host(mu, nc, on_device, m_)) != HL_OK) return st;
    if ((st = to_host(lam, nc, on_device, l)) != HL_OK) return st;
    if ((st = to_host(v_cell, nc * d, on_device, vc)) != HL_OK) return st;
    if ((st = to_host(v_node, nn * d, on_device, vn)) != HL_OK) return st;
    for (size_t i = 0; i < nc; ++i)
        if (!(r[i] > 0) || !(m_[i] >= 0) || !std::isfinite(l[i])) return HL_E_INVALID;
    if (c->permuted) {
        // the caller's numbering -> the internal one
        auto perm_rows = [](std::vector<double> &a, const std::vector<int32_t> &i2u, int w) {
            std::vector<double> o(a.size());
            for (size_t i = 0; i < i2u.size(); ++i)
                for (int k = 0; k < w; ++k) o[i * w + k] = a[(size_t)i2u[i] * w + k];
            a.swap(o);
        };
        perm_rows(r, c->c_i2u, 1);
        perm_rows(m_, c->c_i2u, 1);
        perm_rows(l, c->c_i2u, 1);
        perm_rows(vc, c->c_i2u, d);
        perm_rows(vn, c->n_i2u, d);
    }
    hl_params prm = p ? *p : default_params(d);
    if (!params_valid(prm)) return HL_E_INVALID;

    std::vector<double> mass(nc), K(nc), tau(nc), e(nc), vs(nc * d), Bs(nc * nB, 0.0), vh(nn * d);
    for (size_t cc = 0; cc < nc; ++cc) {
        double X[12];
        for (int k = 0; k < nv; ++k)
            for (int i = 0; i < d; ++i) X[k * d + i] = c->x0_host[(size_t)c->c2n_host[cc * nv + k] * d + i];
        mass[cc] = r[cc] * host_volume(d, X);
        K[cc] = l[cc] + 2.0 * m_[cc] / 3.0;
        tau[cc] = 1.0 / r[cc];
        double k2 = 0.0;
        for (int i = 0; i < d; ++i) {
            vs[i * nc + cc] = vc[cc * d + i];
            k2 += vc[cc * d + i] * vc[cc * d + i];
        }
        e[cc] = 0.5 * k2;
        // stiffened gas at rest pressure p = 0: eps = gamma p_inf tau / (gamma - 1)
        if (prm.eos == 1) e[cc] += prm.sg_gamma * prm.sg_pinf * tau[cc] / (prm.sg_gamma - 1.0);
        for (int s = 0; s < d; ++s) Bs[s * nc + cc] = 1.0;  // diagonal comps first
    }
    // carried node velocity projected on the allowed directions
    std::vector<uint8_t> nal(nn);
    std::vector<double> alw(nn * d * d);
    if (nn) {
        HIPCHK(hipMemcpy(nal.data(), c->nallow, nn, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(alw.data(), c->allow, sizeof(double) * nn * d * d, hipMemcpyDeviceToHost));
    }
    for (size_t pp = 0; pp < nn; ++pp) {
        const double *P = alw.data() + pp * d * d;
        double o[3] = {0, 0, 0};
        for (int t = 0; t < nal[pp]; ++t) {
            double s = 0;
            for (int i = 0; i < d; ++i) s += P[i * d + t] * vn[pp * d + i];
            for (int i = 0; i < d; ++i) o[i] += s * P[i * d + t];
        }
        for (int i = 0; i < d; ++i) vh[i * nn + pp] = o[i];
    }
    hipStream_t s = c->stream;
    // restore positions to the uploaded mesh
    std::vector<double> xs(nn * d);
    for (size_t pp = 0; pp < nn; ++pp)
        for (int i = 0; i < d; ++i) xs[i * nn + pp] = c->x0_host[pp * d + i];
    c->cur = 0;
    HIPCHK(hipMemcpyAsync(c->x[0], xs.data(), sizeof(double) * nn * d, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->mass, mass.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->rho0, r.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->mu, m_.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->K, K.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->tau[0], tau.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->e[0], e.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->v[0], vs.data(), sizeof(double) * nc * d, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->B[0], Bs.data(), sizeof(double) * nc * nB, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->vhat[0], vh.data(), sizeof(double) * nn * d, hipMemcpyHostToDevice, s));
    if (nc) HIPCHK(hipMemsetAsync(c->mask, 0, nc, s));
    if (nn) HIPCHK(hipMemsetAsync(c->vstar, 0, sizeof(double) * nn * d, s));
    HIPCHK(hipStreamSynchronize(s));
    c->prm = prm;
    drop_graphs(c);
    c->have_state = true;
    c->rec_valid = false;
    double dt0;
    return hl_compute_dt(c, &dt0);
}

}  // extern "C"

namespace {

// State snapshot: this header, then the state (x, vhat [D][nn]; tau [nc];
// v [D][nc]; e [nc]; B [nB][nc]), the material (mass, rho0, mu, K [nc]),
// dt_cur and dt_next [n_mesh] as doubles in the internal numbering, the
// cascade levels [nc] and the contact states [n_contact] as bytes.
struct SnapHeader {
    uint64_t magic;
    uint64_t mesh_hash;
    int32_t dim, n_mesh;
    int64_t nn, nc, n_contact, bytes;
    hl_params prm;
};
constexpr uint64_t kSnapMagic = 0x3170616e53676c48ull;

size_t snap_doubles(const hl_ctx *c) {
    const size_t d = c->dim, nn = c->nn, nc = c->nc, nB = d == 3 ? 6 : 3;
    return 2 * d * nn + (2 + d + nB) * nc + 4 * nc + 2 * (size_t)c->n_mesh;
}

size_t snap_bytes(const hl_ctx *c) {
    return sizeof(SnapHeader) + sizeof(double) * snap_doubles(c) + (size_t)c->nc + (size_t)c->ct.n;
}

// device arrays of a snapshot in blob order, with their lengths in doubles
int snap_parts(hl_ctx *c, double **ptr, size_t *len) {
    const size_t d = c->dim, nn = c->nn, nc = c->nc, nB = d == 3 ? 6 : 3;
    const int b = c->cur;
    double *p[12] = {c->x[b], c->vhat[b], c->tau[b], c->v[b], c->e[b], c->B[b],
                     c->mass, c->rho0, c->mu, c->K, c->dt_cur, c->dt_next};
    const size_t l[12] = {d * nn, d * nn, nc, d * nc, nc, nB * nc, nc, nc, nc, nc, (size_t)c->n_mesh,
                          (size_t)c->n_mesh};
    for (int k = 0; k < 12; ++k) {
        ptr[k] = p[k];
        len[k] = l[k];
    }
    return 12;
}

}  // namespace

extern "C" {

hl_status hl_state_save(hl_ctx *c, void *blob, int64_t *bytes) {
    if (!c || !bytes) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    const int64_t need = (int64_t)snap_bytes(c);
    if (!blob) {
        *bytes = need;
        return HL_OK;
    }
    if (*bytes < need) {
        *bytes = need;
        return HL_E_INVALID;
    }
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    hipStream_t s = c->stream;
    SnapHeader h{};
    h.magic = kSnapMagic;
    h.mesh_hash = c->mesh_hash;
    h.dim = c->dim;
    h.n_mesh = c->n_mesh;
    h.nn = c->nn;
    h.nc = c->nc;
    h.n_contact = c->ct.n;
    h.bytes = need;
    h.prm = c->prm;
    char *o = static_cast<char *>(blob);
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    double *ptr[12];
    size_t len[12];
    const int np = snap_parts(c, ptr, len);
    for (int k = 0; k < np; ++k) {
        if (len[k]) HIPCHK(hipMemcpyAsync(o, ptr[k], sizeof(double) * len[k], hipMemcpyDeviceToHost, s));
        o += sizeof(double) * len[k];
    }
    if (c->nc) HIPCHK(hipMemcpyAsync(o, c->mask, (size_t)c->nc, hipMemcpyDeviceToHost, s));
    o += c->nc;
    HIPCHK(hipStreamSynchronize(s));
    if (c->ct.n) std::memcpy(o, c->ct.state_h.data(), (size_t)c->ct.n);
    *bytes = need;
    return HL_OK;
}

hl_status hl_state_restore(hl_ctx *c, const void *blob, int64_t bytes) {
    if (!c || !blob) return HL_E_INVALID;
    if (!c->have_mesh) return HL_E_STATE;
    if (bytes < (int64_t)sizeof(SnapHeader)) return HL_E_INVALID;
    SnapHeader h;
    std::memcpy(&h, blob, sizeof h);
    if (h.magic != kSnapMagic || h.mesh_hash != c->mesh_hash || h.dim != c->dim || h.n_mesh != c->n_mesh ||
        h.nn != c->nn || h.nc != c->nc || h.n_contact != c->ct.n || h.bytes != bytes ||
        bytes != (int64_t)snap_bytes(c) || !params_valid(h.prm)) {
        std::snprintf(g_last_error, sizeof g_last_error, "the snapshot does not belong to the held mesh");
        return HL_E_INVALID;
    }
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    hipStream_t s = c->stream;
    c->cur = 0;
    const char *o = static_cast<const char *>(blob) + sizeof h;
    double *ptr[12];
    size_t len[12];
    const int np = snap_parts(c, ptr, len);
    for (int k = 0; k < np; ++k) {
        if (len[k]) HIPCHK(hipMemcpyAsync(ptr[k], o, sizeof(double) * len[k], hipMemcpyHostToDevice, s));
        o += sizeof(double) * len[k];
    }
    if (c->nc) HIPCHK(hipMemcpyAsync(c->mask, o, (size_t)c->nc, hipMemcpyHostToDevice, s));
    o += c->nc;
    HIPCHK(hipStreamSynchronize(s));
    if (c->ct.n) {
        std::memcpy(c->ct.state_h.data(), o, (size_t)c->ct.n);
        hl_status st = contact_apply(c);
        if (st != HL_OK) return st;
    }
    // captured steps stay valid unless the parameters change (they hold
    // them by value; the state goes to buffer 0, which has its own graph)
    if (std::memcmp(&c->prm, &h.prm, sizeof(hl_params)) != 0) drop_graphs(c);
    c->prm = h.prm;
    c->have_state = true;
    c->rec_valid = false;
    return HL_OK;
}

hl_status hl_compute_dt(hl_ctx *c, double *dt_out) {
    if (!c) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    hipStream_t s = c->stream;
    hl::StepArgs a = make_args(c, c->cur);
    a.tau = c->tau[c->cur];
    if (c->dim == 3)
        hl::launch_acoustic<3>(a, s);
    else
        hl::launch_acoustic<2>(a, s);
    hl::launch_dt_reduce(c->nc, c->dtc, c->cell_mesh, c->pstat, c->dt_red, c->dt_part, c->mesh_cell_off, c->n_mesh,
                         c->counters + hl::CNT_N - 1, s);
    hl::launch_dt_finalize(c->n_mesh, c->dt_red, c->dt_cur, c->prm, 1, c->dt_next, c->dt_parts, s);
    double dt = 0.0;
    HIPCHK(hipMemcpyAsync(&dt, c->dt_next, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (dt_out) *dt_out = dt;
    return HL_OK;
}

static hl_status step_common(hl_ctx *c, double dt, const uint8_t *mask, int on_device, hl_step_info *info) {
    if (!c) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (!std::isfinite(dt)) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    if (mask && c->permuted && c->nc) {
        // the caller's cascade choice, gathered into the internal order
        uint8_t *tmp = reinterpret_cast<uint8_t *>(c->scratch);
        HIPCHK(hipMemcpyAsync(tmp, mask, (size_t)c->nc, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              c->stream));
        hl::launch_gather_u8(c->nc, tmp, c->d_c_i2u, c->mask_in, c->stream);
        mask = c->mask_in;
        on_device = 1;
    }
    hl_status st;
    if (c->ct.n > 0 && !mask && c->nc > 0)
        st = c->dim == 3 ? contact_step<3>(c, dt, info) : contact_step<2>(c, dt, info);
    else
        st = c->dim == 3 ? run_step<3>(c, dt, mask, on_device, info) : run_step<2>(c, dt, mask, on_device, info);
    if (c->prof.on) prof_collect(c);
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return hip_fail(le, "kernel launch", __LINE__);
    return st;
}

hl_status hl_step(hl_ctx *c, double dt, hl_step_info *info) { return step_common(c, dt, nullptr, 0, info); }

hl_status hl_step_batch(hl_ctx *c, const double *dt_per_mesh, int on_device, hl_step_info *info) {
    if (!c) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (!dt_per_mesh) return step_common(c, 0.0, nullptr, 0, info);
    std::vector<double> h;
    hl_status st = to_host(dt_per_mesh, (size_t)c->n_mesh, on_device, h);
    if (st != HL_OK) return st;
    for (double d : h)
        if (!(d > 0.0) || !std::isfinite(d)) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    HIPCHK(hipMemcpyAsync(c->dt_next, h.data(), sizeof(double) * c->n_mesh, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return step_common(c, 0.0, nullptr, 0, info);
}

hl_status hl_query_dt(hl_ctx *c, double *dt_next, int n_meshes, int on_device) {
    if (!c || !dt_next) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (n_meshes != c->n_mesh) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    HIPCHK(hipMemcpyAsync(dt_next, c->dt_next, sizeof(double) * c->n_mesh,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return HL_OK;
}

hl_status hl_step_replay(hl_ctx *c, double dt, const uint8_t *mask, int on_device, hl_step_info *info) {
    if (!mask && c && c->nc) return HL_E_INVALID;
    return step_common(c, dt, mask, on_device, info);
}

hl_status hl_query(hl_ctx *c, int field, void *out, int64_t count, int on_device) {
    if (!c || !out) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    bool node, u8;
    int w = field_width(c, field, &node, &u8);
    if (w < 0) return HL_E_INVALID;
    const int64_t n = node ? c->nn : c->nc;
    if (count != n * w) return HL_E_INVALID;
    hipStream_t s = c->stream;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (n == 0) return HL_OK;
    // row i of the output is internal entity idx[i] (null: i)
    const int32_t *idx = c->permuted ? (node ? c->d_n_u2i : c->d_c_u2i) : nullptr;
    if (u8) {
        if (idx) {
            hl::launch_gather_u8(n, c->mask, idx, reinterpret_cast<uint8_t *>(c->scratch), s);
            HIPCHK(hipMemcpyAsync(out, c->scratch, (size_t)n, k, s));
        } else {
            HIPCHK(hipMemcpyAsync(out, c->mask, (size_t)n, k, s));
        }
    } else if (field == HL_T) {
        hl::StepArgs a = make_args(c, c->cur);
        if (c->dim == 3)
            hl::launch_stress_query<3>(a, idx, c->scratch, s);
        else
            hl::launch_stress_query<2>(a, idx, c->scratch, s);
        HIPCHK(hipMemcpyAsync(out, c->scratch, sizeof(double) * n * w, k, s));
    } else {
        double *src = field_ptr(c, field);
        if (w == 1 && !idx) {
            HIPCHK(hipMemcpyAsync(out, src, sizeof(double) * n, k, s));
        } else {
            hl::launch_soa_to_aos(n, w, src, c->scratch, s, idx);
            HIPCHK(hipMemcpyAsync(out, c->scratch, sizeof(double) * n * w, k, s));
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    return HL_OK;
}

hl_status hl_upload_field(hl_ctx *c, int field, const void *in, int64_t count, int on_device) {
    if (!c || !in) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (field != HL_X && field != HL_VHAT && field != HL_TAU && field != HL_V && field != HL_E && field != HL_B)
        return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    bool node, u8;
    int w = field_width(c, field, &node, &u8);
    const int64_t n = node ? c->nn : c->nc;
    if (count != n * w) return HL_E_INVALID;
    if (n == 0) return HL_OK;
    hipStream_t s = c->stream;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    double *dst = field_ptr(c, field);
    c->rec_valid = false;
    const int32_t *idx = c->permuted ? (node ? c->d_n_u2i : c->d_c_u2i) : nullptr;
    if (w == 1 && !idx) {
        HIPCHK(hipMemcpyAsync(dst, in, sizeof(double) * n, k, s));
    } else {
        HIPCHK(hipMemcpyAsync(c->scratch, in, sizeof(double) * n * w, k, s));
        hl::launch_aos_to_soa(n, w, c->scratch, dst, s, idx);
    }
    HIPCHK(hipStreamSynchronize(s));
    return HL_OK;
}

hl_status hl_forward_record(hl_ctx *c, int nsteps, int ckpt_every) {
    g_last_error[0] = '\0';
    if (!c || nsteps < 1 || ckpt_every < 1) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (c->prm.cascade == 3 || c->prm.shear_a != -1.0 || c->prm.eos != 0 || c->ld.n > 0 || c->ct.n > 0) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "the adjoint covers the two-level cascade and the neo-Hookean law without boundary loads "
                      "or contact (cascade 2, shear_a -1, eos 0)");
        return HL_E_INVALID;
    }
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    const bool prof = c->prof.on, graph = c->graph_on;
    c->prof.on = false;
    c->graph_on = false;
    hl_status st = c->dim == 3 ? forward_record<3>(c, nsteps, ckpt_every) : forward_record<2>(c, nsteps, ckpt_every);
    c->prof.on = prof;
    c->graph_on = graph;
    if (st != HL_OK) free_tape(c);
    return st;
}

hl_status hl_forward_replay(hl_ctx *c) {
    if (!c) return HL_E_INVALID;
    if (!c->have_state || c->tape.nsteps == 0) return HL_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    return c->dim == 3 ? forward_replay<3>(c) : forward_replay<2>(c);
}

hl_status hl_adjoint_run(hl_ctx *c, const double *dL_dx_final, double *dL_dmu, double *dL_dvcell,
                         double *dL_dvnode, int on_device) {
    g_last_error[0] = '\0';
    if (!c || !dL_dx_final || !dL_dmu || !dL_dvcell || !dL_dvnode) return HL_E_INVALID;
    if (!c->have_state || c->tape.nsteps == 0) return HL_E_STATE;
    if (c->prm.cascade == 3 || c->prm.shear_a != -1.0 || c->prm.eos != 0) {
        // parameters changed since the recording to ones the adjoint does
        // not cover (the replays would also write aggregates the tape has
        // no room for)
        std::snprintf(g_last_error, sizeof g_last_error,
                      "the adjoint covers the two-level cascade and the neo-Hookean law (cascade 2, shear_a -1, "
                      "eos 0); the parameters were changed after the recording");
        return HL_E_INVALID;
    }
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    return c->dim == 3 ? adjoint_run<3>(c, dL_dx_final, dL_dmu, dL_dvcell, dL_dvnode, on_device)
                       : adjoint_run<2>(c, dL_dx_final, dL_dmu, dL_dvcell, dL_dvnode, on_device);
}

hl_status hl_tape_get(hl_ctx *c, int step, uint8_t *mask, double *dt) {
    if (!c || step < 0 || step >= c->tape.nsteps) return HL_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    if (mask && c->nc) {
        if (c->permuted) {
            std::vector<uint8_t> tmp((size_t)c->nc);
            HIPCHK(hipMemcpy(tmp.data(), c->tape.masks + (size_t)step * c->nc, (size_t)c->nc, hipMemcpyDeviceToHost));
            for (int64_t u = 0; u < c->nc; ++u) mask[u] = tmp[(size_t)c->c_u2i[u]];
        } else {
            HIPCHK(hipMemcpy(mask, c->tape.masks + (size_t)step * c->nc, (size_t)c->nc, hipMemcpyDeviceToHost));
        }
    }
    if (dt)
        HIPCHK(hipMemcpy(dt, c->tape.dts + (size_t)step * c->n_mesh, sizeof(double) * c->n_mesh,
                         hipMemcpyDeviceToHost));
    return HL_OK;
}

hl_status hl_use_graph(hl_ctx *c, int on, int max_mood_passes) {
    if (!c || max_mood_passes < 0 || max_mood_passes > 64) return HL_E_INVALID;
    if (c->graph_passes != max_mood_passes || !on) drop_graphs(c);
    c->graph_on = on != 0;
    c->graph_passes = max_mood_passes;
    return HL_OK;
}

hl_status hl_set_schedule(hl_ctx *c, int stage, const hl_schedule *sch) {
    if (!c || !sch || stage < 0 || stage >= HL_STAGE_COUNT) return HL_E_INVALID;
    StageCfg g;
    g.tile = sch->tile;
    g.block = sch->block;
    g.blocks_per_cu = sch->blocks_per_cu;
    if (!cfg_valid(g)) return HL_E_INVALID;
    c->cfg[stage] = g;
    c->cfg_set[stage] = true;
    c->sched_ready = false;
    drop_graphs(c);
    return HL_OK;
}

hl_status hl_get_schedule(hl_ctx *c, int stage, hl_schedule *sch) {
    if (!c || !sch || stage < 0 || stage >= HL_STAGE_COUNT) return HL_E_INVALID;
    const StageCfg g = stage == HL_STAGE_PREDICT && !c->cfg_set[stage] ? predict_default(c) : c->cfg[stage];
    sch->tile = g.tile;
    sch->block = g.block;
    sch->blocks_per_cu = g.blocks_per_cu;
    sch->reserved = 0;
    return HL_OK;
}

hl_status hl_autotune(hl_ctx *c, int reps, double *best_ms) {
    if (!c || reps < 1 || reps > 100) return HL_E_INVALID;
    if (!c->have_state) return HL_E_STATE;
    if (hipSetDevice(c->device) != hipSuccess) return HL_E_HIP;
    if (c->nc == 0) return HL_OK;
    return c->dim == 3 ? autotune<3>(c, reps, best_ms) : autotune<2>(c, reps, best_ms);
}

hl_status hl_profile_enable(hl_ctx *c, int on) {
    if (!c) return HL_E_INVALID;
    if (!on && c->prof.on) prof_collect(c);
    c->prof.on = on != 0;
    return HL_OK;
}

hl_status hl_profile_reset(hl_ctx *c) {
    if (!c) return HL_E_INVALID;
    prof_collect(c);
    for (int k = 0; k < PK_COUNT; ++k) {
        c->prof.total_ms[k] = 0.0;
        c->prof.count[k] = 0;
    }
    return HL_OK;
}

hl_status hl_profile_get(hl_ctx *c, const char *name, double *avg_ms, int64_t *launches) {
    if (!c || !name) return HL_E_INVALID;
    prof_collect(c);
    for (int k = 0; k < PK_COUNT; ++k) {
        if (std::strcmp(name, kProfNames[k]) == 0) {
            if (launches) *launches = c->prof.count[k];
            if (avg_ms) *avg_ms = c->prof.count[k] ? c->prof.total_ms[k] / (double)c->prof.count[k] : 0.0;
            return HL_OK;
        }
    }
    return HL_E_INVALID;
}

}  // extern "C"

// ------------------------------------------------------------------ groups
// A 2D and a 3D context stepped together: every stage, MOOD pass and CFL
// reduction of the two runs as one paired launch (hl::launch_*_pair), so a
// family of meshes of both dimensions costs the launches of one context.
struct hl_group {
    hl_ctx *c[2] = {nullptr, nullptr};  // the 2D context, the 3D context
    bool graph_on = false;
    int graph_passes = 6;
    hipStream_t cap_stream = nullptr;
    // captured step per (buffer parity of c[0], of c[1]), with the
    // contexts' generations it was captured at
    hipGraph_t graph[2][2] = {};
    hipGraphExec_t gexec[2][2] = {};
    uint64_t gen[2][2][2] = {};
    // continuation: CONT_PASSES more paired passes, per buffer parities and
    // parity of the input flag lists
    hipGraph_t cgraph[2][2][2] = {};
    hipGraphExec_t cexec[2][2][2] = {};
    uint64_t cgen[2][2][2][2] = {};
};

namespace {

void group_drop_graphs(hl_group *g) {
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            if (g->gexec[i][j]) (void)hipGraphExecDestroy(g->gexec[i][j]);
            if (g->graph[i][j]) (void)hipGraphDestroy(g->graph[i][j]);
            g->gexec[i][j] = nullptr;
            g->graph[i][j] = nullptr;
            for (int f = 0; f < 2; ++f) {
                if (g->cexec[i][j][f]) (void)hipGraphExecDestroy(g->cexec[i][j][f]);
                if (g->cgraph[i][j][f]) (void)hipGraphDestroy(g->cgraph[i][j][f]);
                g->cexec[i][j][f] = nullptr;
                g->cgraph[i][j][f] = nullptr;
            }
        }
}

// The configurations the paired kernels cover, and one launch shape per
// stage where both contexts have work.
hl_status group_check(hl_group *g) {
    const char *why = nullptr;
    for (int i = 0; i < 2 && !why; ++i) {
        const hl_ctx *c = g->c[i];
        if (!c->have_state)
            return HL_E_STATE;
        else if (c->nc == 0)
            why = "a grouped context holds no cells";
        else if (c->prm.shear_a != -1.0 || c->prm.eos != 0 || c->prm.cascade == 3)
            why = "grouped contexts run the neo-Hookean law with the two-level cascade";
        else if (c->ld.n > 0 || c->ct.n > 0)
            why = "grouped contexts take no boundary loads or contact";
    }
    if (!why && g->c[0]->prm.detect != g->c[1]->prm.detect) why = "grouped contexts differ in detection";
    if (!why && (g->c[0]->device != g->c[1]->device || g->c[0]->stream != g->c[1]->stream))
        why = "grouped contexts use one device and one stream";
    if (!why)
        for (int st = 0; st < HL_STAGE_COUNT; ++st)
            if (g->c[0]->sk[st].w.n_items && g->c[1]->sk[st].w.n_items &&
                g->c[0]->sk[st].block != g->c[1]->sk[st].block)
                why = "grouped contexts need one block size per stage";
    if (why) {
        std::snprintf(g_last_error, sizeof g_last_error, "%s", why);
        return HL_E_INVALID;
    }
    return HL_OK;
}

hl::PairBook pair_book(hl_ctx *c) {
    hl::PairBook b{};
    b.counters = c->counters;
    b.dt_cur = c->dt_cur;
    b.dt_next = c->dt_next;
    b.n_mesh = c->n_mesh;
    b.copy_dt = 1;
    b.mask = c->mask;
    b.nc = c->nc;
    b.dtc = c->dtc;
    b.cell_mesh = c->cell_mesh;
    b.pstat = c->pstat;
    b.red = c->dt_red;
    b.part = c->dt_part;
    b.parts = c->dt_parts;
    b.mesh_cell_off = c->mesh_cell_off;
    b.bad_count = c->counters + hl::CNT_BAD;
    b.c_cfl = c->prm.c_cfl;
    b.c_v = c->prm.c_v;
    b.c_i = c->prm.c_i;
    return b;
}

// the step's first part (enqueue_first of both contexts, clearing the masks)
void group_first(hl_group *g, hl::StepArgs a[2], hipStream_t s) {
    hl_ctx *c0 = g->c[0], *c1 = g->c[1];
    hl::launch_step_begin_pair(pair_book(c0), pair_book(c1), s);
    for (int i = 0; i < 2; ++i) {
        a[i].flist_out = g->c[i]->flist[0];
        a[i].fcount_out = g->c[i]->counters + hl::CNT_F0;
    }
    hl::launch_node_agg_pair(a[0], c0->sk[HL_STAGE_NODE_AGG], a[1], c1->sk[HL_STAGE_NODE_AGG], s);
    hl::launch_predict_pair(a[0], c0->sk[HL_STAGE_PREDICT], a[1], c1->sk[HL_STAGE_PREDICT], s);
    hl::launch_node_solve_pair(a[0], c0->sk[HL_STAGE_NODE_SOLVE], a[1], c1->sk[HL_STAGE_NODE_SOLVE], s);
    hl::launch_update_pair(a[0], c0->sk[HL_STAGE_UPDATE], a[1], c1->sk[HL_STAGE_UPDATE], s);
}

// one MOOD pass of both contexts reading flag list fb (a context with no
// flagged cell runs an empty pass: its lists and stamp move on, nothing else)
void group_pass(hl_group *g, hl::StepArgs a[2], int fb, int log_index, const int64_t nflag[2], bool fixed,
                hipStream_t s) {
    hl::PairPass p[2];
    for (int i = 0; i < 2; ++i) {
        hl_ctx *c = g->c[i];
        a[i].flist_out = c->flist[1 - fb];
        a[i].fcount_out = c->counters + hl::CNT_F0 + (1 - fb);
        p[i] = hl::PairPass{c->flist[fb], c->counters + hl::CNT_F0 + fb, nflag[i], c->max_deg,
                            log_index >= 0 ? c->pass_log : nullptr};
    }
    hl::launch_mood_sparse_pair(a[0], p[0], a[1], p[1], fixed, log_index >= 0 ? log_index : 0, s);
}

hl_status group_read_counters(hl_group *g, hipStream_t s) {
    for (int i = 0; i < 2; ++i)
        HIPCHK(hipMemcpyAsync(g->c[i]->counters_host, g->c[i]->counters, hl::CNT_N * sizeof(unsigned),
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HL_OK;
}

hl_status group_capture(hl_group *g, int s0, int s1) {
    if (!g->cap_stream) HIPCHK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = g->cap_stream;
    hl::StepArgs a[2] = {make_args(g->c[0], s0), make_args(g->c[1], s1)};
    const int64_t zero[2] = {0, 0};
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    group_first(g, a, cs);
    for (int p = 0; p < g->graph_passes; ++p) group_pass(g, a, p & 1, p, zero, true, cs);
    hl::launch_dt_reduce_pair(pair_book(g->c[0]), pair_book(g->c[1]), cs);
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamEndCapture(cs, &gr));
    g->graph[s0][s1] = gr;
    HIPCHK(hipGraphInstantiate(&g->gexec[s0][s1], gr, nullptr, nullptr, 0));
    g->gen[s0][s1][0] = g->c[0]->gen;
    g->gen[s0][s1][1] = g->c[1]->gen;
    return HL_OK;
}

// CONT_PASSES paired passes from input list parity fb, captured
hl_status group_capture_cont(hl_group *g, int s0, int s1, int fb) {
    if (!g->cap_stream) HIPCHK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = g->cap_stream;
    hl::StepArgs a[2] = {make_args(g->c[0], s0), make_args(g->c[1], s1)};
    const int64_t zero[2] = {0, 0};
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int p = 0; p < CONT_PASSES; ++p) group_pass(g, a, fb ^ (p & 1), 64 + p, zero, true, cs);
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamEndCapture(cs, &gr));
    g->cgraph[s0][s1][fb] = gr;
    HIPCHK(hipGraphInstantiate(&g->cexec[s0][s1][fb], gr, nullptr, nullptr, 0));
    g->cgen[s0][s1][fb][0] = g->c[0]->gen;
    g->cgen[s0][s1][fb][1] = g->c[1]->gen;
    return HL_OK;
}

hl_status group_step(hl_group *g, hl_step_info *info0, hl_step_info *info1) {
    hl_ctx *c[2] = {g->c[0], g->c[1]};
    hl_status st;
    for (int i = 0; i < 2; ++i)
        if ((st = ensure_scheds(c[i], c[1 - i])) != HL_OK) return st;
    if ((st = group_check(g)) != HL_OK) return st;
    if (hipSetDevice(c[0]->device) != hipSuccess) return HL_E_HIP;
    hipStream_t s = c[0]->stream;
    const int src[2] = {c[0]->cur, c[1]->cur};
    hl::StepArgs a[2] = {make_args(c[0], src[0]), make_args(c[1], src[1])};
    for (int i = 0; i < 2; ++i) {
        if (c[i]->stamp_host > INT32_MAX - 4096) {
            HIPCHK(hipMemsetAsync(c[i]->nstamp, 0, sizeof(int32_t) * c[i]->nn, s));
            HIPCHK(hipMemsetAsync(c[i]->cstamp, 0, sizeof(int32_t) * c[i]->nc, s));
            HIPCHK(hipMemsetAsync(c[i]->stamp_dev, 0, sizeof(int32_t), s));
            c[i]->stamp_host = 0;
        }
        if (!c[i]->rec_valid) {
            if (i == 0)
                hl::launch_centroids<2>(a[0], c[0]->sk[HL_STAGE_PACK], s);
            else
                hl::launch_centroids<3>(a[1], c[1]->sk[HL_STAGE_PACK], s);
            c[i]->rec_valid = true;
        }
    }
    const bool detect = a[0].detect != 0;
    int64_t nflag[2] = {0, 0}, first[2] = {0, 0};
    int iters[2] = {1, 1};
    int fb = 0;
    auto more = [&]() { return detect && (nflag[0] > 0 || nflag[1] > 0); };
    auto eager_passes = [&]() -> hl_status {
        while (more()) {
            group_pass(g, a, fb, -1, nflag, false, s);
            for (int i = 0; i < 2; ++i) {
                c[i]->stamp_host++;
                iters[i] += nflag[i] > 0;
            }
            hl_status r = group_read_counters(g, s);
            if (r != HL_OK) return r;
            fb = 1 - fb;
            for (int i = 0; i < 2; ++i) nflag[i] = c[i]->counters_host[hl::CNT_F0 + fb];
        }
        return HL_OK;
    };
    if (g->graph_on) {
        hipGraphExec_t &ge = g->gexec[src[0]][src[1]];
        if (ge && (g->gen[src[0]][src[1]][0] != c[0]->gen || g->gen[src[0]][src[1]][1] != c[1]->gen)) {
            (void)hipGraphExecDestroy(ge);
            (void)hipGraphDestroy(g->graph[src[0]][src[1]]);
            ge = nullptr;
            g->graph[src[0]][src[1]] = nullptr;
        }
        if (!ge && (st = group_capture(g, src[0], src[1])) != HL_OK) return st;
        HIPCHK(hipGraphLaunch(ge, s));
        const int np = std::min(g->graph_passes, 64);
        unsigned *log[2] = {c[0]->counters_host + hl::CNT_N, c[1]->counters_host + hl::CNT_N};  // pinned
        for (int i = 0; i < 2; ++i) {
            c[i]->stamp_host += g->graph_passes;
            if (np) HIPCHK(hipMemcpyAsync(log[i], c[i]->pass_log, sizeof(unsigned) * np, hipMemcpyDeviceToHost, s));
        }
        if ((st = group_read_counters(g, s)) != HL_OK) return st;
        fb = g->graph_passes & 1;
        for (int i = 0; i < 2; ++i) {
            nflag[i] = c[i]->counters_host[hl::CNT_F0 + fb];
            first[i] = np ? log[i][0] : nflag[i];
            for (int p = 0; p < np; ++p) iters[i] += log[i][p] > 0;
        }
        if (more()) {
            // the captured passes did not reach the fixpoint: captured blocks
            // of CONT_PASSES paired passes (a pass with no input exits at
            // once) until no cell is flagged, then the reduction again
            while (more()) {
                hipGraphExec_t &ce = g->cexec[src[0]][src[1]][fb];
                const uint64_t *cg = g->cgen[src[0]][src[1]][fb];
                if (ce && (cg[0] != c[0]->gen || cg[1] != c[1]->gen)) {
                    (void)hipGraphExecDestroy(ce);
                    (void)hipGraphDestroy(g->cgraph[src[0]][src[1]][fb]);
                    ce = nullptr;
                    g->cgraph[src[0]][src[1]][fb] = nullptr;
                }
                if (!ce && (st = group_capture_cont(g, src[0], src[1], fb)) != HL_OK) return st;
                HIPCHK(hipGraphLaunch(ce, s));
                unsigned *clog[2] = {c[0]->counters_host + hl::CNT_N + 64, c[1]->counters_host + hl::CNT_N + 64};
                for (int i = 0; i < 2; ++i) {
                    c[i]->stamp_host += CONT_PASSES;
                    HIPCHK(hipMemcpyAsync(clog[i], c[i]->pass_log + 64, sizeof(unsigned) * CONT_PASSES,
                                          hipMemcpyDeviceToHost, s));
                }
                if ((st = group_read_counters(g, s)) != HL_OK) return st;
                for (int i = 0; i < 2; ++i) {
                    for (int p = 0; p < CONT_PASSES; ++p) iters[i] += clog[i][p] > 0;
                    nflag[i] = c[i]->counters_host[hl::CNT_F0 + fb];
                }
            }
            hl::launch_dt_reduce_pair(pair_book(c[0]), pair_book(c[1]), s);
            if ((st = group_read_counters(g, s)) != HL_OK) return st;
        }
    } else {
        group_first(g, a, s);
        if ((st = group_read_counters(g, s)) != HL_OK) return st;
        for (int i = 0; i < 2; ++i) first[i] = nflag[i] = c[i]->counters_host[hl::CNT_F0];
        if ((st = eager_passes()) != HL_OK) return st;
        hl::launch_dt_reduce_pair(pair_book(c[0]), pair_book(c[1]), s);
        if ((st = group_read_counters(g, s)) != HL_OK) return st;
    }
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return hip_fail(le, "kernel launch", __LINE__);
    bool inadm = false;
    hl_step_info *info[2] = {info0, info1};
    for (int i = 0; i < 2; ++i) {
        c[i]->last_first = first[i];
        c[i]->last_iters = iters[i];
        c[i]->last_inadm = c[i]->counters_host[hl::CNT_BAD];
        c[i]->last_recomp = c[i]->counters_host[hl::CNT_RECOMP];
        inadm = inadm || c[i]->last_inadm;
        c[i]->cur = 1 - src[i];
        if (info[i]) {
            st = i == 0 ? fill_info<2>(c[0], src[0], info[0]) : fill_info<3>(c[1], src[1], info[1]);
            if (st != HL_OK) return st;
        }
    }
    return inadm ? HL_WARN_PARACHUTE_INADMISSIBLE : HL_OK;
}

}  // namespace

extern "C" {

hl_status hl_group_create(hl_group **out, hl_ctx *ctx_2d, hl_ctx *ctx_3d) {
    g_last_error[0] = '\0';
    if (!out) return HL_E_INVALID;
    *out = nullptr;
    if (!ctx_2d || !ctx_3d || ctx_2d == ctx_3d) return HL_E_INVALID;
    if (!ctx_2d->have_mesh || !ctx_3d->have_mesh) return HL_E_STATE;
    if (ctx_2d->dim != 2 || ctx_3d->dim != 3) return HL_E_INVALID;
    hl_group *g = new (std::nothrow) hl_group;
    if (!g) return HL_E_OOM;
    g->c[0] = ctx_2d;
    g->c[1] = ctx_3d;
    *out = g;
    return HL_OK;
}

hl_status hl_group_destroy(hl_group *g) {
    if (!g) return HL_OK;
    if (g->c[0]) (void)hipSetDevice(g->c[0]->device);
    group_drop_graphs(g);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    delete g;
    return HL_OK;
}

hl_status hl_group_use_graph(hl_group *g, int on, int max_mood_passes) {
    if (!g || max_mood_passes < 0 || max_mood_passes > 64) return HL_E_INVALID;
    if (g->graph_passes != max_mood_passes || !on) group_drop_graphs(g);
    g->graph_on = on != 0;
    g->graph_passes = max_mood_passes;
    return HL_OK;
}

hl_status hl_group_step(hl_group *g, hl_step_info *info_2d, hl_step_info *info_3d) {
    g_last_error[0] = '\0';
    if (!g) return HL_E_INVALID;
    hl_status st = group_step(g, info_2d, info_3d);
    if (st != HL_OK && st != HL_WARN_PARACHUTE_INADMISSIBLE) {
        // a failed step leaves no half-captured graph behind
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (g->cap_stream && hipStreamIsCapturing(g->cap_stream, &cs) == hipSuccess &&
            cs != hipStreamCaptureStatusNone) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(g->cap_stream, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
        }
    }
    return st;
}

}  // extern "C"
