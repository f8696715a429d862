// hl_refine.hip -- conforming red refinement of a simplicial mesh on the
// GPU: every tetrahedron into 8 (4 corner tetrahedra and 4 from the inner
// octahedron, split along its shortest diagonal), every triangle into 4.
// This is the local 1 -> 8 refinement the paper applies to the partitions
// of a coarse mesh to reach large meshes (Section 3.9, "Implementation
// considerations").
//
// Edges are numbered by a device radix sort of their (min node, max node)
// keys; the midpoint of edge e becomes node nn + e.  Children of cell c are
// cells 8c .. 8c+7 (4c .. 4c+3 in 2D), in this order:
//   3D  (v0,m01,m02,m03) (m01,v1,m12,m13) (m02,m12,v2,m23) (m03,m13,m23,v3)
//       then (a,b,c0,c1) (a,b,c1,c2) (a,b,c2,c3) (a,b,c3,c0) for the
//       diagonal (a,b) of the octahedron and the cycle (c0..c3) of the
//       other four midpoints around it:
//         (m01,m23): (m02,m03,m13,m12)   (m02,m13): (m01,m03,m23,m12)
//         (m03,m12): (m01,m02,m23,m13)
//       the shortest diagonal (squared length, no fused operations), ties
//       to the first; a child of negative volume has its last two nodes
//       swapped;
//   2D  (v0,m01,m02) (m01,v1,m12) (m02,m12,v2) (m01,m12,m02).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <vector>

#include "hl_kernels.h"

namespace hl {
namespace {

template <int D>
struct RefineShape;
template <>
struct RefineShape<3> {
    static constexpr int NV = 4, NE = 6, NCH = 8;
};
template <>
struct RefineShape<2> {
    static constexpr int NV = 3, NE = 3, NCH = 4;
};

// local edge e joins nodes (ea[e], eb[e])
__device__ __forceinline__ void edge_nodes(int D, int e, int &a, int &b) {
    if (D == 3) {
        const int A[6] = {0, 0, 0, 1, 1, 2}, B[6] = {1, 2, 3, 2, 3, 3};
        a = A[e];
        b = B[e];
    } else {
        const int A[3] = {0, 0, 1}, B[3] = {1, 2, 2};
        a = A[e];
        b = B[e];
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

__device__ __forceinline__ int64_t tid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

template <int D>
__global__ void k_edge_keys(int64_t nc, const int32_t *__restrict__ cells, uint64_t *__restrict__ keys,
                            int64_t *__restrict__ vals) {
    using S = RefineShape<D>;
    const int64_t i = tid();
    if (i >= nc * S::NE) return;
    const int64_t c = i / S::NE;
    const int e = (int)(i % S::NE);
    int a, b;
    edge_nodes(D, e, a, b);
    const uint32_t p = (uint32_t)cells[c * S::NV + a], q = (uint32_t)cells[c * S::NV + b];
    const uint32_t lo = p < q ? p : q, hi = p < q ? q : p;
    keys[i] = ((uint64_t)lo << 32) | hi;
    vals[i] = i;
}

__global__ void k_edge_heads(int64_t n, const uint64_t *__restrict__ keys, int32_t *__restrict__ head) {
    const int64_t i = tid();
    if (i >= n) return;
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// cell-edge table and the node pair of every edge
__global__ void k_edge_scatter(int64_t n, const uint64_t *__restrict__ keys, const int64_t *__restrict__ vals,
                               const int32_t *__restrict__ head, const int32_t *__restrict__ eid,
                               int32_t *__restrict__ cedge, uint64_t *__restrict__ epair) {
    const int64_t i = tid();
    if (i >= n) return;
    const int32_t e = eid[i] - 1;
    cedge[vals[i]] = e;
    if (head[i]) epair[e] = keys[i];
}

// old positions, then the midpoint of every edge
template <int D>
__global__ void k_midpoints(int64_t nn, int64_t ne, const double *__restrict__ x, const uint64_t *__restrict__ epair,
                            double *__restrict__ xo) {
    const int64_t i = tid();
    if (i < nn) {
#pragma unroll
        for (int j = 0; j < D; ++j) xo[i * D + j] = x[i * D + j];
    } else if (i < nn + ne) {
        const uint64_t k = epair[i - nn];
        const int64_t p = (int64_t)(k >> 32), q = (int64_t)(k & 0xffffffffu);
#pragma unroll
        for (int j = 0; j < D; ++j) xo[i * D + j] = 0.5 * (x[p * D + j] + x[q * D + j]);
    }
}

template <int D>
__device__ __forceinline__ double signed_measure(const double *__restrict__ x, const int32_t (&v)[D + 1]) {
    double e[D][D];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int j = 0; j < D; ++j) e[k][j] = x[(int64_t)v[k + 1] * D + j] - x[(int64_t)v[0] * D + j];
    if (D == 3)
        return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
               e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    return e[0][0] * e[1][1] - e[0][1] * e[1][0];
}

template <int D>
__device__ __forceinline__ void emit(int32_t *__restrict__ out, const double *__restrict__ x, int32_t (&v)[D + 1]) {
    if (signed_measure<D>(x, v) < 0.0) {
        const int32_t t = v[D - 1];
        v[D - 1] = v[D];
        v[D] = t;
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) out[k] = v[k];
}

// squared distance of two nodes, every product and sum rounded on its own
__device__ __forceinline__ double dist2(const double *__restrict__ x, int64_t p, int64_t q) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double d = __dsub_rn(x[p * 3 + j], x[q * 3 + j]);
        s = __dadd_rn(s, __dmul_rn(d, d));
    }
    return s;
}

template <int D>
__global__ void k_children(int64_t nc, int64_t nn, const int32_t *__restrict__ cells, const int32_t *__restrict__ cedge,
                           const double *__restrict__ xo, int32_t *__restrict__ out) {
    using S = RefineShape<D>;
    const int64_t c = tid();
    if (c >= nc) return;
    int32_t v[S::NV], m[S::NE];
#pragma unroll
    for (int k = 0; k < S::NV; ++k) v[k] = cells[c * S::NV + k];
#pragma unroll
    for (int e = 0; e < S::NE; ++e) m[e] = (int32_t)(nn + cedge[c * S::NE + e]);
    int32_t *o = out + c * S::NCH * S::NV;
    if constexpr (D == 2) {
        // m[0] = m01, m[1] = m02, m[2] = m12
        int32_t t0[3] = {v[0], m[0], m[1]}, t1[3] = {m[0], v[1], m[2]}, t2[3] = {m[1], m[2], v[2]},
                t3[3] = {m[0], m[2], m[1]};
        emit<2>(o + 0, xo, t0);
        emit<2>(o + 3, xo, t1);
        emit<2>(o + 6, xo, t2);
        emit<2>(o + 9, xo, t3);
    } else {
        // m[0..5] = m01, m02, m03, m12, m13, m23
        const int32_t m01 = m[0], m02 = m[1], m03 = m[2], m12 = m[3], m13 = m[4], m23 = m[5];
        int32_t t0[4] = {v[0], m01, m02, m03}, t1[4] = {m01, v[1], m12, m13}, t2[4] = {m02, m12, v[2], m23},
                t3[4] = {m03, m13, m23, v[3]};
        emit<3>(o + 0, xo, t0);
        emit<3>(o + 4, xo, t1);
        emit<3>(o + 8, xo, t2);
        emit<3>(o + 12, xo, t3);
        const double d0 = dist2(xo, m01, m23), d1 = dist2(xo, m02, m13), d2 = dist2(xo, m03, m12);
        int32_t a, b, cy[4];
        if (d0 <= d1 && d0 <= d2) {
            a = m01, b = m23, cy[0] = m02, cy[1] = m03, cy[2] = m13, cy[3] = m12;
        } else if (d1 <= d2) {
            a = m02, b = m13, cy[0] = m01, cy[1] = m03, cy[2] = m23, cy[3] = m12;
        } else {
            a = m03, b = m12, cy[0] = m01, cy[1] = m02, cy[2] = m23, cy[3] = m13;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t u[4] = {a, b, cy[j], cy[(j + 1) & 3]};
            emit<3>(o + 16 + 4 * j, xo, u);
        }
    }
}

template <class T>
hipError_t dmalloc(T **p, size_t n, std::vector<void *> &mem) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n * sizeof(T), 256));
    if (e == hipSuccess) mem.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return e;
}

}  // namespace

template <int D>
hipError_t refine_once(int64_t nn, int64_t nc, const double *x_host, const int32_t *cells_host, hipStream_t s,
                       std::vector<double> &x_out, std::vector<int32_t> &cells_out,
                       std::vector<uint64_t> &edges_out) {
    using S = RefineShape<D>;
    std::vector<void *> mem;
    auto release = [&]() {
        (void)hipStreamSynchronize(s);
        for (void *p : mem) (void)hipFree(p);
    };
    const int64_t nk = nc * S::NE;
    if (nk >= (int64_t)INT32_MAX || (nn + nk) >= (int64_t)INT32_MAX || nc * S::NCH * S::NV >= (int64_t)INT32_MAX)
        return hipErrorInvalidValue;
    double *x = nullptr, *xo = nullptr;
    int32_t *cells = nullptr, *head = nullptr, *eid = nullptr, *cedge = nullptr, *out = nullptr;
    uint64_t *k0 = nullptr, *k1 = nullptr, *epair = nullptr;
    int64_t *v0 = nullptr, *v1 = nullptr;
    hipError_t e = hipSuccess;
#define R_(call)                  \
    do {                          \
        if ((e = (call)) != hipSuccess) { \
            release();            \
            return e;             \
        }                         \
    } while (0)
    R_(dmalloc(&x, (size_t)nn * D, mem));
    R_(dmalloc(&cells, (size_t)nc * S::NV, mem));
    R_(dmalloc(&k0, (size_t)nk, mem));
    R_(dmalloc(&k1, (size_t)nk, mem));
    R_(dmalloc(&v0, (size_t)nk, mem));
    R_(dmalloc(&v1, (size_t)nk, mem));
    R_(dmalloc(&head, (size_t)nk, mem));
    R_(dmalloc(&eid, (size_t)nk, mem));
    R_(dmalloc(&cedge, (size_t)nk, mem));
    R_(hipMemcpyAsync(x, x_host, sizeof(double) * nn * D, hipMemcpyHostToDevice, s));
    R_(hipMemcpyAsync(cells, cells_host, sizeof(int32_t) * nc * S::NV, hipMemcpyHostToDevice, s));
    if (nk) k_edge_keys<D><<<blocks(nk), 256, 0, s>>>(nc, cells, k0, v0);
    size_t tmp_sort = 0, tmp_scan = 0;
    R_(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_sort, k0, k1, v0, v1, (int)nk, 0, 64, s));
    R_(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_scan, head, eid, (int)nk, s));
    void *tmp = nullptr;
    R_(dmalloc(reinterpret_cast<char **>(&tmp), std::max(tmp_sort, tmp_scan), mem));
    size_t t1 = tmp_sort, t2 = tmp_scan;
    if (nk) {
        R_(hipcub::DeviceRadixSort::SortPairs(tmp, t1, k0, k1, v0, v1, (int)nk, 0, 64, s));
        k_edge_heads<<<blocks(nk), 256, 0, s>>>(nk, k1, head);
        R_(hipcub::DeviceScan::InclusiveSum(tmp, t2, head, eid, (int)nk, s));
    }
    int32_t ne32 = 0;
    if (nk) R_(hipMemcpyAsync(&ne32, eid + nk - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    R_(hipStreamSynchronize(s));
    const int64_t ne = ne32;
    R_(dmalloc(&epair, (size_t)ne, mem));
    R_(dmalloc(&xo, (size_t)(nn + ne) * D, mem));
    R_(dmalloc(&out, (size_t)nc * S::NCH * S::NV, mem));
    if (nk) k_edge_scatter<<<blocks(nk), 256, 0, s>>>(nk, k1, v1, head, eid, cedge, epair);
    if (nn + ne) k_midpoints<D><<<blocks(nn + ne), 256, 0, s>>>(nn, ne, x, epair, xo);
    if (nc) k_children<D><<<blocks(nc), 256, 0, s>>>(nc, nn, cells, cedge, xo, out);
    R_(hipGetLastError());
    x_out.resize((size_t)(nn + ne) * D);
    cells_out.resize((size_t)nc * S::NCH * S::NV);
    edges_out.resize((size_t)ne);
    R_(hipMemcpyAsync(x_out.data(), xo, sizeof(double) * x_out.size(), hipMemcpyDeviceToHost, s));
    R_(hipMemcpyAsync(cells_out.data(), out, sizeof(int32_t) * cells_out.size(), hipMemcpyDeviceToHost, s));
    R_(hipMemcpyAsync(edges_out.data(), epair, sizeof(uint64_t) * edges_out.size(), hipMemcpyDeviceToHost, s));
    R_(hipStreamSynchronize(s));
#undef R_
    release();
    return hipSuccess;
}

template hipError_t refine_once<2>(int64_t, int64_t, const double *, const int32_t *, hipStream_t,
                                   std::vector<double> &, std::vector<int32_t> &, std::vector<uint64_t> &);
template hipError_t refine_once<3>(int64_t, int64_t, const double *, const int32_t *, hipStream_t,
                                   std::vector<double> &, std::vector<int32_t> &, std::vector<uint64_t> &);

}  // namespace hl
