// hl_mesh.hip -- host-side mesh services of libhyperlag: the conformity
// check of an uploaded simplicial mesh and its internal numbering (cells
// along a Hilbert curve through their centroids, nodes in the order the
// cells first use them).  Host code only.
#include "hl_mesh.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

namespace hl {

namespace {

// Face of cell c opposite local node k, oriented outward for a positively
// oriented simplex (3D: (1,2,3), (0,3,2), (0,1,3), (0,2,1); 2D: the edges
// (1,2), (2,0), (0,1) of a counter-clockwise triangle).
int oriented_face(int d, const int32_t *cell, int k, int32_t *f) {
    static const int F3[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    static const int F2[3][2] = {{1, 2}, {2, 0}, {0, 1}};
    for (int j = 0; j < d; ++j) f[j] = cell[d == 3 ? F3[k][j] : F2[k][j]];
    // sort ascending, counting transpositions (parity of the orientation)
    int par = 0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j + 1 < d - i; ++j)
            if (f[j] > f[j + 1]) {
                std::swap(f[j], f[j + 1]);
                par ^= 1;
            }
    return par;
}

void sub3(const double *a, const double *b, double *o) {
    for (int i = 0; i < 3; ++i) o[i] = a[i] - b[i];
}
void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Does point P lie on the closed boundary face with corners Q[0..d-1]
// (a triangle in 3D, a segment in 2D), up to a relative tolerance?
bool point_on_face(int d, const double *P, const double (*Q)[3]) {
    constexpr double tol = 1e-9;
    if (d == 2) {
        double e[3], w[3];
        sub3(Q[1], Q[0], e);
        sub3(P, Q[0], w);
        const double l2 = e[0] * e[0] + e[1] * e[1];
        if (!(l2 > 0.0)) return false;
        const double cr = e[0] * w[1] - e[1] * w[0];
        if (std::fabs(cr) > tol * l2) return false;   // distance > tol |e|
        const double t = (e[0] * w[0] + e[1] * w[1]) / l2;
        return t >= -tol && t <= 1.0 + tol;
    }
    double e1[3], e2[3], n[3], w[3];
    sub3(Q[1], Q[0], e1);
    sub3(Q[2], Q[0], e2);
    cross3(e1, e2, n);
    const double n2 = dot3(n, n);
    if (!(n2 > 0.0)) return false;
    sub3(P, Q[0], w);
    double L = std::max(dot3(e1, e1), dot3(e2, e2));
    double e3[3];
    sub3(Q[2], Q[1], e3);
    L = std::sqrt(std::max(L, dot3(e3, e3)));
    if (std::fabs(dot3(w, n)) > tol * L * std::sqrt(n2)) return false;   // off the plane
    // barycentric coordinates of the projection
    for (int j = 0; j < 3; ++j) {
        const double *A = Q[(j + 1) % 3], *B = Q[(j + 2) % 3];
        double ab[3], ap[3], c[3];
        sub3(B, A, ab);
        sub3(P, A, ap);
        cross3(ab, ap, c);
        if (dot3(c, n) / n2 < -tol) return false;
    }
    return true;
}

}  // namespace

hl_status check_conforming(int d, const double *x, const int32_t *cells, int64_t n0, int64_t n1, int64_t c0,
                           int64_t c1) {
    const int nv = d + 1;
    const int64_t nn = n1 - n0, nc = c1 - c0;
    if (nc == 0) return HL_OK;
    // faces grouped by their smallest node (counting sort), then sorted
    // within each group by the remaining node(s); the low bit of a key holds
    // the orientation parity
    std::vector<int64_t> off((size_t)nn + 1, 0);
    int32_t f[3];
    for (int64_t c = c0; c < c1; ++c)
        for (int k = 0; k < nv; ++k) {
            oriented_face(d, cells + c * nv, k, f);
            off[(size_t)(f[0] - n0) + 1]++;
        }
    for (int64_t p = 0; p < nn; ++p) off[p + 1] += off[p];
    std::vector<uint64_t> key((size_t)(nc * nv));
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int64_t c = c0; c < c1; ++c)
            for (int k = 0; k < nv; ++k) {
                const int par = oriented_face(d, cells + c * nv, k, f);
                uint64_t kk = d == 3 ? ((uint64_t)(f[1] - n0) << 32) | ((uint64_t)(f[2] - n0) << 1)
                                     : ((uint64_t)(f[1] - n0) << 1);
                key[(size_t)fill[f[0] - n0]++] = kk | (uint64_t)par;
            }
    }
    // boundary faces (seen once), as node triples / pairs
    std::vector<int32_t> bface;
    for (int64_t p = 0; p < nn; ++p) {
        uint64_t *b = key.data() + off[p], *e = key.data() + off[p + 1];
        std::sort(b, e);
        for (uint64_t *q = b; q < e;) {
            uint64_t *r = q + 1;
            while (r < e && (*r >> 1) == (*q >> 1)) ++r;
            const int64_t run = r - q;
            if (run > 2) return HL_E_NONCONFORMING;            // a face of three cells
            if (run == 2 && (q[0] & 1) == (q[1] & 1)) return HL_E_NONCONFORMING;  // same side
            if (run == 1) {
                bface.push_back((int32_t)(p + n0));
                if (d == 3) {
                    bface.push_back((int32_t)((*q >> 32) + n0));
                    bface.push_back((int32_t)(((*q & 0xffffffffu) >> 1) + n0));
                } else {
                    bface.push_back((int32_t)((*q >> 1) + n0));
                }
            }
            q = r;
        }
    }
    std::vector<uint64_t>().swap(key);
    const int64_t nb = (int64_t)bface.size() / d;
    if (nb == 0) return HL_OK;
    // 3D: the boundary surface closes up, every boundary edge on an even
    // number of boundary faces (a hanging node leaves an edge on one)
    if (d == 3) {
        std::vector<uint64_t> edges;
        edges.reserve((size_t)nb * 3);
        for (int64_t t = 0; t < nb; ++t) {
            const int32_t *q = bface.data() + 3 * t;   // ascending
            edges.push_back(((uint64_t)q[0] << 32) | (uint32_t)q[1]);
            edges.push_back(((uint64_t)q[0] << 32) | (uint32_t)q[2]);
            edges.push_back(((uint64_t)q[1] << 32) | (uint32_t)q[2]);
        }
        std::sort(edges.begin(), edges.end());
        for (size_t i = 0; i < edges.size();) {
            size_t j = i + 1;
            while (j < edges.size() && edges[j] == edges[i]) ++j;
            if ((j - i) & 1) return HL_E_NONCONFORMING;
            i = j;
        }
    }
    // no node lies on a boundary face it is not a vertex of: boundary faces
    // binned on a uniform grid by their bounding boxes, each boundary node
    // tested against the faces of its bin
    std::vector<int32_t> bnode(bface);
    std::sort(bnode.begin(), bnode.end());
    bnode.erase(std::unique(bnode.begin(), bnode.end()), bnode.end());
    auto pos = [&](int32_t p, double *o) {
        for (int i = 0; i < 3; ++i) o[i] = i < d ? x[(size_t)p * d + i] : 0.0;
    };
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hsum = 0.0;
    for (int32_t p : bnode) {
        double P[3];
        pos(p, P);
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], P[i]);
            hi[i] = std::max(hi[i], P[i]);
        }
    }
    std::vector<double> fb((size_t)nb * 6);   // face bounding boxes
    for (int64_t t = 0; t < nb; ++t) {
        double *b = fb.data() + 6 * t;
        for (int i = 0; i < 3; ++i) {
            b[i] = INFINITY;
            b[3 + i] = -INFINITY;
        }
        for (int j = 0; j < d; ++j) {
            double P[3];
            pos(bface[(size_t)(d * t + j)], P);
            for (int i = 0; i < 3; ++i) {
                b[i] = std::min(b[i], P[i]);
                b[3 + i] = std::max(b[3 + i], P[i]);
            }
        }
        double ext = 0.0;
        for (int i = 0; i < d; ++i) ext = std::max(ext, b[3 + i] - b[i]);
        hsum += ext;
    }
    const double h = std::max(hsum / (double)nb, 1e-300);
    int64_t ncell[3] = {1, 1, 1};
    for (int i = 0; i < d; ++i) ncell[i] = std::min<int64_t>(1 << 20, (int64_t)((hi[i] - lo[i]) / h) + 1);
    auto bin = [&](const double *P, int64_t *b) {
        for (int i = 0; i < 3; ++i)
            b[i] = i < d ? std::min<int64_t>(ncell[i] - 1, std::max<int64_t>(0, (int64_t)((P[i] - lo[i]) / h))) : 0;
    };
    auto bkey = [&](const int64_t *b) { return (uint64_t)((b[2] * ncell[1] + b[1]) * ncell[0] + b[0]); };
    std::vector<std::pair<uint64_t, int32_t>> cellface;
    for (int64_t t = 0; t < nb; ++t) {
        const double *b = fb.data() + 6 * t;
        double bl[3], bh[3];
        for (int i = 0; i < 3; ++i) {
            const double pad = 1e-9 * h;
            bl[i] = b[i] - pad;
            bh[i] = b[3 + i] + pad;
        }
        int64_t i0[3], i1[3];
        bin(bl, i0);
        bin(bh, i1);
        int64_t q[3];
        for (q[2] = i0[2]; q[2] <= i1[2]; ++q[2])
            for (q[1] = i0[1]; q[1] <= i1[1]; ++q[1])
                for (q[0] = i0[0]; q[0] <= i1[0]; ++q[0]) cellface.emplace_back(bkey(q), (int32_t)t);
    }
    std::sort(cellface.begin(), cellface.end());
    for (int32_t p : bnode) {
        double P[3];
        pos(p, P);
        int64_t b[3];
        bin(P, b);
        const uint64_t k = bkey(b);
        auto it = std::lower_bound(cellface.begin(), cellface.end(), std::make_pair(k, (int32_t)-1));
        for (; it != cellface.end() && it->first == k; ++it) {
            const int32_t *q = bface.data() + (size_t)d * it->second;
            bool vertex = false;
            for (int j = 0; j < d; ++j) vertex |= q[j] == p;
            if (vertex) continue;
            double Q[3][3];
            for (int j = 0; j < d; ++j) pos(q[j], Q[j]);
            if (point_on_face(d, P, Q)) return HL_E_NONCONFORMING;
        }
    }
    return HL_OK;
}

// Hilbert index of a point with `bits`-bit coordinates in n = 2 or 3
// dimensions, by J. Skilling's transpose method ("Programming the Hilbert
// curve", AIP Conf. Proc. 707, 2004): undo the excess work of the curve's
// recursion on the transposed coordinates, Gray-code them, then interleave
// their bits, most significant first.
uint64_t hilbert_key(uint32_t *X, int bits, int n) {
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < n; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < n; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[n - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < n; ++i) X[i] ^= t;
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < n; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
    return key;
}

void spatial_numbering(int d, const double *x, const int32_t *cells, const std::vector<int64_t> &node_off,
                       const std::vector<int64_t> &cell_off, std::vector<int32_t> &cell_i2u,
                       std::vector<int32_t> &node_i2u) {
    const int nv = d + 1;
    const int nmesh = (int)cell_off.size() - 1;
    const int bits = d == 3 ? 21 : 31;
    cell_i2u.resize((size_t)cell_off[nmesh]);
    node_i2u.resize((size_t)node_off[nmesh]);
    std::vector<std::pair<uint64_t, int32_t>> ord;
    std::vector<char> seen;
    for (int m = 0; m < nmesh; ++m) {
        const int64_t c0 = cell_off[m], c1 = cell_off[m + 1], n0 = node_off[m], n1 = node_off[m + 1];
        // bounding box of the mesh's cell centroids, one scale for all axes
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        std::vector<double> xc((size_t)(c1 - c0) * d);
        for (int64_t c = c0; c < c1; ++c)
            for (int i = 0; i < d; ++i) {
                double s = 0.0;
                for (int k = 0; k < nv; ++k) s += x[(size_t)cells[c * nv + k] * d + i];
                s /= nv;
                xc[(size_t)(c - c0) * d + i] = s;
                lo[i] = std::min(lo[i], s);
                hi[i] = std::max(hi[i], s);
            }
        double ext = 0.0;
        for (int i = 0; i < d; ++i) ext = std::max(ext, hi[i] - lo[i]);
        const double scale = ext > 0.0 ? ((double)((1u << bits) - 1u)) / ext : 0.0;
        ord.clear();
        ord.reserve((size_t)(c1 - c0));
        for (int64_t c = c0; c < c1; ++c) {
            uint32_t X[3] = {0, 0, 0};
            for (int i = 0; i < d; ++i) {
                const double q = (xc[(size_t)(c - c0) * d + i] - lo[i]) * scale;
                X[i] = (uint32_t)std::min<double>(std::max(q, 0.0), (double)((1u << bits) - 1u));
            }
            ord.emplace_back(hilbert_key(X, bits, d), (int32_t)c);
        }
        std::sort(ord.begin(), ord.end());   // ties: the caller's order
        for (int64_t i = 0; i < c1 - c0; ++i) cell_i2u[(size_t)(c0 + i)] = ord[(size_t)i].second;
        // nodes in the order the cells first use them; unused nodes last,
        // in the caller's order
        seen.assign((size_t)(n1 - n0), 0);
        int64_t next = n0;
        for (int64_t i = c0; i < c1; ++i) {
            const int32_t c = cell_i2u[(size_t)i];
            for (int k = 0; k < nv; ++k) {
                const int32_t p = cells[(size_t)c * nv + k];
                if (!seen[(size_t)(p - n0)]) {
                    seen[(size_t)(p - n0)] = 1;
                    node_i2u[(size_t)next++] = p;
                }
            }
        }
        for (int64_t p = n0; p < n1; ++p)
            if (!seen[(size_t)(p - n0)]) node_i2u[(size_t)next++] = (int32_t)p;
    }
}

}  // namespace hl
