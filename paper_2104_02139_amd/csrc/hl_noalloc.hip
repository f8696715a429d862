// hl_noalloc.hip -- the allocation-free entry point of libhyperlag: the
// acoustic time step of hl_compute_dt for callers that cannot allocate
// device memory (work under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  Its partial minima live in a file-scope device array
// of fixed size instead of a buffer of a context.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "hl_device.h"
#include "hyperlag.h"

namespace {

constexpr int64_t kPartials = 65536;   // partial minima: 512 KiB on each GPU used
constexpr int kTile = 2048;            // cells per partial minimum (8 per thread)
constexpr int kMaxDevices = 64;

// Workspace: one partial minimum per tile of kTile cells.  In host code this
// name is only a stand-in for the symbol; kernels get its device address
// (g_scratch[device]) as an argument.
static __device__ __align__(256) double scratch[kPartials];

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

__device__ __forceinline__ double wave_min64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Block b: minimum of L_c / a_c over cells [b kTile, (b+1) kTile), with L_c
// the in-sphere diameter 2 d V / sum_f |f| and a_c the sound speed of the
// neo-Hookean law at J = rho0 tau (K = lambda + 2 mu / 3), the same device
// functions and operations as the context's acoustic kernel.  A node id out
// of range makes the block's partial NaN (no read happens).
template <int D>
__global__ __launch_bounds__(256) void k_acoustic_tiles(int64_t nn, const double *__restrict__ x, int64_t nc,
                                                        const int32_t *__restrict__ cells,
                                                        const double *__restrict__ rho0, const double *__restrict__ mu,
                                                        const double *__restrict__ lam, const double *__restrict__ tau,
                                                        double *__restrict__ part) {
    constexpr int NV = D + 1;
    __shared__ double sm[4];
    double m = __builtin_huge_val();
    int bad = 0;
    for (int j = 0; j < kTile / 256; ++j) {
        const int64_t c = (int64_t)blockIdx.x * kTile + j * 256 + threadIdx.x;
        if (c >= nc) break;
        double X[NV][D];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int64_t p = cells[c * NV + k];
            if (p < 0 || p >= nn) {
                ok = false;
                continue;
            }
#pragma unroll
            for (int i = 0; i < D; ++i) X[k][i] = x[p * D + i];
        }
        if (!ok) {
            bad = 1;
            continue;
        }
        hl::Geo<D> g;
        hl::geom<D>(X, g);
        double S = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) S += g.cn[k];
        const double K = lam[c] + 2.0 * mu[c] / 3.0;
        const double a = hl::sound(rho0[c], mu[c], K, tau[c]);
        const double v = 2.0 * g.V / S / a;
        m = fmin(m, v >= 0.0 ? v : __builtin_huge_val());
    }
    const int any_bad = __syncthreads_or(bad);
    m = wave_min64(m);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = any_bad ? __builtin_nan("") : fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3]));
}

// dt = c_cfl * min over the partials (NaN if a partial is NaN)
__global__ __launch_bounds__(256) void k_acoustic_final(int64_t n, const double *__restrict__ part, double c_cfl,
                                                        double *__restrict__ dt_out) {
    __shared__ double sm[4];
    __shared__ int sbad;
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    double m = __builtin_huge_val();
    int bad = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = part[i];
        bad |= v != v;
        m = fmin(m, v);
    }
    if (bad) atomicOr(&sbad, 1);
    m = wave_min64(m);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        dt_out[0] = sbad ? __builtin_nan("") : c_cfl * fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3]));
}

}  // namespace

extern "C" hl_status hl_acoustic_dt_noalloc(int device, void *hip_stream, int dim, int64_t n_nodes,
                                            const double *x, int64_t n_cells, const int32_t *cells,
                                            const double *rho0, const double *mu, const double *lam,
                                            const double *tau, double c_cfl, double *dt_out) {
    if ((dim != 2 && dim != 3) || n_nodes < 0 || n_cells < 0 || !dt_out || !(c_cfl > 0.0) || !std::isfinite(c_cfl))
        return HL_E_INVALID;
    if (n_cells > 0 && (!x || !cells || !rho0 || !mu || !lam || !tau)) return HL_E_INVALID;
    if (device < 0 || device >= kMaxDevices) return HL_E_INVALID;
    const int64_t nb = (n_cells + kTile - 1) / kTile;
    if (nb > kPartials) return HL_E_INVALID;   // more than kPartials * kTile cells
    if (hipSetDevice(device) != hipSuccess) return HL_E_HIP;
    double *ws = nullptr;
    {
        // the device address of the workspace, looked up once per device
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_scratch[device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HL_E_HIP;
            g_scratch[device] = static_cast<double *>(p);
        }
        ws = g_scratch[device];
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (nb > 0) {
        if (dim == 3)
            k_acoustic_tiles<3><<<(unsigned)nb, 256, 0, s>>>(n_nodes, x, n_cells, cells, rho0, mu, lam, tau, ws);
        else
            k_acoustic_tiles<2><<<(unsigned)nb, 256, 0, s>>>(n_nodes, x, n_cells, cells, rho0, mu, lam, tau, ws);
    }
    k_acoustic_final<<<1, 256, 0, s>>>(nb, ws, c_cfl, dt_out);
    return hipGetLastError() == hipSuccess ? HL_OK : HL_E_HIP;
}
