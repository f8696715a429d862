// hl_kernels.h -- launch interface between the host side of libhyperlag
// (hl_api.hip) and its HIP kernels (hl_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
    uint8_t *flag;
    unsigned int *counters;  // [0] troubled P1 cells, [1] inadmissible P0 cells
    double delta0, delta1, eps_tol;
    int detect;
};

template <int D> void launch_centroids(const StepArgs &a, hipStream_t s);
template <int D> void launch_node_agg(const StepArgs &a, hipStream_t s);
template <int D> void launch_predict(const StepArgs &a, hipStream_t s);
template <int D> void launch_node_solve(const StepArgs &a, hipStream_t s);
template <int D> void launch_update(const StepArgs &a, hipStream_t s);
template <int D> void launch_acoustic(const StepArgs &a, hipStream_t s);
template <int D>
int64_t launch_diag(const StepArgs &a, const double *tau, const double *v, const double *e, const double *B,
                    double *part, double *out, hipStream_t s);
template <int D> void launch_stress_query(const StepArgs &a, double *out, hipStream_t s);
void launch_apply_flags(int64_t nc, uint8_t *mask, const uint8_t *flag, hipStream_t s);
void launch_dt_reduce(int64_t nc, const double *dtc, const int32_t *cell_mesh, double *red, int n_mesh,
                      hipStream_t s);
void launch_dt_finalize(int n_mesh, const double *red, const double *dt, const hl_params &p, int first,
                        double *dt_next, double *parts, hipStream_t s);
void launch_fill(double *p, int64_t n, double v, hipStream_t s);
void launch_aos_to_soa(int64_t n, int w, const double *in, double *out, hipStream_t s);
void launch_soa_to_aos(int64_t n, int w, const double *in, double *out, hipStream_t s);

}  // namespace hl
