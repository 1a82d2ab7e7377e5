/*
 * sbli_scalar.h -- scalar advection-diffusion of libsbli.so, the equation of the
 * paper's first two verification cases (Sec. "Propagation of a wave": first-order
 * wave equation; Sec. "Method of manufactured solutions": 2D advection-diffusion
 * with a source), on the same central stencils and low-storage RK3 as the
 * Navier-Stokes path:
 *
 *   d phi / dt = - sum_j c_j D_j phi + k sum_j D2_j phi - S
 *
 * with D, D2 the order-p central first / second derivatives (p even, 2..12) on a
 * periodic grid of n[0] x n[1] x n[2] points (x fastest; an axis with one point is
 * inactive), spacing length[d] / n[d], constant velocity c and diffusivity k >= 0,
 * and an optional source S (device array of the grid's size, or NULL).
 * Every active axis needs n >= 2; indices wrap modulo n as often as the stencil
 * needs, so a stencil wider than the grid (the manufactured-solution study's
 * coarsest grids, 4 points at order 12) is the periodic operator on those points.
 * phi, phi_tmp, dphi, source and rhs are
 * FP64 device arrays of n[0] n[1] n[2] values; work is enqueued on hip_stream.
 * Errors: SBLI_ERR_ARG / SBLI_ERR_HIP with a message from sbli_scalar_last_error
 * (per calling thread).
 */
#ifndef SBLI_SCALAR_H
#define SBLI_SCALAR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbli_scalar_params {
    int n[3];
    double length[3];
    int order;
    double c[3];
    double k;
} sbli_scalar_params;

/* rhs = the right-hand side above evaluated on phi. */
int sbli_scalar_rhs(const sbli_scalar_params* p, const double* phi, const double* source, double* rhs,
                    void* hip_stream);
/* nsteps steps of the three-stage 2N RK3 scheme (A = (0, -5/9, -153/128),
 * B = (1/3, 15/16, 8/15)); result in phi; phi_tmp and dphi are workspaces. */
int sbli_scalar_rk3(const sbli_scalar_params* p, double* phi, double* phi_tmp, double* dphi, const double* source,
                    double dt, int nsteps, void* hip_stream);
const char* sbli_scalar_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SBLI_SCALAR_H */
