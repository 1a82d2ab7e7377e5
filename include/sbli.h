/*
 * sbli.h -- C ABI of libsbli.so, an MI355X (gfx950) implementation of the
 * explicit residual evaluation and low-storage RK3 time stepping of the 3D
 * compressible Navier-Stokes equations described in Jacobs, Jammy & Sandham,
 * "OpenSBLI" (arXiv:1609.01277).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: every call returns an int, SBLI_OK (0) on success and a negative
 *    SBLI_ERR_* code otherwise.  No call aborts the process; after an error,
 *    sbli_last_error() returns a human-readable message for that context.
 *  - Memory: the caller allocates and owns every state-sized buffer; all state
 *    pointers are DEVICE pointers.  The library owns only the context and small
 *    device scratch (reduction partials), allocated in sbli_init.
 *  - Layout of a state q: five fields back to back, q[f][z][y][x], x fastest,
 *    f = (rho, rho*u, rho*v, rho*w, rho*E); element type double (SBLI_F64) or
 *    float (SBLI_F32) as chosen at init; nx*ny*nz*5 elements.
 *  - Streams: all device work is enqueued on the hipStream_t given at init
 *    (pass NULL for the default stream).  Calls return without waiting unless
 *    stated otherwise.
 *  - Grid: x_i = i*lx/nx (same in y, z); each axis periodic or with symmetry
 *    boundaries (sbli_params.bc); the reference length L = 1.
 */
#ifndef SBLI_H
#define SBLI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBLI_OK 0
#define SBLI_ERR_ARG (-1)         /* invalid argument (message says which)            */
#define SBLI_ERR_HIP (-2)         /* a HIP runtime call failed                        */
#define SBLI_ERR_NONFINITE (-3)   /* diagnostics found NaN/Inf, rho <= 0 or p <= 0    */
#define SBLI_ERR_ALLOC (-4)       /* device or host allocation failed                 */
#define SBLI_ERR_UNSUPPORTED (-5) /* a valid request the library does not implement  */

#define SBLI_F64 0
#define SBLI_F32 1

/*
 * Problem statement (paper Sec. "Grid" and Sec. "3D Taylor-Green vortex"):
 * grid points per axis, box lengths, Reynolds, Mach and Prandtl numbers, ratio
 * of specific heats, central-difference order and the state element type.
 * Requirements: order even, 2 to 12; every n >= 2*order + 1 (the nested
 * derivative terms reach 2*(order/2) points each way); lengths, Re, Mach, Pr > 0;
 * gamma > 1; dtype SBLI_F64 or SBLI_F32.
 */
typedef struct sbli_params {
    int nx, ny, nz;
    double lx, ly, lz;
    double Re, Mach, Pr, gamma;
    int order;
    int dtype;
    /* Boundary condition per axis (x, y, z), Sec. "Boundary conditions":
     * SBLI_BC_PERIODIC (0), or SBLI_BC_SYMMETRY (1): beyond each end the
     * fields are the mirror image of the points inside (point N is point N-1,
     * N+1 is N-2, -1 is 0, ...), the momentum component normal to the
     * boundary with opposite sign.  The points sit at x_i = i * lx / nx. */
    int bc[3];
} sbli_params;

#define SBLI_BC_PERIODIC 0
#define SBLI_BC_SYMMETRY 1

typedef struct sbli_ctx sbli_ctx;

/*
 * sbli_init: validate `p`, derive the grid spacing, build the central
 * difference weights of the requested order (Sec. "Discretisation schemes":
 * arbitrary-order central first and second derivatives, rationals evaluated
 * once) and the reciprocal constants (1/Re, heat-flux coefficient
 * 1/((gamma-1) M^2 Pr Re) with mu = 1).  `hip_stream` is a hipStream_t (or
 * NULL).  On success *out receives a new context, to be released with
 * sbli_destroy.  On failure *out is set to NULL and the message is available
 * from sbli_last_error(NULL).
 */
int sbli_init(const sbli_params* p, void* hip_stream, sbli_ctx** out);

/* Release a context and its scratch; waits for its stream first.  NULL is a no-op.
 * Everything is released even when a HIP call fails; the first failure is then
 * returned (SBLI_ERR_HIP, message from sbli_last_error(NULL)). */
int sbli_destroy(sbli_ctx* ctx);

/* Message of the last failed call on `ctx` (or of the last failed sbli_init when
 * ctx is NULL).  The string is owned by the library. */
const char* sbli_last_error(const sbli_ctx* ctx);

/*
 * sbli_tgv_init: write the Taylor-Green initial state (Sec. "3D Taylor-Green
 * vortex", initial conditions, with rho = 1) into the device state `q`:
 *   u = sin X cos Y cos Z, v = -cos X sin Y cos Z, w = 0,
 *   p = 1/(gamma M^2) + (cos 2X + cos 2Y)(cos 2Z + 2)/16,
 *   rho E = p/(gamma-1) + rho |u|^2 / 2,
 * at X = x_i + phase[0], Y = y_j + phase[1], Z = z_k + phase[2].  `phase` is a
 * host array of three doubles or NULL (no shift).
 */
int sbli_tgv_init(sbli_ctx* ctx, void* q, const double* phase);

/*
 * sbli_rhs: rhs = dq/dt of the compressible Navier-Stokes equations (eq. mass,
 * momentum, energy; stress tensor; heat flux; eq. eos; total energy) with the
 * skew-symmetric convective form (eq. skew_symmetric_formulation), the viscous
 * Laplacian by the second-derivative stencil, nested derivatives inner-first,
 * with the boundary condition of each axis (sbli_params.bc; on a symmetry axis
 * every stencil, the nested ones included, sees the mirror image of the state,
 * which makes the result that of the periodic box of twice the length holding
 * the state and its mirror image).  `q` and `rhs` are device states of the
 * context's dtype and must not overlap.
 */
int sbli_rhs(sbli_ctx* ctx, const void* q, void* rhs);

/*
 * sbli_rk3_step: advance `q` by `nsteps` steps of the three-stage low-storage
 * third-order Runge-Kutta scheme (Sec. "Discretisation schemes"), in 2N form
 *   dq <- A_k dq + dt R(q),  q <- q + B_k dq,  A = (0, -5/9, -153/128),
 *   B = (1/3, 15/16, 8/15).
 * `q_tmp` and `dq` are caller-provided device workspaces of the state's size;
 * `q`, `q_tmp` and `dq` must be three distinct, non-overlapping buffers.  The
 * result is in `q` on return (stream-ordered).  The contents of q_tmp and dq
 * afterwards are unspecified.  nsteps >= 0; dt finite.
 */
int sbli_rk3_step(sbli_ctx* ctx, void* q, void* q_tmp, void* dq, double dt, int nsteps);

/*
 * sbli_diagnostics: volume averages of the state (Sec. "3D Taylor-Green
 * vortex", kinetic energy and enstrophy integrals, rho_ref = 1), computed in
 * FP64 with compensated summation whatever the state dtype:
 *   out[0] = E_k = <1/2 rho u_j u_j>
 *   out[1] = enstrophy = <1/2 rho |omega|^2>, omega = curl u with the context's
 *            order-p central first derivative
 *   out[2..6] = <rho>, <rho u>, <rho v>, <rho w>, <rho E>
 * where <f> = sum over the grid / (nx ny nz).  `out` is a host array of 7
 * doubles.  Synchronises the stream.  Returns SBLI_ERR_NONFINITE (with `out`
 * filled) if any value is NaN/Inf or any point has rho <= 0 or p <= 0.
 */
int sbli_diagnostics(sbli_ctx* ctx, const void* q, double out[7]);

/*
 * Launch tuning of the stage kernel.  Each (dtype, order) up to order 8 has a
 * small set of compiled variants of the fused stage kernel (x/y tile of a
 * workgroup, how far the global loads run ahead, how the register window
 * advances, the barrier schedule); together with the number of z-planes per
 * workgroup ("zchunk") they fix the launch configuration.  The last variant of
 * every (dtype, order) is the staged form: two launches, one thread per point,
 * with the nested fields (6 words per point) in library-owned device memory,
 * allocated when the form is first selected and kept until sbli_destroy; orders 10 and 12 have only this variant, selected at
 * sbli_init.  All variants compute bitwise identical results; only speed differs.
 *
 * sbli_num_variants: number of variants for the context (>= 1), or < 0 on error.
 * sbli_variant_info: info = {tile x, tile y, load-ahead depth, register-window
 *   rotation (1) or shifting (0), wavefronts per SIMD its register allocation
 *   allows at least (1: as many registers as the kernel wants), barrier
 *   schedule (0: two barriers per z-plane; 1: double-buffered LDS planes, one
 *   barrier, where the R planes below the output plane are kept (0: registers,
 *   1: LDS)} of a variant (7 ints written); all seven are 0 for the staged form.
 * sbli_set_tuning / sbli_get_tuning: select / read the variant and zchunk used
 *   by sbli_rhs and sbli_rk3_step (1 <= zchunk <= nz; the staged form ignores
 *   zchunk).  sbli_set_tuning waits for the context's stream (it updates a small
 *   device table).  Selecting the staged form may allocate its scratch
 *   (SBLI_ERR_ALLOC if that fails; the previous selection then stays).
 * sbli_autotune: time every variant with several zchunks (hipEvents on the
 *   context's stream, `reps` RK3 steps each after one warm-up step) using the
 *   caller's device buffers, then select the fastest (a later candidate replaces
 *   the best so far only when more than 1 % faster, so near-ties resolve to the
 *   earlier variant and the longer zchunk); *best_ms (may be NULL) receives the
 *   selected candidate's time per step.  The contents of q, q_tmp and dq afterwards are
 *   unspecified (they are advanced in time).  Synchronises the stream.
 */
int sbli_num_variants(const sbli_ctx* ctx);
int sbli_variant_info(const sbli_ctx* ctx, int variant, int info[7]);
int sbli_set_tuning(sbli_ctx* ctx, int variant, int zchunk);
int sbli_get_tuning(const sbli_ctx* ctx, int* variant, int* zchunk);
int sbli_autotune(sbli_ctx* ctx, void* q, void* q_tmp, void* dq, double dt, int reps, double* best_ms);

/*
 * Ensembles ("batches") of independent periodic boxes: cubic grids of uneven
 * size with their own Re, Mach, Pr, gamma, time step and Taylor-Green phase,
 * sharing one order and dtype.  Every RK3 stage of every box is one launch of
 * the fused stage kernel, whose workgroups are split between the boxes by a
 * device table; nsteps of such launches can be recorded once into a hipGraph
 * and replayed with a single call.  Boxes are packed back to back in caller
 * buffers: box i occupies elements [offsets[i], offsets[i+1]) with its own
 * q[f][z][y][x] layout (sbli_batch_layout).  Every box is a 2*pi periodic cube.
 * Results are bitwise identical to stepping each box with its own context
 * (sbli_batch_step_sequential) in the same launch configuration.
 *
 * Orders 2, 4, 6 and 8 (the fused stage kernel takes a table of boxes).
 * sbli_instance: n (>= 2*order+1) points per axis, Re, Mach, Pr > 0,
 *   gamma > 1, dt > 0 its time step, phase the shift of its initial state.
 * sbli_batch_init: validate and set up `count` boxes; *out receives the batch.
 * sbli_batch_layout: offsets[0..count] (count+1 entries, elements).
 * sbli_batch_tgv_init: Taylor-Green initial state of every box.
 * sbli_batch_step: nsteps steps of every box, 3 launches per step.
 * sbli_batch_step_sequential: the same, each box by its own sbli_rk3_step
 *   (3 launches per box per step: the reference the ensemble is timed against).
 * sbli_batch_capture: record nsteps steps on the given buffers into a hipGraph
 *   (replacing any earlier one); the buffers must stay valid while it is used.
 * sbli_batch_launch: replay the recorded graph on the batch's stream.
 * sbli_batch_diagnostics: out[7*i .. 7*i+6] = sbli_diagnostics of box i;
 *   returns SBLI_ERR_NONFINITE if any box is flagged.  Synchronises the stream.
 * sbli_batch_set_tuning / get_tuning / autotune: variant (as for a single box)
 *   and the cap on z-planes per workgroup (zmax); changing them drops the graph.
 * In all calls q, q_tmp, dq are distinct device buffers of offsets[count]
 * elements; the result is in q.
 */
typedef struct sbli_instance {
    int n;
    double Re, Mach, Pr, gamma;
    double dt;
    double phase[3];
} sbli_instance;

typedef struct sbli_batch sbli_batch;

int sbli_batch_init(const sbli_instance* inst, int count, int order, int dtype, void* hip_stream, sbli_batch** out);
/* Release an ensemble (its graph, table and per-box contexts) after waiting for
 * its stream; everything is released even when a call fails, and the first
 * failure is returned (message from sbli_batch_last_error(NULL)). */
int sbli_batch_destroy(sbli_batch* b);
const char* sbli_batch_last_error(const sbli_batch* b);
int sbli_batch_layout(const sbli_batch* b, size_t* offsets);
int sbli_batch_tgv_init(sbli_batch* b, void* q);
int sbli_batch_step(sbli_batch* b, void* q, void* q_tmp, void* dq, int nsteps);
int sbli_batch_step_sequential(sbli_batch* b, void* q, void* q_tmp, void* dq, int nsteps);
int sbli_batch_capture(sbli_batch* b, void* q, void* q_tmp, void* dq, int nsteps);
int sbli_batch_launch(sbli_batch* b);
int sbli_batch_diagnostics(sbli_batch* b, const void* q, double* out);
int sbli_batch_set_tuning(sbli_batch* b, int variant, int zmax);
int sbli_batch_get_tuning(const sbli_batch* b, int* variant, int* zmax);
int sbli_batch_autotune(sbli_batch* b, void* q, void* q_tmp, void* dq, int reps, double* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* SBLI_H */
