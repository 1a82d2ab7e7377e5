/*
 * sbli_oracle.c -- plain FP64 CPU reference ("the oracle") for the compressible
 * Navier-Stokes hot path described in Jacobs, Jammy & Sandham, "OpenSBLI"
 * (arXiv:1609.01277).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.  The stencil weights are handed in by the
 * caller (computed in exact rationals by oracle/stencil.py).
 *
 * Everything is written as whole-array loops in the order the paper states the
 * method, in double precision, built with -O2 -ffp-contract=off.  No blocking,
 * fusion or reordering beyond the definitions:
 *   - grid x_i = i*dx; per axis either periodic (indices wrap mod N) or with
 *     symmetry boundaries (mirror images beyond each end, vector components
 *     normal to the boundary negated) (Sec. "Grid", Sec. "Boundary conditions");
 *   - central first / second derivative of order p = 2r (Sec. "Discretisation
 *     schemes"), the Laplacian of the viscous term by the second-derivative
 *     stencil (Sec. "3D Taylor-Green vortex", after the skew-symmetric equation);
 *   - nested derivatives: inner derivative evaluated first, then the outer one
 *     (Sec. "Expanding");
 *   - conservation laws eq. (mass), (momentum), (energy), stress tensor, heat
 *     flux, equation of state eq. (eos), total energy (Sec. "3D Taylor-Green
 *     vortex");
 *   - skew-symmetric convective form, eq. (skew_symmetric_formulation);
 *   - low-storage three-stage third-order Runge-Kutta (Sec. "Discretisation
 *     schemes", after Carpenter & Kennedy), in the 2N-storage form with
 *     A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15);
 *   - the Taylor-Green initial condition and the kinetic-energy and enstrophy
 *     integrals (Sec. "3D Taylor-Green vortex").
 *
 * Readings where the paper is silent (mu = 1; rho(t=0) = 1; which RK3 2N
 * coefficients; conservative viscous work; heat-flux sign) are listed in the
 * design notes of the repository.
 *
 * Layout: q[f][z][y][x], f in (rho, rho*u, rho*v, rho*w, rho*E), x fastest.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXR 8

typedef struct {
    int n[3];              /* points per axis (x, y, z)                      */
    double h[3];           /* grid spacing per axis                          */
    int r;                 /* stencil radius, order p = 2r                   */
    double a[ORA_MAXR];    /* first-derivative weights a_1..a_r              */
    double c0;             /* second-derivative centre weight                */
    double c[ORA_MAXR];    /* second-derivative weights c_1..c_r             */
    double Re, Mach, Pr, gamma;
    int sym[3];            /* per axis: 0 periodic, 1 symmetry boundaries     */
} ora_grid;

static long npts(const ora_grid* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static int wrapi(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

static double* alloc_arr(long n) {
    double* p = (double*)malloc(sizeof(double) * (size_t)n);
    return p;
}

/*
 * Value of array f at (i,j,k) shifted by m along `axis` (|m| < n).  Periodic
 * axes wrap.  On a symmetry axis (Sec. "Boundary conditions") the points beyond
 * each end mirror the points inside, the last point mirroring to the first halo
 * point (f at index N is f at N-1, at N+1 is f at N-2; at -1 is f at 0, at -2 is
 * f at 1); a field that is a vector component in that direction (or any field
 * odd under the mirror, par = -1) changes sign there.
 */
static double at_shift(const ora_grid* g, const double* f, int i, int j, int k, int axis, int m, int par) {
    int idx[3] = {i, j, k};
    int v = idx[axis] + m;
    const int n = g->n[axis];
    double sign = 1.0;
    if (g->sym[axis]) {
        if (v < 0) { v = -1 - v; sign = par; }
        else if (v >= n) { v = 2 * n - 1 - v; sign = par; }
    } else {
        v = wrapi(v, n);
    }
    idx[axis] = v;
    return sign * f[((long)idx[2] * g->n[1] + idx[1]) * g->n[0] + idx[0]];
}

/* First derivative along `axis`: D f_i = sum_m a_m (f_{i+m} - f_{i-m}) / h.
 * par: parity of f under the mirror of a symmetry boundary on `axis`. */
void ora_d1(const ora_grid* g, const double* f, int axis, int par, double* out) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int m = 1; m <= g->r; ++m) {
                    double fp = at_shift(g, f, i, j, k, axis, m, par);
                    double fm = at_shift(g, f, i, j, k, axis, -m, par);
                    s += g->a[m - 1] * (fp - fm);
                }
                out[((long)k * ny + j) * nx + i] = s / g->h[axis];
            }
}

/* Second derivative along `axis`:
 * D2 f_i = [c0 f_i + sum_m c_m (f_{i+m} + f_{i-m})] / h^2.  par as in ora_d1. */
void ora_d2(const ora_grid* g, const double* f, int axis, int par, double* out) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const double h2 = g->h[axis] * g->h[axis];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long id = ((long)k * ny + j) * nx + i;
                double s = g->c0 * f[id];
                for (int m = 1; m <= g->r; ++m) {
                    double fp = at_shift(g, f, i, j, k, axis, m, par);
                    double fm = at_shift(g, f, i, j, k, axis, -m, par);
                    s += g->c[m - 1] * (fp + fm);
                }
                out[id] = s / h2;
            }
}

/* out += alpha * x * y (elementwise; y may be NULL meaning 1). */
static void axpy_prod(long n, double alpha, const double* x, const double* y, double* out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] += alpha * x[i] * (y ? y[i] : 1.0);
}

/*
 * Residual R = dq/dt of the compressible Navier-Stokes equations
 * (eq. mass, momentum, energy) with:
 *   u_i = (rho u_i)/rho,  p = (gamma-1)(rho E - 1/2 (rho u_k) u_k)   [total energy]
 *   T = gamma M^2 p / rho                                            [eq. eos]
 *   g_ij = D_j u_i, theta = g_kk,
 *   tau_ij = (1/Re)(g_ij + g_ji - 2/3 delta_ij theta)                [stress tensor]
 *   kappa = 1/((gamma-1) M^2 Pr Re), mu = 1                          [heat flux]
 * Convective terms in the skew-symmetric form (eq. skew_symmetric_formulation)
 * with phi = 1, u_i, E:
 *   d_j(rho phi u_j) -> 1/2 [D_j(rho phi u_j) + u_j D_j(rho phi) + rho phi D_j u_j]
 * Pressure gradient D_i p, pressure work D_j(p u_j), viscous work D_j(u_i tau_ij)
 * in conservative form; the viscous Laplacian by the second-derivative stencil,
 * the mixed second derivatives by nested first derivatives (inner first).
 *   R_rho  = -1/2 sum_j [D_j(rho u_j) + u_j D_j rho + rho g_jj]
 *   R_mi   = -1/2 sum_j [D_j(rho u_i u_j) + u_j D_j(rho u_i) + rho u_i g_jj] - D_i p
 *            + (1/Re)[sum_j D2_j u_i + 1/3 D2_i u_i + 1/3 sum_{k!=i} D_i(g_kk)]
 *   R_E    = -1/2 sum_j [D_j(rho E u_j) + u_j D_j(rho E) + rho E g_jj]
 *            - sum_j D_j(p u_j) + kappa sum_j D2_j T + sum_j D_j(sum_i u_i tau_ij)
 */
/*
 * Parity under the mirror of a symmetry boundary on axis a of the velocity (or
 * momentum) component i: odd for the component normal to the boundary, even
 * otherwise.  Density, energy, pressure and temperature are even; a product's
 * parity is the product of its factors' parities; the viscous-work flux
 * V_j = u_i tau_ij is odd under the mirror on axis j (tau_ij has the parity of
 * u_i u_j).  With these, a derivative on a symmetry axis sees exactly the
 * mirror image of the field beyond the boundary.
 */
#define SGN(i, a) ((i) == (a) ? -1 : 1)

void ora_rhs(const ora_grid* g, const double* q, double* R) {
    const long P = npts(g);
    const double gam = g->gamma, M2 = g->Mach * g->Mach;
    const double inv_Re = 1.0 / g->Re;
    const double kappa = 1.0 / ((gam - 1.0) * M2 * g->Pr * g->Re);
    const double* rho = q;
    const double* m[3] = {q + P, q + 2 * P, q + 3 * P};
    const double* rE = q + 4 * P;
    double* R_rho = R;
    double* R_m[3] = {R + P, R + 2 * P, R + 3 * P};
    double* R_E = R + 4 * P;

    double* u[3];
    double *p, *T, *gr[3][3], *theta, *V[3], *t1, *t2, *t3;
    for (int i = 0; i < 3; ++i) u[i] = alloc_arr(P);
    p = alloc_arr(P);
    T = alloc_arr(P);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gr[i][j] = alloc_arr(P);
    theta = alloc_arr(P);
    for (int j = 0; j < 3; ++j) V[j] = alloc_arr(P);
    t1 = alloc_arr(P);
    t2 = alloc_arr(P);
    t3 = alloc_arr(P);

    /* primitives */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < P; ++n) {
        for (int i = 0; i < 3; ++i) u[i][n] = m[i][n] / rho[n];
        double ke = 0.5 * (m[0][n] * u[0][n] + m[1][n] * u[1][n] + m[2][n] * u[2][n]);
        p[n] = (gam - 1.0) * (rE[n] - ke);
        T[n] = gam * M2 * p[n] / rho[n];
    }
    /* velocity gradient g_ij = D_j u_i (inner derivatives of the nested terms) */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) ora_d1(g, u[i], j, SGN(i, j), gr[i][j]);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < P; ++n) theta[n] = gr[0][0][n] + gr[1][1][n] + gr[2][2][n];
    /* viscous work flux V_j = sum_i u_i tau_ij */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < P; ++n) {
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) {
                double tau = inv_Re * (gr[i][j][n] + gr[j][i][n] - (i == j ? (2.0 / 3.0) * theta[n] : 0.0));
                s += u[i][n] * tau;
            }
            V[j][n] = s;
        }
    }

    memset(R, 0, sizeof(double) * (size_t)(5 * P));

    /* ---- continuity ---- */
    for (int j = 0; j < 3; ++j) {
        ora_d1(g, m[j], j, -1, t1);        /* D_j(rho u_j)   */
        ora_d1(g, rho, j, 1, t2);          /* D_j rho        */
        axpy_prod(P, -0.5, t1, NULL, R_rho);
        axpy_prod(P, -0.5, u[j], t2, R_rho);
        axpy_prod(P, -0.5, rho, gr[j][j], R_rho);
    }

    /* ---- momentum ---- */
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
#pragma omp parallel for schedule(static)
            for (long n = 0; n < P; ++n) t3[n] = m[i][n] * u[j][n];   /* rho u_i u_j */
            ora_d1(g, t3, j, -SGN(i, j), t1);                            /* D_j(rho u_i u_j) */
            ora_d1(g, m[i], j, SGN(i, j), t2);                           /* D_j(rho u_i)     */
            axpy_prod(P, -0.5, t1, NULL, R_m[i]);
            axpy_prod(P, -0.5, u[j], t2, R_m[i]);
            axpy_prod(P, -0.5, m[i], gr[j][j], R_m[i]);
        }
        ora_d1(g, p, i, 1, t1);                                          /* D_i p */
        axpy_prod(P, -1.0, t1, NULL, R_m[i]);
        /* (1/Re) [ sum_j D2_j u_i + 1/3 D2_i u_i + 1/3 sum_{k != i} D_i(g_kk) ] */
        for (int j = 0; j < 3; ++j) {
            ora_d2(g, u[i], j, SGN(i, j), t1);
            axpy_prod(P, inv_Re, t1, NULL, R_m[i]);
            if (j == i) axpy_prod(P, inv_Re / 3.0, t1, NULL, R_m[i]);
        }
        for (int k = 0; k < 3; ++k) {
            if (k == i) continue;
            ora_d1(g, gr[k][k], i, 1, t1);                               /* D_i(D_k u_k) */
            axpy_prod(P, inv_Re / 3.0, t1, NULL, R_m[i]);
        }
    }

    /* ---- energy ---- */
    for (int j = 0; j < 3; ++j) {
#pragma omp parallel for schedule(static)
        for (long n = 0; n < P; ++n) t3[n] = rE[n] * u[j][n];           /* rho E u_j */
        ora_d1(g, t3, j, -1, t1);
        ora_d1(g, rE, j, 1, t2);
        axpy_prod(P, -0.5, t1, NULL, R_E);
        axpy_prod(P, -0.5, u[j], t2, R_E);
        axpy_prod(P, -0.5, rE, gr[j][j], R_E);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < P; ++n) t3[n] = p[n] * u[j][n];            /* p u_j */
        ora_d1(g, t3, j, -1, t1);
        axpy_prod(P, -1.0, t1, NULL, R_E);
        ora_d2(g, T, j, 1, t1);                                         /* D2_j T */
        axpy_prod(P, kappa, t1, NULL, R_E);
        ora_d1(g, V[j], j, -1, t1);                                     /* D_j(u_i tau_ij) */
        axpy_prod(P, 1.0, t1, NULL, R_E);
    }

    for (int i = 0; i < 3; ++i) free(u[i]);
    free(p);
    free(T);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) free(gr[i][j]);
    free(theta);
    for (int j = 0; j < 3; ++j) free(V[j]);
    free(t1);
    free(t2);
    free(t3);
}

/*
 * Generic three-stage low-storage (2N) Runge-Kutta step, k = 1..3:
 *   dq <- A_k dq + dt R(y);   y <- y + B_k dq
 * with A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15).  A_1 = 0, so the first
 * stage does not read the previous content of dq.
 * rhs(ctx, y, R) evaluates R = f(y) for a vector of n values.
 */
typedef void (*ora_rhs_fn)(void* ctx, const double* y, double* R);

void ora_rk3_generic(long n, double* y, double* dq, double dt, int nsteps, ora_rhs_fn rhs, void* ctx) {
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    double* R = alloc_arr(n);
    for (int s = 0; s < nsteps; ++s) {
        for (int k = 0; k < 3; ++k) {
            rhs(ctx, y, R);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                dq[i] = (k == 0) ? dt * R[i] : A[k] * dq[i] + dt * R[i];
                y[i] = y[i] + B[k] * dq[i];
            }
        }
    }
    free(R);
}

static void ns_rhs_cb(void* ctx, const double* y, double* R) { ora_rhs((const ora_grid*)ctx, y, R); }

/* nsteps RK3 steps of the Navier-Stokes residual, in place on q; dq is workspace. */
void ora_rk3_step(const ora_grid* g, double* q, double* dq, double dt, int nsteps) {
    ora_rk3_generic(5 * npts(g), q, dq, dt, nsteps, ns_rhs_cb, (void*)g);
}

/*
 * Taylor-Green initial condition (Sec. "3D Taylor-Green vortex"), L = 1,
 * x_i = i*h + phase:
 *   u = sin x cos y cos z, v = -cos x sin y cos z, w = 0, rho = 1,
 *   p = 1/(gamma M^2) + (cos 2x + cos 2y)(cos 2z + 2)/16,
 *   rho E = p/(gamma-1) + 1/2 rho (u^2 + v^2 + w^2).
 */
void ora_tgv_init(const ora_grid* g, double* q, const double phase[3]) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const long P = npts(g);
    const double gam = g->gamma, M2 = g->Mach * g->Mach;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long id = ((long)k * ny + j) * nx + i;
                double x = i * g->h[0] + phase[0];
                double y = j * g->h[1] + phase[1];
                double z = k * g->h[2] + phase[2];
                double u = sin(x) * cos(y) * cos(z);
                double v = -cos(x) * sin(y) * cos(z);
                double w = 0.0;
                double rho = 1.0;
                double p = 1.0 / (gam * M2) + (cos(2.0 * x) + cos(2.0 * y)) * (cos(2.0 * z) + 2.0) / 16.0;
                q[id] = rho;
                q[P + id] = rho * u;
                q[2 * P + id] = rho * v;
                q[3 * P + id] = rho * w;
                q[4 * P + id] = p / (gam - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
            }
}

/* Neumaier compensated accumulation. */
typedef struct { double s, c; } neum;
static void neum_add(neum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/*
 * Diagnostics (Sec. "3D Taylor-Green vortex", after DeBonis):
 *   out[0] = E_k = (1/P) sum 1/2 rho u_j u_j
 *   out[1] = eps = (1/P) sum 1/2 rho |omega|^2,
 *            omega = (D_y w - D_z v, D_z u - D_x w, D_x v - D_y u)  (order-p D)
 *   out[2..6] = (1/P) sum q_f
 * flags[0] = number of non-finite values, flags[1] = points with rho <= 0,
 * flags[2] = points with p <= 0.  Sums are sequential and Neumaier-compensated.
 */
void ora_diagnostics(const ora_grid* g, const double* q, double out[7], long flags[3]) {
    const long P = npts(g);
    const double gam = g->gamma;
    double* u[3];
    for (int i = 0; i < 3; ++i) {
        u[i] = alloc_arr(P);
        for (long n = 0; n < P; ++n) u[i][n] = q[(i + 1) * P + n] / q[n];
    }
    double *dwdy = alloc_arr(P), *dvdz = alloc_arr(P), *dudz = alloc_arr(P);
    double *dwdx = alloc_arr(P), *dvdx = alloc_arr(P), *dudy = alloc_arr(P);
    ora_d1(g, u[2], 1, 1, dwdy);
    ora_d1(g, u[1], 2, 1, dvdz);
    ora_d1(g, u[0], 2, 1, dudz);
    ora_d1(g, u[2], 0, 1, dwdx);
    ora_d1(g, u[1], 0, 1, dvdx);
    ora_d1(g, u[0], 1, 1, dudy);
    neum acc[7];
    memset(acc, 0, sizeof(acc));
    long nonfinite = 0, badrho = 0, badp = 0;
    for (long n = 0; n < P; ++n) {
        double rho = q[n];
        double ek = 0.5 * rho * (u[0][n] * u[0][n] + u[1][n] * u[1][n] + u[2][n] * u[2][n]);
        double wx = dwdy[n] - dvdz[n];
        double wy = dudz[n] - dwdx[n];
        double wz = dvdx[n] - dudy[n];
        double en = 0.5 * rho * (wx * wx + wy * wy + wz * wz);
        neum_add(&acc[0], ek);
        neum_add(&acc[1], en);
        for (int f = 0; f < 5; ++f) {
            double v = q[f * P + n];
            if (!isfinite(v)) ++nonfinite;
            neum_add(&acc[2 + f], v);
        }
        double ke = 0.5 * (q[P + n] * u[0][n] + q[2 * P + n] * u[1][n] + q[3 * P + n] * u[2][n]);
        double p = (gam - 1.0) * (q[4 * P + n] - ke);
        if (!(rho > 0.0)) ++badrho;
        if (!(p > 0.0)) ++badp;
    }
    for (int d = 0; d < 7; ++d) out[d] = (acc[d].s + acc[d].c) / (double)P;
    if (flags) {
        flags[0] = nonfinite;
        flags[1] = badrho;
        flags[2] = badp;
    }
    for (int i = 0; i < 3; ++i) free(u[i]);
    free(dwdy);
    free(dvdz);
    free(dudz);
    free(dwdx);
    free(dvdx);
    free(dudy);
}

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
