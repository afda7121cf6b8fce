/*
 * Oracle for the explicit 3-D heat-diffusion step: plain FP64 CPU loops.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the HIP library it is used to check.
 *
 * What it computes (Omlin & Raess, "High-performance xPU Stencil
 * Computations in Julia", Fig. 1):
 *   - the scalars of the solver driver: dx = lx/(nx-1), the inverse spacings
 *     1/dx, and dt = min(dx^2, dy^2, dz^2)/lam/max(Ci)/6.1;
 *   - the time step on interior points
 *       T2 = T + dt*(lam*Ci*(d2x(T)*(1/dx)^2 + d2y(T)*(1/dy)^2 + d2z(T)*(1/dz)^2)),
 *     where d2x is the second difference along x, written as the difference
 *     of the two one-sided differences; boundary values are never written,
 *     so they keep the values of the initial field (T2 starts as a copy of T);
 *   - nt steps with the two buffers swapped after each step.
 * Expressions are evaluated left to right as written in Fig. 1 with no
 * fused multiply-add (built with -ffp-contract=off).
 *
 * The reverse sweep (gradient of a loss of the final field with respect to
 * the initial field and to Ci) is not in the paper; it is the transpose of
 * the step above, derived by hand:
 *   with c = dt*lam*Ci on interior points,
 *     gCi += dt*lam*lambda*Lap(T_k)             (interior points)
 *     mu   = dt*lam*Ci*lambda on interior points, 0 on the boundary
 *     lambda_k = lambda_{k+1} + Lap(mu)         (all points, mu = 0 outside)
 *   where Lap is the same weighted 7-point expression as in the step.
 *
 * Layout: linear index ix + nx*(iy + ny*iz), x fastest (Julia arrays are
 * column-major, so the first index is contiguous).
 *
 * The 2-D form (not printed in the paper, whose Fig. 1 is the 3-D solver):
 * the same expression without the z term,
 *       T2 = T + dt*(lam*Ci*(d2x(T)*(1/dx)^2 + d2y(T)*(1/dy)^2)),
 * on interior points of an nx x ny grid (index ix + nx*iy), boundary fixed.
 *
 * The operators of the kernel notation (Fig. 1 writes the step with @inn,
 * @d2_xi, @d2_yi and @d2_zi), each applied to a whole field: the interior
 * values, the second difference along one axis at interior points, and the
 * weighted Laplacian (d2x*(1/dx)^2 + d2y*(1/dy)^2) + d2z*(1/dz)^2, as dense
 * arrays over the interior.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(ix, iy, iz) ((size_t)(ix) + (size_t)nx * ((size_t)(iy) + (size_t)ny * (size_t)(iz)))

/* Scalars of the driver in Fig. 1 (physics and numerics blocks, and the dt
 * rule just before the time loop).  maximum(Ci) runs over the whole array.
 * Julia's x^2 with a literal 2 is x*x.  out = {dx, dy, dz, 1/dx, 1/dy, 1/dz, dt}. */
void oracle_scalars(int nx, int ny, int nz, double lx, double ly, double lz,
                    double lam, const double* Ci, double* out)
{
    size_t n = (size_t)nx * ny * nz;
    double cmax = Ci[0];
    for (size_t i = 1; i < n; ++i)
        if (Ci[i] > cmax) cmax = Ci[i];
    double dx = lx / (nx - 1);
    double dy = ly / (ny - 1);
    double dz = lz / (nz - 1);
    double m = dx * dx;
    if (dy * dy < m) m = dy * dy;
    if (dz * dz < m) m = dz * dz;
    out[0] = dx;
    out[1] = dy;
    out[2] = dz;
    out[3] = 1.0 / dx;
    out[4] = 1.0 / dy;
    out[5] = 1.0 / dz;
    out[6] = m / lam / cmax / 6.1;
}

/* One time step on interior points; the boundary of T2 is left alone. */
static void step(double* T2, const double* T, const double* Ci, int nx, int ny, int nz,
                 double lam, double dt, double rdx, double rdy, double rdz)
{
    const double cx = rdx * rdx, cy = rdy * rdy, cz = rdz * rdz;
    int iz;
#pragma omp parallel for schedule(static)
    for (iz = 1; iz < nz - 1; ++iz)
        for (int iy = 1; iy < ny - 1; ++iy)
            for (int ix = 1; ix < nx - 1; ++ix) {
                double t = T[IDX(ix, iy, iz)];
                double d2x = (T[IDX(ix + 1, iy, iz)] - t) - (t - T[IDX(ix - 1, iy, iz)]);
                double d2y = (T[IDX(ix, iy + 1, iz)] - t) - (t - T[IDX(ix, iy - 1, iz)]);
                double d2z = (T[IDX(ix, iy, iz + 1)] - t) - (t - T[IDX(ix, iy, iz - 1)]);
                T2[IDX(ix, iy, iz)] = t + dt * ((lam * Ci[IDX(ix, iy, iz)]) * ((d2x * cx + d2y * cy) + d2z * cz));
            }
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* T := T0 stepped nt times.  T and T2 are both set to T0 first (T2 = copy(T)
 * in Fig. 1); after each step the roles swap.  The result is copied into T. */
int oracle_forward(double* T, const double* T0, const double* Ci, int nx, int ny, int nz,
                   double lam, double dt, double rdx, double rdy, double rdz, int nt, int nthreads)
{
    if (nx < 3 || ny < 3 || nz < 3 || nt < 0) return -1;
    set_threads(nthreads);
    size_t n = (size_t)nx * ny * nz;
    double* T2 = (double*)malloc(n * sizeof(double));
    if (!T2) return -2;
    memcpy(T, T0, n * sizeof(double));
    memcpy(T2, T0, n * sizeof(double));
    double* a = T;
    double* b = T2;
    for (int it = 0; it < nt; ++it) {
        step(b, a, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz);
        double* s = a;
        a = b;
        b = s;
    }
    if (a != T) memcpy(T, a, n * sizeof(double));
    free(T2);
    return 0;
}

/* Reverse sweep for a loss of T_nt, given g_nt = dLoss/dT_nt.
 * Writes gT0 = dLoss/dT0 and gCi = dLoss/dCi (zero on the boundary).
 * States T_k are recomputed from stored states every `keep` steps
 * (keep = 1 stores every state). */
int oracle_reverse(const double* T0, const double* Ci, const double* g_nt, double* gT0, double* gCi,
                   int nx, int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz,
                   int nt, int keep, int nthreads)
{
    if (nx < 3 || ny < 3 || nz < 3 || nt < 0 || keep < 1) return -1;
    set_threads(nthreads);
    const size_t n = (size_t)nx * ny * nz;
    const double cx = rdx * rdx, cy = rdy * rdy, cz = rdz * rdz;
    const int nkept = nt > 0 ? (nt - 1) / keep + 1 : 1;
    double* kept = (double*)malloc((size_t)nkept * n * sizeof(double));
    double* Tk = (double*)malloc(n * sizeof(double));
    double* Tw = (double*)malloc(n * sizeof(double));
    double* mu = (double*)malloc(n * sizeof(double));
    double* lnext = (double*)malloc(n * sizeof(double));
    if (!kept || !Tk || !Tw || !mu || !lnext) {
        free(kept); free(Tk); free(Tw); free(mu); free(lnext);
        return -2;
    }

    /* forward pass, keeping T_0, T_keep, T_2keep, ... */
    memcpy(Tk, T0, n * sizeof(double));
    memcpy(Tw, T0, n * sizeof(double));
    for (int k = 0; k < nt; ++k) {
        if (k % keep == 0) memcpy(kept + (size_t)(k / keep) * n, Tk, n * sizeof(double));
        step(Tw, Tk, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz);
        double* s = Tk; Tk = Tw; Tw = s;
    }

    double* lam_k = gT0;
    memcpy(lam_k, g_nt, n * sizeof(double));
    memset(gCi, 0, n * sizeof(double));

    for (int k = nt - 1; k >= 0; --k) {
        /* T_k: from the kept state at or below k, stepped forward */
        int base = (k / keep) * keep;
        memcpy(Tk, kept + (size_t)(k / keep) * n, n * sizeof(double));
        memcpy(Tw, Tk, n * sizeof(double));
        for (int j = base; j < k; ++j) {
            step(Tw, Tk, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz);
            double* s = Tk; Tk = Tw; Tw = s;
        }

        /* Ci gradient from this step, and mu = dt*lam*Ci*lambda on the interior */
        int iz;
#pragma omp parallel for schedule(static)
        for (iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    size_t i = IDX(ix, iy, iz);
                    int interior = ix > 0 && ix < nx - 1 && iy > 0 && iy < ny - 1 && iz > 0 && iz < nz - 1;
                    if (!interior) {
                        mu[i] = 0.0;
                        continue;
                    }
                    double t = Tk[i];
                    double d2x = (Tk[IDX(ix + 1, iy, iz)] - t) - (t - Tk[IDX(ix - 1, iy, iz)]);
                    double d2y = (Tk[IDX(ix, iy + 1, iz)] - t) - (t - Tk[IDX(ix, iy - 1, iz)]);
                    double d2z = (Tk[IDX(ix, iy, iz + 1)] - t) - (t - Tk[IDX(ix, iy, iz - 1)]);
                    double lap = (d2x * cx + d2y * cy) + d2z * cz;
                    gCi[i] += dt * lam * lam_k[i] * lap;
                    mu[i] = dt * lam * Ci[i] * lam_k[i];
                }

        /* lambda_k = lambda_{k+1} + Lap(mu) at every point, mu = 0 outside */
#pragma omp parallel for schedule(static)
        for (iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    size_t i = IDX(ix, iy, iz);
                    double m = mu[i];
                    double xm = ix > 0 ? mu[IDX(ix - 1, iy, iz)] : 0.0;
                    double xp = ix < nx - 1 ? mu[IDX(ix + 1, iy, iz)] : 0.0;
                    double ym = iy > 0 ? mu[IDX(ix, iy - 1, iz)] : 0.0;
                    double yp = iy < ny - 1 ? mu[IDX(ix, iy + 1, iz)] : 0.0;
                    double zm = iz > 0 ? mu[IDX(ix, iy, iz - 1)] : 0.0;
                    double zp = iz < nz - 1 ? mu[IDX(ix, iy, iz + 1)] : 0.0;
                    double d2x = (xp - m) - (m - xm);
                    double d2y = (yp - m) - (m - ym);
                    double d2z = (zp - m) - (m - zm);
                    lnext[i] = lam_k[i] + ((d2x * cx + d2y * cy) + d2z * cz);
                }
        memcpy(lam_k, lnext, n * sizeof(double));
    }

    free(kept); free(Tk); free(Tw); free(mu); free(lnext);
    return 0;
}

/* The 2-D form of the step on interior points; the boundary of T2 is left
 * alone.  Evaluated left to right: t + dt*((lam*Ci)*(d2x*cx + d2y*cy)). */
static void step2d(double* T2, const double* T, const double* Ci, int nx, int ny, double lam, double dt,
                   double rdx, double rdy)
{
    const double cx = rdx * rdx, cy = rdy * rdy;
    const size_t sy = (size_t)nx;
#pragma omp parallel for schedule(static)
    for (int iy = 1; iy < ny - 1; ++iy)
        for (int ix = 1; ix < nx - 1; ++ix) {
            const size_t i = (size_t)ix + sy * (size_t)iy;
            const double t = T[i];
            const double d2x = (T[i + 1] - t) - (t - T[i - 1]);
            const double d2y = (T[i + sy] - t) - (t - T[i - sy]);
            T2[i] = t + dt * ((lam * Ci[i]) * (d2x * cx + d2y * cy));
        }
}

/* T := T0 stepped nt times with the 2-D form, two buffers swapped after
 * each step; the result is copied into T. */
int oracle_forward2d(double* T, const double* T0, const double* Ci, int nx, int ny, double lam, double dt,
                     double rdx, double rdy, int nt, int nthreads)
{
    if (nx < 3 || ny < 3 || nt < 0) return -1;
    set_threads(nthreads);
    const size_t n = (size_t)nx * ny;
    double* T2 = (double*)malloc(n * sizeof(double));
    if (!T2) return -2;
    memcpy(T, T0, n * sizeof(double));
    memcpy(T2, T0, n * sizeof(double));
    double* a = T;
    double* b = T2;
    for (int it = 0; it < nt; ++it) {
        step2d(b, a, Ci, nx, ny, lam, dt, rdx, rdy);
        double* s = a;
        a = b;
        b = s;
    }
    if (a != T) memcpy(T, a, n * sizeof(double));
    free(T2);
    return 0;
}

/* ------------------------------------------------------------ operators */
/* The operators of Fig. 1's kernel notation applied to the field A (nz == 1:
 * a 2-D field of nx*ny points).  At each interior point, in order x fastest:
 *   op 0  @inn(A):   A itself;
 *   op 1  @d2_xi(A): (A[x+1] - A[x]) - (A[x] - A[x-1]), the second difference
 *                    along x (the paper does not print its definition; this
 *                    is the difference of the two one-sided differences);
 *   op 2, op 3: the same along y and along z;
 *   op 4  (d2x*(rdx*rdx) + d2y*(rdy*rdy)) + d2z*(rdz*rdz), the Laplacian the
 *         step multiplies by dt*lam*Ci (2-D: d2x*(rdx*rdx) + d2y*(rdy*rdy)).
 * out holds (nx-2)*(ny-2)*(nz-2) values (2-D: (nx-2)*(ny-2)). */
int oracle_apply(int op, double* out, const double* A, int nx, int ny, int nz, double rdx, double rdy, double rdz)
{
    const int twod = nz == 1;
    if (op < 0 || op > 4 || nx < 3 || ny < 3 || (!twod && nz < 3) || (twod && op == 3)) return -1;
    const double cx = rdx * rdx, cy = rdy * rdy, cz = rdz * rdz;
    const int z0 = twod ? 0 : 1, z1 = twod ? 1 : nz - 1;
    size_t o = 0;
    for (int iz = z0; iz < z1; ++iz)
        for (int iy = 1; iy < ny - 1; ++iy)
            for (int ix = 1; ix < nx - 1; ++ix) {
                const double t = A[IDX(ix, iy, iz)];
                const double d2x = (A[IDX(ix + 1, iy, iz)] - t) - (t - A[IDX(ix - 1, iy, iz)]);
                const double d2y = (A[IDX(ix, iy + 1, iz)] - t) - (t - A[IDX(ix, iy - 1, iz)]);
                double d2z = 0.0;
                if (!twod) d2z = (A[IDX(ix, iy, iz + 1)] - t) - (t - A[IDX(ix, iy, iz - 1)]);
                double v;
                switch (op) {
                case 0: v = t; break;
                case 1: v = d2x; break;
                case 2: v = d2y; break;
                case 3: v = d2z; break;
                default: v = twod ? d2x * cx + d2y * cy : (d2x * cx + d2y * cy) + d2z * cz; break;
                }
                out[o++] = v;
            }
    return 0;
}
