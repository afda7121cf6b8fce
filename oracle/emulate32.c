/*
 * Reduced-precision emulator for the explicit 3-D heat-diffusion step:
 * plain CPU loops in FP32 arithmetic with FP32 or BF16 storage.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the HIP library it is used to check.
 *
 * What it computes (the step of Omlin & Raess, "High-performance xPU Stencil
 * Computations in Julia", Fig. 1, with the storage forms added to it):
 *   - fields are stored as FP32, or as BF16 (the upper 16 bits of an FP32
 *     pattern); a stored value is widened to FP32 exactly;
 *   - lam, dt and (1/h)^2 are each formed in FP64 and rounded once to FP32;
 *   - one step on interior points, in FP32 with no fused multiply-add and in
 *     Fig. 1's order:
 *       T2 = t + dt*((lam*Ci)*((d2x*cx + d2y*cy) + d2z*cz)),
 *       d2x = (T[x+1] - t) - (t - T[x-1])  (likewise y, z);
 *     boundary values never change;
 *   - a run is a sequence of passes of n steps each; inside a pass the
 *     states stay in FP32, and only the state at the end of a pass is
 *     stored, i.e. rounded to the storage type: to nearest even, or
 *     stochastically;
 *   - stochastic rounding of the state stored after global step index k:
 *     the 16 random bits r of point i are half of one output word of the
 *     Philox4x32-10 generator (Salmon, Moraes, Dror, Shaw, "Parallel random
 *     numbers: as easy as 1, 2, 3", SC'11) evaluated at key (seed low word,
 *     seed high word) and counter (g low word, g high word, k low word,
 *     k high word), g = i / 8: word (i % 8) / 2, its low half for even i and
 *     its high half for odd i.  The stored value is the FP32 pattern plus r,
 *     keeping the upper 16 bits (NaN and infinity unchanged);
 *   - the reverse sweep in FP32 storage, the transpose of the step derived
 *     by hand (as the FP64 oracle's), with dt*lam formed as
 *     float(dt)*float(lam) in FP32:
 *       gCi += ((dt*lam)*lambda)*Lap(T_k)     interior points
 *       mu   = ((dt*lam)*Ci)*lambda            interior points, 0 elsewhere
 *       lambda_k = lambda_{k+1} + Lap(mu)      every point (mu = 0 outside).
 *   - the operators of the kernel notation (@inn, @d2_xi, @d2_yi, @d2_zi
 *     and the weighted Laplacian) in FP32 on widened stored values, as the
 *     FP64 oracle defines them;
 *   - the 2-D form (a single plane, nz = 1, linear index x + nx*y): the same
 *     step without the z term, T2 = t + dt*((lam*Ci)*(d2x*cx + d2y*cy)),
 *     with the same passes and rounding (index i = x + nx*y).
 * Built with -ffp-contract=off; x86-64 evaluates float expressions in FP32.
 * Layout: linear index ix + nx*(iy + ny*iz), x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EIDX(ix, iy, iz) ((size_t)(ix) + (size_t)nx * ((size_t)(iy) + (size_t)ny * (size_t)(iz)))

enum { ST_F32 = 1, ST_BF16_SR = 2, ST_BF16_RNE = 3 };

/* ------------------------------------------------------------ Philox4x32-10
 * Ten rounds.  A round multiplies counter words 0 and 2 by the two Philox
 * multipliers (64-bit products split into high and low halves) and permutes:
 *   (c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
 * the key advances by the Weyl constants between rounds. */
void emul_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)mul0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)mul1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += weyl0;
        k1 += weyl1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* The 16 random bits of point i for the state stored after step k. */
static uint16_t sr_bits_of(uint64_t seed, uint64_t k, uint64_t i)
{
    const uint64_t g = i / 8;
    const uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), (uint32_t)k, (uint32_t)(k >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    emul_philox4x32_10(ctr, key, out);
    const uint32_t w = out[(i % 8) / 2];
    return (i % 2) ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xFFFFu);
}

void emul_sr_bits(uint64_t seed, uint64_t k, const uint64_t* idx, uint16_t* out, size_t n)
{
    for (size_t j = 0; j < n; ++j) out[j] = sr_bits_of(seed, k, idx[j]);
}

/* ------------------------------------------------------------ FP32 and BF16 */
static uint32_t bits_of(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float float_of(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

static int is_nan_bits(uint32_t u) { return (u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0; }
static int is_inf_bits(uint32_t u) { return (u & 0x7FFFFFFFu) == 0x7F800000u; }

static float widen_bf16(uint16_t h) { return float_of((uint32_t)h << 16); }

/* Round to nearest, ties to even; NaN stays a (quiet) NaN. */
static uint16_t bf16_nearest(float f)
{
    const uint32_t u = bits_of(f);
    if (is_nan_bits(u)) return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

/* Stochastic: add r below the kept bits and truncate; NaN and infinity kept. */
static uint16_t bf16_stochastic(float f, uint16_t r)
{
    const uint32_t u = bits_of(f);
    if (is_nan_bits(u)) return (uint16_t)((u >> 16) | 0x0040u);
    if (is_inf_bits(u)) return (uint16_t)(u >> 16);
    return (uint16_t)((u + (uint32_t)r) >> 16);
}

void emul_bf16_nearest(const float* x, uint16_t* out, size_t n)
{
    for (size_t i = 0; i < n; ++i) out[i] = bf16_nearest(x[i]);
}

void emul_bf16_stochastic(const float* x, const uint16_t* r, uint16_t* out, size_t n)
{
    for (size_t i = 0; i < n; ++i) out[i] = bf16_stochastic(x[i], r[i]);
}

static void set_threads32(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ------------------------------------------------------------ forward */
/* One FP32 step on interior points; the boundary of T2 is left alone. */
static void step32(float* T2, const float* T, const float* Ci, int nx, int ny, int nz, float lam, float dt,
                   float cx, float cy, float cz)
{
    int iz;
#pragma omp parallel for schedule(static)
    for (iz = 1; iz < nz - 1; ++iz)
        for (int iy = 1; iy < ny - 1; ++iy)
            for (int ix = 1; ix < nx - 1; ++ix) {
                float t = T[EIDX(ix, iy, iz)];
                float d2x = (T[EIDX(ix + 1, iy, iz)] - t) - (t - T[EIDX(ix - 1, iy, iz)]);
                float d2y = (T[EIDX(ix, iy + 1, iz)] - t) - (t - T[EIDX(ix, iy - 1, iz)]);
                float d2z = (T[EIDX(ix, iy, iz + 1)] - t) - (t - T[EIDX(ix, iy, iz - 1)]);
                T2[EIDX(ix, iy, iz)] = t + dt * ((lam * Ci[EIDX(ix, iy, iz)]) * ((d2x * cx + d2y * cy) + d2z * cz));
            }
}

/* One FP32 step of the 2-D form (a single plane) on interior points. */
static void step2d32(float* T2, const float* T, const float* Ci, int nx, int ny, float lam, float dt, float cx,
                     float cy)
{
    int iy;
#pragma omp parallel for schedule(static)
    for (iy = 1; iy < ny - 1; ++iy)
        for (int ix = 1; ix < nx - 1; ++ix) {
            const size_t i = (size_t)ix + (size_t)nx * (size_t)iy;
            float t = T[i];
            float d2x = (T[i + 1] - t) - (t - T[i - 1]);
            float d2y = (T[i + (size_t)nx] - t) - (t - T[i - (size_t)nx]);
            T2[i] = t + dt * ((lam * Ci[i]) * (d2x * cx + d2y * cy));
        }
}

/* Stored values (storage type) -> FP32. */
static void widen_field(float* out, const void* in, size_t n, int storage)
{
    if (storage == ST_F32) {
        memcpy(out, in, n * sizeof(float));
        return;
    }
    const uint16_t* h = (const uint16_t*)in;
    size_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) out[i] = widen_bf16(h[i]);
}

/* Store the interior of an FP32 state into `out` (storage type), drawing
 * with step index k under stochastic rounding. */
static void store_interior(void* out, const float* x, int nx, int ny, int nz, int storage, uint64_t seed, uint64_t k)
{
    /* a single plane (the 2-D form) is all interior along z */
    const int z0 = nz == 1 ? 0 : 1, z1 = nz == 1 ? 1 : nz - 1;
    int iz;
#pragma omp parallel for schedule(static)
    for (iz = z0; iz < z1; ++iz)
        for (int iy = 1; iy < ny - 1; ++iy) {
            /* the Philox output of the current block of 8 points, reused
             * while consecutive points stay in it */
            uint64_t blk = UINT64_MAX;
            uint32_t words[4] = {0, 0, 0, 0};
            for (int ix = 1; ix < nx - 1; ++ix) {
                const size_t i = EIDX(ix, iy, iz);
                if (storage == ST_F32) {
                    ((float*)out)[i] = x[i];
                } else if (storage == ST_BF16_RNE) {
                    ((uint16_t*)out)[i] = bf16_nearest(x[i]);
                } else {
                    if ((uint64_t)i / 8 != blk) {
                        blk = (uint64_t)i / 8;
                        const uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), (uint32_t)k,
                                                 (uint32_t)(k >> 32)};
                        const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
                        emul_philox4x32_10(ctr, key, words);
                    }
                    const uint32_t w = words[(i % 8) / 2];
                    const uint16_t r = (i % 2) ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xFFFFu);
                    ((uint16_t*)out)[i] = bf16_stochastic(x[i], r);
                }
            }
        }
}

/* T := T0 advanced by the passes (passes[j] steps each), storage as above;
 * the j-th stored state draws with index step0 + (steps up to and
 * including that pass) - 1.  T and T0 hold nx*ny*nz stored values; nz = 1
 * selects the 2-D form (rdz unused). */
int emul_forward(void* T, const void* T0, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, const int* passes, int npasses, int storage, uint64_t seed, uint64_t step0,
                 int nthreads)
{
    if (nx < 3 || ny < 3 || (nz < 3 && nz != 1) || npasses < 0) return -1;
    if (storage != ST_F32 && storage != ST_BF16_SR && storage != ST_BF16_RNE) return -1;
    for (int j = 0; j < npasses; ++j)
        if (passes[j] < 1) return -1;
    set_threads32(nthreads);
    const size_t n = (size_t)nx * ny * nz;
    const size_t esz = storage == ST_F32 ? 4 : 2;
    float* a = (float*)malloc(n * sizeof(float));
    float* b = (float*)malloc(n * sizeof(float));
    float* c = (float*)malloc(n * sizeof(float));
    if (!a || !b || !c) {
        free(a); free(b); free(c);
        return -2;
    }
    const float lamf = (float)lam, dtf = (float)dt;
    const float cx = (float)(rdx * rdx), cy = (float)(rdy * rdy), cz = (float)(rdz * rdz);
    widen_field(c, Ci, n, storage);
    memcpy(T, T0, n * esz);
    uint64_t k = step0;
    for (int j = 0; j < npasses; ++j) {
        widen_field(a, T, n, storage);
        memcpy(b, a, n * sizeof(float));
        float* cur = a;
        float* nxt = b;
        for (int s = 0; s < passes[j]; ++s) {
            if (nz == 1)
                step2d32(nxt, cur, c, nx, ny, lamf, dtf, cx, cy);
            else
                step32(nxt, cur, c, nx, ny, nz, lamf, dtf, cx, cy, cz);
            float* t = cur;
            cur = nxt;
            nxt = t;
        }
        k += (uint64_t)passes[j];
        store_interior(T, cur, nx, ny, nz, storage, seed, k - 1);
    }
    free(a);
    free(b);
    free(c);
    return 0;
}

/* ------------------------------------------------------------ reverse (FP32) */
/* Reverse sweep in FP32 for a loss of T_nt, given g_nt = dLoss/dT_nt; states
 * are kept every `keep` steps and recomputed in between (FP32 states are
 * the same whichever way they are recomputed). */
int emul_reverse32(const float* T0, const float* Ci, const float* g_nt, float* gT0, float* gCi, int nx, int ny,
                   int nz, double lam, double dt, double rdx, double rdy, double rdz, int nt, int keep, int nthreads)
{
    if (nx < 3 || ny < 3 || nz < 3 || nt < 0 || keep < 1) return -1;
    set_threads32(nthreads);
    const size_t n = (size_t)nx * ny * nz;
    const float lamf = (float)lam, dtf = (float)dt;
    const float dtlam = dtf * lamf;
    const float cx = (float)(rdx * rdx), cy = (float)(rdy * rdy), cz = (float)(rdz * rdz);
    const int nkept = nt > 0 ? (nt - 1) / keep + 1 : 1;
    float* kept = (float*)malloc((size_t)nkept * n * sizeof(float));
    float* Tk = (float*)malloc(n * sizeof(float));
    float* Tw = (float*)malloc(n * sizeof(float));
    float* mu = (float*)malloc(n * sizeof(float));
    float* lnext = (float*)malloc(n * sizeof(float));
    if (!kept || !Tk || !Tw || !mu || !lnext) {
        free(kept); free(Tk); free(Tw); free(mu); free(lnext);
        return -2;
    }
    memcpy(Tk, T0, n * sizeof(float));
    memcpy(Tw, T0, n * sizeof(float));
    for (int k = 0; k < nt; ++k) {
        if (k % keep == 0) memcpy(kept + (size_t)(k / keep) * n, Tk, n * sizeof(float));
        step32(Tw, Tk, Ci, nx, ny, nz, lamf, dtf, cx, cy, cz);
        float* s = Tk; Tk = Tw; Tw = s;
    }
    float* lk = gT0;
    memcpy(lk, g_nt, n * sizeof(float));
    memset(gCi, 0, n * sizeof(float));
    for (int k = nt - 1; k >= 0; --k) {
        const int base = (k / keep) * keep;
        memcpy(Tk, kept + (size_t)(k / keep) * n, n * sizeof(float));
        memcpy(Tw, Tk, n * sizeof(float));
        for (int j = base; j < k; ++j) {
            step32(Tw, Tk, Ci, nx, ny, nz, lamf, dtf, cx, cy, cz);
            float* s = Tk; Tk = Tw; Tw = s;
        }
        int iz;
#pragma omp parallel for schedule(static)
        for (iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    const size_t i = EIDX(ix, iy, iz);
                    const int interior = ix > 0 && ix < nx - 1 && iy > 0 && iy < ny - 1 && iz > 0 && iz < nz - 1;
                    if (!interior) {
                        mu[i] = 0.0f;
                        continue;
                    }
                    float t = Tk[i];
                    float d2x = (Tk[EIDX(ix + 1, iy, iz)] - t) - (t - Tk[EIDX(ix - 1, iy, iz)]);
                    float d2y = (Tk[EIDX(ix, iy + 1, iz)] - t) - (t - Tk[EIDX(ix, iy - 1, iz)]);
                    float d2z = (Tk[EIDX(ix, iy, iz + 1)] - t) - (t - Tk[EIDX(ix, iy, iz - 1)]);
                    float lap = (d2x * cx + d2y * cy) + d2z * cz;
                    gCi[i] = gCi[i] + (dtlam * lk[i]) * lap;
                    mu[i] = (dtlam * Ci[i]) * lk[i];
                }
#pragma omp parallel for schedule(static)
        for (iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    const size_t i = EIDX(ix, iy, iz);
                    float m = mu[i];
                    float xm = ix > 0 ? mu[EIDX(ix - 1, iy, iz)] : 0.0f;
                    float xp = ix < nx - 1 ? mu[EIDX(ix + 1, iy, iz)] : 0.0f;
                    float ym = iy > 0 ? mu[EIDX(ix, iy - 1, iz)] : 0.0f;
                    float yp = iy < ny - 1 ? mu[EIDX(ix, iy + 1, iz)] : 0.0f;
                    float zm = iz > 0 ? mu[EIDX(ix, iy, iz - 1)] : 0.0f;
                    float zp = iz < nz - 1 ? mu[EIDX(ix, iy, iz + 1)] : 0.0f;
                    float d2x = (xp - m) - (m - xm);
                    float d2y = (yp - m) - (m - ym);
                    float d2z = (zp - m) - (m - zm);
                    lnext[i] = lk[i] + ((d2x * cx + d2y * cy) + d2z * cz);
                }
        memcpy(lk, lnext, n * sizeof(float));
    }
    free(kept); free(Tk); free(Tw); free(mu); free(lnext);
    return 0;
}

/* ------------------------------------------------------------ operators */
/* The operators of the kernel notation in FP32 on the widened values of A
 * (storage ST_F32 or a BF16 form; nz == 1: a 2-D field): op 0 the interior
 * values, ops 1-3 the second difference (A[p] - A[c]) - (A[c] - A[m]) along
 * x, y, z, op 4 the Laplacian (d2x*cx + d2y*cy) + d2z*cz with cx the FP32
 * rounding of rdx*rdx formed in FP64 (2-D: d2x*cx + d2y*cy).  out holds the
 * interior, x fastest. */
int emul_apply32(int op, float* out, const void* A, int nx, int ny, int nz, double rdx, double rdy, double rdz,
                 int storage)
{
    const int twod = nz == 1;
    if (op < 0 || op > 4 || nx < 3 || ny < 3 || (!twod && nz < 3) || (twod && op == 3)) return -1;
    if (storage != ST_F32 && storage != ST_BF16_SR && storage != ST_BF16_RNE) return -1;
    const size_t n = (size_t)nx * ny * nz;
    float* a = (float*)malloc(n * sizeof(float));
    if (!a) return -2;
    widen_field(a, A, n, storage);
    const float cx = (float)(rdx * rdx), cy = (float)(rdy * rdy), cz = (float)(rdz * rdz);
    const int z0 = twod ? 0 : 1, z1 = twod ? 1 : nz - 1;
    size_t o = 0;
    for (int iz = z0; iz < z1; ++iz)
        for (int iy = 1; iy < ny - 1; ++iy)
            for (int ix = 1; ix < nx - 1; ++ix) {
                const float t = a[EIDX(ix, iy, iz)];
                const float d2x = (a[EIDX(ix + 1, iy, iz)] - t) - (t - a[EIDX(ix - 1, iy, iz)]);
                const float d2y = (a[EIDX(ix, iy + 1, iz)] - t) - (t - a[EIDX(ix, iy - 1, iz)]);
                float d2z = 0.0f;
                if (!twod) d2z = (a[EIDX(ix, iy, iz + 1)] - t) - (t - a[EIDX(ix, iy, iz - 1)]);
                float v;
                switch (op) {
                case 0: v = t; break;
                case 1: v = d2x; break;
                case 2: v = d2y; break;
                case 3: v = d2z; break;
                default: v = twod ? d2x * cx + d2y * cy : (d2x * cx + d2y * cy) + d2z * cz; break;
                }
                out[o++] = v;
            }
    free(a);
    return 0;
}
