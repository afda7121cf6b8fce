/*
 * diff3d: explicit 3-D heat diffusion on one MI355X (gfx950), C ABI.
 *
 * The operation is the time step of Omlin & Raess, "High-performance xPU
 * Stencil Computations in Julia" (JuliaCon 2019), Fig. 1 (kernel `step!` and
 * driver `diffusion3D`):
 *
 *   on interior points (1 <= ix <= nx-2, same for y and z)
 *     T2 = T + dt*((lam*Ci)*((d2x(T)*cx + d2y(T)*cy) + d2z(T)*cz))
 *   with d2x(A) = (A[x+1] - A[x]) - (A[x] - A[x-1]) (likewise y, z) and
 *   cx = rdx*rdx, rdx = 1/dx (likewise y, z); boundary points are never
 *   written (fixed values); the two buffers then swap roles.
 *
 * Added to the paper's method: reduced-precision storage (FP32, BF16 with
 * FP32 arithmetic) and a checkpointed reverse sweep (adjoint) giving the
 * gradient of a loss of T_nt with respect to T0 and Ci.
 *
 * Conventions for every entry point:
 *  - Fields are dense nx*ny*nz arrays in device memory with linear index
 *    ix + nx*(iy + ny*iz): x is contiguous (the paper's column-major Julia
 *    arrays).  A torch tensor of shape (nz, ny, nx), contiguous, has this
 *    layout.  Element type is given by `dtype` (diff3d_dtype).
 *  - All buffers are owned by the caller.  The library never allocates or
 *    frees device memory and keeps no pointer after a call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work on it and return without synchronising, except where stated.
 *  - Scalars are passed as double.  FP32/BF16 forms round each of lam, dt
 *    and (1/h)^2 once to float.
 *  - Return value is a diff3d_status.  Arguments are validated on the host
 *    before anything is enqueued; on error nothing is enqueued.  Errors from
 *    the HIP runtime (launch failures) are reported as DIFF3D_EHIP.
 *  - Sizes: each of nx, ny, nz must be >= 3 (a grid with an interior) and
 *    nx*ny*nz < 2^40.
 */
#ifndef DIFF3D_H
#define DIFF3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DIFF3D_F64 = 0,       /* FP64 storage, FP64 arithmetic (the paper's Float64) */
    DIFF3D_F32 = 1,       /* FP32 storage, FP32 arithmetic */
    DIFF3D_BF16 = 2,      /* BF16 storage, FP32 arithmetic, stores rounded stochastically */
    DIFF3D_BF16_RNE = 3   /* BF16 storage, FP32 arithmetic, stores rounded to nearest even */
} diff3d_dtype;

typedef enum {
    DIFF3D_OK = 0,
    DIFF3D_EINVAL = -1,      /* bad pointer, size, count or aliasing */
    DIFF3D_EDTYPE = -2,      /* unknown dtype, or dtype not supported by this entry point */
    DIFF3D_EWORKSPACE = -3,  /* workspace missing or smaller than required */
    DIFF3D_EHIP = -4         /* the HIP runtime reported an error */
} diff3d_status;

typedef enum {
    DIFF3D_KERNEL_AUTO = 0,    /* the fastest validated variant: z-march single steps; in
                                  diff3d_run S-step passes (S = 4 for both BF16 forms;
                                  FP64: S = 4, 3 on x-y planes of at most 160^2 points;
                                  FP32: S = 4, 3 on x-y planes above 768^2 points); in
                                  diff3d_adjoint_run fused three-step reverse passes */
    DIFF3D_KERNEL_NAIVE = 1,   /* one thread per point, neighbours from cache */
    DIFF3D_KERNEL_ZMARCH = 2,  /* x-y tiles marching along z, planes in registers and LDS */
    DIFF3D_KERNEL_TB2 = 3,     /* diff3d_run: two steps per pass (temporal blocking), z-march
                                  for single steps; bit-identical results */
    DIFF3D_KERNEL_TBS = 4      /* diff3d_run: S steps per pass with the S-step kernel (S from
                                  diff3d_config.pass_steps), z-march for single steps; diff3d_stepn
                                  also uses it for two steps; diff3d_adjoint_run: fused reverse
                                  passes of min(S, 3) steps (forward states recomputed on chip);
                                  bit-identical results */
} diff3d_kernel;

/* Tile configuration override of one kernel family; all zero = the tuned
 * default.  p[] by family:
 *   zmarch, tb2 (single-step and two-step kernels): V (points per lane along
 *       x), R (rows per thread), NW (waves per workgroup), NT (1: Ci loads
 *       and T2 stores non-temporal);
 *   adj, adj2 (single-step and two-step adjoint kernels): V, R, NW, unused;
 *   tbs (S-step kernel): W0, H0 (region), NTH (threads), NT;
 *   rev (fused reverse passes): W0, H0, NTH, unused.
 * `steps` names the pass length a tbs or rev override applies to (2 ..
 * DIFF3D_MAX_PASS_STEPS; other pass lengths keep their defaults); it must be
 * 0 for the other families.  zlen = planes per z-chunk (0 = automatic).  An
 * override naming a configuration the library does not instantiate for the
 * call's dtype is rejected (DIFF3D_EINVAL, nothing enqueued). */
typedef struct {
    int steps;
    int p[4];
    int zlen;
} diff3d_tile;

/* Everything that selects how a call runs, owned by the caller and passed to
 * each call (NULL = all defaults, i.e. a zero-filled struct).  The library
 * keeps no state between calls: equal arguments give equal bits. */
typedef struct {
    int kernel;          /* diff3d_kernel */
    int pass_steps;      /* under DIFF3D_KERNEL_TBS: steps per pass of diff3d_run, 2 ..
                            DIFF3D_MAX_PASS_STEPS, or 0 for the dtype's default */
    int narrow;          /* 1: one point per lane in the z-march, two-step and adjoint kernels */
    int reserved;        /* must be 0 */
    uint64_t sr_seed;    /* key of the stochastic rounding of DIFF3D_BF16 */
    uint64_t sr_step;    /* index of the first time step the call takes (see diff3d_step) */
    diff3d_tile zmarch, tb2, tbs, adj, adj2, rev;
} diff3d_config;

/* Largest number of time steps one pass over memory can take (diff3d_stepn). */
#define DIFF3D_MAX_PASS_STEPS 4

/* Number of doubles in the device buffer `acc` of the reductions below. */
#define DIFF3D_REDUCE_DOUBLES 1025

/* Human-readable name of a status code (static string, never NULL). */
const char* diff3d_strerror(int status);

/* Element size in bytes of a dtype, or 0 if unknown. */
size_t diff3d_dtype_size(int dtype);

/* Driver scalars of Fig. 1 (host arithmetic only, no GPU work):
 *   dx = lx/(nx-1), dy, dz likewise; rdx = 1.0/dx etc.;
 *   dt = min(dx*dx, dy*dy, dz*dz)/lam/cimax/6.1, evaluated left to right,
 * where cimax is the maximum of Ci over the whole array (diff3d_max).
 * out receives {dx, dy, dz, rdx, rdy, rdz, dt}.  EINVAL if out is NULL,
 * a size is < 3, or lam or cimax is not positive. */
int diff3d_scalars(int nx, int ny, int nz, double lx, double ly, double lz, double lam,
                   double cimax, double* out);

/* Maximum of n elements of x (device, `dtype`), written as a double to
 * acc[0].  acc is a device buffer of DIFF3D_REDUCE_DOUBLES doubles used as
 * scratch; the result is deterministic. */
int diff3d_max(const void* x, size_t n, int dtype, double* acc, void* stream);

/* Reduced-precision storage (DIFF3D_F32, DIFF3D_BF16, DIFF3D_BF16_RNE): loads
 * widen to FP32, the step is evaluated in FP32 in the order above, and a
 * value is rounded to the storage type only when a state is written to
 * memory.  A pass that takes several steps on chip (diff3d_stepn, the time
 * loop) keeps its intermediate states in FP32, so BF16 results depend on the
 * pass lengths (diff3d_pass_plan); FP64 and FP32 results do not.
 * Stochastic rounding (DIFF3D_BF16): the state written after global step
 * index k (k = cfg->sr_step + the number of steps the call has taken before
 * that step) draws for point i the 16 random bits r of Philox4x32-10 with key
 * (sr_seed low word, sr_seed high word) and counter (g low word, g high word,
 * k low word, k high word), g = i / 8: the low (i even) or high (i odd) half
 * of output word (i % 8) / 2.  The stored BF16 value is the upper half of
 * the FP32 bit pattern plus r, truncated to its upper 16 bits (NaN and
 * infinity kept): it rounds up with probability equal to the discarded
 * fraction of a BF16 unit in the last place. */

/* One time step (Fig. 1, `step!`).  Writes the interior of T2 from T and Ci;
 * T2's boundary is not touched (the caller keeps it equal to T's, as
 * T2 = copy(T) does in the paper).  T2 must not alias T or Ci.  cfg selects
 * the kernel (naive or z-march; other values mean z-march) and the
 * stochastic rounding's seed and step index. */
int diff3d_step(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam,
                double dt, double rdx, double rdy, double rdz, int dtype, void* stream,
                const diff3d_config* cfg);

/* Two time steps in one pass over memory (temporal blocking): writes the
 * interior of T2 with the state two steps after T; FP64 and FP32 results are
 * bit-identical to two diff3d_step calls, BF16 keeps the intermediate state
 * in FP32 and rounds once (step index cfg->sr_step + 1).  Same buffer rules
 * as diff3d_step. */
int diff3d_step2(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam,
                 double dt, double rdx, double rdy, double rdz, int dtype, void* stream,
                 const diff3d_config* cfg);

/* nsteps time steps (1 <= nsteps <= DIFF3D_MAX_PASS_STEPS) in one pass over
 * memory (temporal blocking over S = nsteps steps): each workgroup reads its
 * tile of T padded by nsteps points on every side and computes the
 * intermediate states on shrinking regions on chip.  Writes the interior of
 * T2 with the state nsteps steps after T: FP64 and FP32 bit-identical to
 * nsteps diff3d_step calls; BF16 rounds once, with step index
 * cfg->sr_step + nsteps - 1.  nsteps = 1 is diff3d_step; nsteps = 2 runs the
 * kernel of diff3d_step2 except under DIFF3D_KERNEL_TBS (and, under
 * DIFF3D_KERNEL_AUTO, for the BF16 forms).  Same buffer rules as
 * diff3d_step; EINVAL for nsteps out of range. */
int diff3d_stepn(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam,
                 double dt, double rdx, double rdy, double rdz, int nsteps, int dtype, void* stream,
                 const diff3d_config* cfg);

/* The pass lengths diff3d_run takes for these arguments, in order (host
 * logic only).  Passes are at most S steps (the kernel's pass length for the
 * dtype and x-y plane size, or cfg->pass_steps under DIFF3D_KERNEL_TBS); a
 * pass never crosses a checkpointed state (a multiple of ckpt_every below
 * nt; ckpt_every = 0: no checkpoints); with the default pass length each
 * stretch between checkpoints is split into passes of near-equal length
 * (14 steps at S = 4: 4, 4, 3, 3), with a set pass length into passes of
 * exactly that length and a shorter last one.  Returns the number of passes
 * (writing at most max_lengths of them to lengths, which may be NULL), or a
 * negative diff3d_status. */
int diff3d_pass_plan(int nx, int ny, int nz, int nt, int ckpt_every, int dtype,
                     const diff3d_config* cfg, int* lengths, int max_lengths);

/* nt time steps with the buffer swap of Fig. 1.  First copies T's boundary
 * into T2, then runs the passes of diff3d_pass_plan, alternating
 * T -> T2 -> T ...  The result T_nt is always left in T (one extra copy when
 * the last pass ends in T2); T2 is scratch.
 * Checkpoints: if ckpt is not NULL, the states T_{j*C} for j = 1 .. nck-1,
 * C = ckpt_every, nck = ceil(nt/C), are stored in consecutive fields of ckpt
 * (field j-1 holds T_{j*C}, boundary included, each field rounded up to a
 * multiple of 256 bytes): the pass that reaches such a state writes it
 * there; this is the first part of the workspace of diff3d_adjoint_run,
 * which can then be called with ckpt_ready = 1.  ckpt_every must be >= 1
 * when ckpt is given.  nt = 0 leaves T unchanged.  Stochastic rounding uses
 * step indices cfg->sr_step .. cfg->sr_step + nt - 1. */
int diff3d_run(void* T, void* T2, const void* Ci, int nx, int ny, int nz, double lam, double dt,
               double rdx, double rdy, double rdz, int nt, int dtype, void* stream, void* ckpt,
               int ckpt_every, const diff3d_config* cfg);

/* Bytes of workspace for diff3d_adjoint_run with the same cfg: (nck - 1)
 * checkpoint fields, the fields for states recomputed inside a checkpoint
 * segment, and one field for the adjoint ping-pong, each
 * nx*ny*nz*sizeof(dtype) rounded up to a multiple of 256 bytes.  The
 * recomputed states are those at the starts of the fused reverse passes
 * (DIFF3D_KERNEL_AUTO, DIFF3D_KERNEL_TBS: ceil(L/P) - 1 fields, L =
 * min(ckpt_every, nt), P the fused pass length) or every state of a segment
 * (the other kernels: L - 1 fields).  Returns 0 for invalid arguments. */
size_t diff3d_adjoint_workspace_bytes(int nx, int ny, int nz, int nt, int ckpt_every, int dtype,
                                      const diff3d_config* cfg);

/* Reverse sweep of nt steps (the transpose of the step, derived by hand):
 * given gTnt = dLoss/dT_nt, writes gT0 = dLoss/dT0 and overwrites gCi with
 * dLoss/dCi (0 on the boundary).  Per step k = nt-1 .. 0, with
 * lambda_nt = gTnt and c = dt*lam*Ci:
 *   gCi += dt*lam*lambda_{k+1}*Lap(T_k)       on interior points
 *   mu   = dt*lam*Ci*lambda_{k+1} on interior points, 0 elsewhere
 *   lambda_k = lambda_{k+1} + Lap(mu)          at every point (mu = 0 outside)
 * Lap is the weighted 7-point expression of the step.  States T_k are
 * recomputed segment by segment from checkpoints every ckpt_every steps:
 * either every state of the segment (then one or two reverse steps per
 * launch), or only the states at the starts of fused reverse passes, which
 * recompute the states in between on chip (diff3d_kernel).  Checkpoints are
 * computed here from T0 unless ckpt_ready = 1, in which case the workspace
 * already holds them from diff3d_run with the same T0, Ci, scalars, nt,
 * ckpt_every and dtype).  Only DIFF3D_F64 and DIFF3D_F32 are supported
 * (EDTYPE otherwise).  gT0, gCi and the workspace must not overlap each
 * other or the inputs; ws_bytes must be at least
 * diff3d_adjoint_workspace_bytes(..., cfg). */
int diff3d_adjoint_run(const void* T0, const void* Ci, const void* gTnt, void* gT0, void* gCi,
                       void* workspace, size_t ws_bytes, int ckpt_ready, int nx, int ny, int nz,
                       double lam, double dt, double rdx, double rdy, double rdz, int nt,
                       int ckpt_every, int dtype, void* stream, const diff3d_config* cfg);

/* Loss of the gradient examples: L = 0.5*sum((T - Tt)^2) over all n points,
 * accumulated in FP64 into acc[0] (acc: DIFF3D_REDUCE_DOUBLES doubles of
 * device scratch; deterministic order), and the seed of the reverse sweep
 * r = T - Tt written to `seed` (may be NULL) in the storage dtype. */
int diff3d_loss(const void* T, const void* Tt, void* seed, size_t n, int dtype, double* acc,
                void* stream);

/* diff3d_loss for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result bits, with the partial sums in a
 * fixed array of DIFF3D_NOALLOC_PARTIALS doubles that the library holds on
 * each GPU it runs on until the process ends, instead of caller scratch.
 * out is one device double that receives L; seed as in diff3d_loss.  Every
 * call on one GPU uses that GPU's array, so calls that overlap on one GPU
 * (concurrent streams or threads) race and must be serialised by the
 * caller.  Allocates nothing, enqueues no memset.  EINVAL for NULL pointers
 * or n outside 1 .. 2^40-1; EHIP if the array's device address cannot be
 * looked up (first call on a device). */
#define DIFF3D_NOALLOC_PARTIALS 1024
int diff3d_loss_noalloc(const void* T, const void* Tt, void* seed, size_t n, int dtype, double* out,
                        void* stream);

/* Squared 2-norm of n elements of x, accumulated in FP64 into acc[0]
 * (deterministic order). */
int diff3d_norm2(const void* x, size_t n, int dtype, double* acc, void* stream);

/* Plain device copy of `bytes` bytes (16-byte vector loads and stores; the
 * measured copy bandwidth is the reachable-peak reference).  dst and src
 * must not overlap and must be 16-byte aligned. */
int diff3d_copy(void* dst, const void* src, size_t bytes, void* stream);

/* The 2-D form of the step (not printed in the paper, whose Fig. 1 is the
 * 3-D solver): the Fig. 1 expression without the z term,
 *   T2 = T + dt*((lam*Ci)*(d2x(T)*rdx^2 + d2y(T)*rdy^2))   on interior points,
 * on an nx x ny grid, linear index x + nx*y (x fastest); T2's boundary is not
 * written.  Storage types as for the 3-D step: FP64, FP32 and both BF16
 * forms (FP32 arithmetic; a value is rounded to BF16 only when a state is
 * written to memory, so BF16 results depend on the pass lengths).  Under
 * DIFF3D_BF16 the state written after global step index k (k = cfg->sr_step
 * + the number of steps the call has taken before that step) rounds point
 * i = x + nx*y with the random bits the 3-D step defines for index i and
 * step k (Philox4x32-10, key cfg->sr_seed).  Only cfg's sr_seed and sr_step
 * apply to the 2-D form (NULL: both zero).  Unknown dtype: DIFF3D_EDTYPE;
 * nx, ny >= 3; T2 must not overlap T or Ci (EINVAL).  Device pointers,
 * enqueued on `stream`. */
int diff2d_step(void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt,
                double rdx, double rdy, int dtype, void* stream, const diff3d_config* cfg);

/* nsteps steps of the 2-D form in one pass over memory (1 <= nsteps <=
 * DIFF2D_MAX_PASS_STEPS): the interior of T2 receives the state nsteps steps
 * after T, bit-identical to nsteps single steps for FP64 and FP32
 * (intermediate states stay in the compute type on chip; BF16 rounds once,
 * drawing with step index cfg->sr_step + nsteps - 1).  Precondition: T2's
 * boundary equals T's.  Same argument rules as diff2d_step; nsteps out of
 * range is EINVAL. */
#define DIFF2D_MAX_PASS_STEPS 8
int diff2d_stepn(void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt, double rdx,
                 double rdy, int nsteps, int dtype, void* stream, const diff3d_config* cfg);

/* nt steps of the 2-D form with the buffer swap: passes of several steps
 * each (diff2d_stepn; near-equal lengths of at most 7 steps for FP64 and 8
 * for the other types: nt = 20 with at most 8 is 7, 7, 6) alternating
 * between T and T2, after T's boundary is copied into T2 (and, for an odd
 * number of passes, all of T, the first pass then reading T2, so that the
 * last one writes T); the result T_nt is left in T (T2 is scratch),
 * bit-identical to nt single steps for FP64 and FP32.  Same
 * argument rules as diff2d_step, plus nt >= 0 and T not overlapping Ci;
 * nt = 0 leaves T unchanged. */
int diff2d_run(void* T, void* T2, const void* Ci, int nx, int ny, double lam, double dt, double rdx,
               double rdy, int nt, int dtype, void* stream, const diff3d_config* cfg);

/* The finite-difference operators of the paper's kernel notation (Fig. 1
 * composes the step of @inn, @d2_xi, @d2_yi and @d2_zi), applied to a whole
 * field.  Every stencil of the library is built of the same device functions,
 * so these calls show the operation order the steps use.  At interior point
 * (ix, iy, iz), 1 <= ix <= nx-2 (likewise y, z):
 *   DIFF3D_OP_INN    A[ix, iy, iz]                        (interior selection)
 *   DIFF3D_OP_D2_XI  (A[ix+1] - A[ix]) - (A[ix] - A[ix-1]) (along x; likewise
 *   DIFF3D_OP_D2_YI  along y with stride nx,
 *   DIFF3D_OP_D2_ZI  along z with stride nx*ny)
 *   DIFF3D_OP_LAP    (d2x*cx + d2y*cy) + d2z*cz, cx = rdx*rdx (likewise y, z):
 *                    the weighted Laplacian the step multiplies by lam*Ci*dt
 * The paper does not print the definition of @d2_xi: the difference of the two
 * one-sided differences is the reading taken (exactly A[x+1] - 2A[x] + A[x-1]
 * in real arithmetic).
 *
 * `in` is an nx*ny*nz field (layout as above); nz == 1 selects a 2-D field of
 * nx*ny points (linear index x + nx*y), for which D2_ZI is invalid and LAP
 * drops the z term (the 2-D step, diff2d_step).  `out` receives the interior,
 * (nx-2)*(ny-2)*max(nz-2, 1) elements, dense, x fastest, in the arithmetic
 * type: double for DIFF3D_F64, float for DIFF3D_F32 and both BF16 forms (BF16
 * inputs are widened exactly; nothing is rounded to BF16).  rdx, rdy, rdz are
 * used by LAP only (rounded once to float for the FP32 types).  Rejected
 * (nothing enqueued): unknown op (EINVAL), unknown dtype (EDTYPE), NULL
 * pointers, nx or ny < 3, nz == 2 or nz < 1, D2_ZI with nz == 1, and `out`
 * overlapping `in` (EINVAL).  Device pointers, enqueued on `stream`. */
typedef enum {
    DIFF3D_OP_INN = 0,
    DIFF3D_OP_D2_XI = 1,
    DIFF3D_OP_D2_YI = 2,
    DIFF3D_OP_D2_ZI = 3,
    DIFF3D_OP_LAP = 4
} diff3d_op;
int diff3d_apply(int op, void* out, const void* in, int nx, int ny, int nz, double rdx, double rdy,
                 double rdz, int dtype, void* stream);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the counter-based
 * generator behind the stochastic rounding: out = bijection of ctr under
 * key.  Host function (same code as on the device), for tests. */
void diff3d_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Library version string. */
const char* diff3d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DIFF3D_H */
