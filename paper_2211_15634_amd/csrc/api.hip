// C ABI of the diff3d library: argument validation, kernel selection and
// launch, the time loop with the buffer swap, and the checkpointed reverse
// sweep.  Everything is enqueued on the caller's stream; no device memory is
// allocated here.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "adjoint_launch.hpp"
#include "diff2d_launch.hpp"
#include "diff3d.h"
#include "fd_apply.hpp"
#include "forward_launch.hpp"
#include "host_common.hpp"
#include "util_launch.hpp"

using namespace diff3d;

namespace {

// The time loop of Fig. 1: states alternate between T and T2, except that
// the pass reaching T_{j*C} (j >= 1, j*C <= klast) writes it into checkpoint
// field j-1, from which the next pass reads.  With want_result the final
// state is left in T.
int run_loop(int dtype, void* T, void* T2, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
             double rdy, double rdz, int nt, hipStream_t st, void* ckpt, int C, size_t field_stride, int klast,
             bool want_result, const diff3d_config& c)
{
    int rc = boundary_dispatch(dtype, T2, T, nx, ny, nz, st);
    if (rc) return rc;
    const size_t fbytes = npoints(nx, ny, nz) * elem_size(dtype);
    void* cur = T;                                // holds the current state
    for_each_pass(dtype, nx, ny, nt, ckpt ? C : 0, klast, c, [&](int it, int n) {
        if (rc) return;
        const int k = it + n;
        // a pass ending on a checkpointed state writes it into its slot,
        // whose boundary is set first (passes write interior points only;
        // T's boundary is the initial one throughout)
        void* dst = cur == T ? T2 : T;
        if (ckpt && k % C == 0 && k <= klast) {
            dst = static_cast<char*>(ckpt) + (size_t)(k / C - 1) * field_stride;
            rc = boundary_dispatch(dtype, dst, T, nx, ny, nz, st);
            if (rc) return;
        }
        rc = pass_dispatch(dtype, dst, cur, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, n, c.sr_step + (uint64_t)it, c,
                           st);
        cur = dst;
    });
    if (rc) return rc;
    if (want_result && cur != T) return copy_bytes(T, cur, fbytes, st);
    return DIFF3D_OK;
}

inline int nck_of(int nt, int C) { return nt > 0 ? (nt + C - 1) / C : 0; }

// Device scratch of diff3d_loss_noalloc: the partial sums of its first
// reduction pass (one per workgroup, at most kRedParts).  Every GPU the
// library runs on holds its own copy until the process ends; calls on one
// GPU share it.
__device__ __align__(256) double scratch[kRedParts];

// The device address of `scratch` on each device, looked up once per device
// with that device current (the host-side name is only a stand-in).
constexpr int kMaxDevices = 64;
std::atomic<double*> g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;

int scratch_on_current_device(double** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DIFF3D_EHIP;
    double* p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_addr[dev].load(std::memory_order_acquire);
        if (!p) {
            void* q = nullptr;
            if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return DIFF3D_EHIP;
            p = static_cast<double*>(q);
            g_scratch_addr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return DIFF3D_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* diff3d_strerror(int status)
{
    switch (status) {
    case DIFF3D_OK: return "ok";
    case DIFF3D_EINVAL: return "invalid argument (pointer, size, count or aliasing)";
    case DIFF3D_EDTYPE: return "unsupported dtype";
    case DIFF3D_EWORKSPACE: return "workspace missing or too small";
    case DIFF3D_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

size_t diff3d_dtype_size(int dtype) { return elem_size(dtype); }

const char* diff3d_version(void) { return "diff3d 0.1 gfx950"; }

int diff3d_scalars(int nx, int ny, int nz, double lx, double ly, double lz, double lam, double cimax, double* out)
{
    if (!out || check_grid(nx, ny, nz)) return DIFF3D_EINVAL;
    if (!(lam > 0.0) || !(cimax > 0.0) || !(lx > 0.0) || !(ly > 0.0) || !(lz > 0.0)) return DIFF3D_EINVAL;
    const double dx = lx / (nx - 1), dy = ly / (ny - 1), dz = lz / (nz - 1);
    double m = dx * dx;
    if (dy * dy < m) m = dy * dy;
    if (dz * dz < m) m = dz * dz;
    out[0] = dx;
    out[1] = dy;
    out[2] = dz;
    out[3] = 1.0 / dx;
    out[4] = 1.0 / dy;
    out[5] = 1.0 / dz;
    out[6] = m / lam / cimax / 6.1;
    return DIFF3D_OK;
}

int diff3d_max(const void* x, size_t n, int dtype, double* acc, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!x || !acc || n == 0) return DIFF3D_EINVAL;
    return reduce_dispatch<RED_MAX>(dtype, x, nullptr, nullptr, n, acc + 1, acc, as_stream(stream));
}

int diff3d_loss(const void* T, const void* Tt, void* seed, size_t n, int dtype, double* acc, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T || !Tt || !acc || n == 0) return DIFF3D_EINVAL;
    return reduce_dispatch<RED_SUMSQ_DIFF>(dtype, T, Tt, seed, n, acc + 1, acc, as_stream(stream));
}

int diff3d_loss_noalloc(const void* T, const void* Tt, void* seed, size_t n, int dtype, double* out, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T || !Tt || !out || n == 0 || n >= kMaxPoints) return DIFF3D_EINVAL;
    double* partials = nullptr;
    const int rc = scratch_on_current_device(&partials);
    if (rc) return rc;
    return reduce_dispatch<RED_SUMSQ_DIFF>(dtype, T, Tt, seed, n, partials, out, as_stream(stream));
}

int diff3d_norm2(const void* x, size_t n, int dtype, double* acc, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!x || !acc || n == 0) return DIFF3D_EINVAL;
    return reduce_dispatch<RED_SUMSQ>(dtype, x, nullptr, nullptr, n, acc + 1, acc, as_stream(stream));
}

int diff3d_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (bytes == 0) return DIFF3D_OK;
    if (!dst || !src || overlap(dst, bytes, src, bytes)) return DIFF3D_EINVAL;
    if ((uintptr_t)dst % 16 || (uintptr_t)src % 16) return DIFF3D_EINVAL;
    return copy_bytes(dst, src, bytes, as_stream(stream));
}

// Common checks of the forward entry points: dtype, pointers, grid, the
// configuration, and T2 overlapping neither T nor Ci.
static int check_step_args(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, int dtype,
                           const diff3d_config& c)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T2 || !T || !Ci || check_grid(nx, ny, nz)) return DIFF3D_EINVAL;
    if (check_forward_config(c, dtype)) return DIFF3D_EINVAL;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb)) return DIFF3D_EINVAL;
    return DIFF3D_OK;
}

int diff3d_step(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, int dtype, void* stream, const diff3d_config* cfg)
{
    const diff3d_config c = config_of(cfg);
    const int rc = check_step_args(T2, T, Ci, nx, ny, nz, dtype, c);
    if (rc) return rc;
    return step_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c.sr_step, c, as_stream(stream));
}

int diff3d_step2(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, int dtype, void* stream, const diff3d_config* cfg)
{
    const diff3d_config c = config_of(cfg);
    const int rc = check_step_args(T2, T, Ci, nx, ny, nz, dtype, c);
    if (rc) return rc;
    return pair_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c.sr_step + 1, c, as_stream(stream));
}

int diff3d_stepn(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, int nsteps, int dtype, void* stream, const diff3d_config* cfg)
{
    const diff3d_config c = config_of(cfg);
    const int rc = check_step_args(T2, T, Ci, nx, ny, nz, dtype, c);
    if (rc) return rc;
    if (nsteps < 1 || nsteps > DIFF3D_MAX_PASS_STEPS) return DIFF3D_EINVAL;
    return pass_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, c.sr_step, c,
                         as_stream(stream));
}

int diff3d_pass_plan(int nx, int ny, int nz, int nt, int ckpt_every, int dtype, const diff3d_config* cfg,
                     int* lengths, int max_lengths)
{
    const diff3d_config c = config_of(cfg);
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (check_grid(nx, ny, nz) || nt < 0 || ckpt_every < 0 || max_lengths < 0) return DIFF3D_EINVAL;
    if (check_forward_config(c, dtype)) return DIFF3D_EINVAL;
    int count = 0;
    for_each_pass(dtype, nx, ny, nt, ckpt_every, nt - 1, c, [&](int, int n) {
        if (lengths && count < max_lengths) lengths[count] = n;
        ++count;
    });
    return count;
}

int diff3d_run(void* T, void* T2, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
               double rdy, double rdz, int nt, int dtype, void* stream, void* ckpt, int ckpt_every,
               const diff3d_config* cfg)
{
    const diff3d_config c = config_of(cfg);
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T || !T2 || !Ci || check_grid(nx, ny, nz) || nt < 0) return DIFF3D_EINVAL;
    if (check_forward_config(c, dtype)) return DIFF3D_EINVAL;
    if (ckpt && ckpt_every < 1) return DIFF3D_EINVAL;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb) || overlap(T, fb, Ci, fb)) return DIFF3D_EINVAL;
    const size_t stride = align256(fb);
    if (ckpt) {
        const int nck = nck_of(nt, ckpt_every);
        const size_t cb = nck > 1 ? (size_t)(nck - 1) * stride : 0;
        if (cb && (overlap(ckpt, cb, T, fb) || overlap(ckpt, cb, T2, fb) || overlap(ckpt, cb, Ci, fb)))
            return DIFF3D_EINVAL;
    }
    if (nt == 0) return DIFF3D_OK;
    return run_loop(dtype, T, T2, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nt, as_stream(stream), ckpt, ckpt_every,
                    stride, nt - 1, true, c);
}

size_t diff3d_adjoint_workspace_bytes(int nx, int ny, int nz, int nt, int ckpt_every, int dtype,
                                      const diff3d_config* cfg)
{
    const diff3d_config c = config_of(cfg);
    if (!known_dtype(dtype) || check_grid(nx, ny, nz) || nt < 0 || ckpt_every < 1) return 0;
    if (check_forward_config(c, dtype) || check_adjoint_config(c, dtype)) return 0;
    const size_t stride = align256(npoints(nx, ny, nz) * elem_size(dtype));
    const int nck = nck_of(nt, ckpt_every);
    const size_t fields =
        (size_t)(nck > 1 ? nck - 1 : 0) + (size_t)recompute_fields(dtype, nt, ckpt_every, c) + 1;
    return fields * stride;
}

int diff3d_adjoint_run(const void* T0, const void* Ci, const void* gTnt, void* gT0, void* gCi, void* workspace,
                       size_t ws_bytes, int ckpt_ready, int nx, int ny, int nz, double lam, double dt, double rdx,
                       double rdy, double rdz, int nt, int ckpt_every, int dtype, void* stream,
                       const diff3d_config* cfg)
{
    const diff3d_config c = config_of(cfg);
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (dtype != DIFF3D_F64 && dtype != DIFF3D_F32) return DIFF3D_EDTYPE;
    if (!T0 || !Ci || !gTnt || !gT0 || !gCi || check_grid(nx, ny, nz) || nt < 0 || ckpt_every < 1)
        return DIFF3D_EINVAL;
    if (check_forward_config(c, dtype) || check_adjoint_config(c, dtype)) return DIFF3D_EINVAL;
    const size_t need = diff3d_adjoint_workspace_bytes(nx, ny, nz, nt, ckpt_every, dtype, cfg);
    if (!workspace || ws_bytes < need) return DIFF3D_EWORKSPACE;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    const void* ins[3] = {T0, Ci, gTnt};
    void* outs[2] = {gT0, gCi};
    for (int o = 0; o < 2; ++o) {
        for (int i = 0; i < 3; ++i)
            if (overlap(outs[o], fb, ins[i], fb)) return DIFF3D_EINVAL;
        if (overlap(outs[o], fb, workspace, need)) return DIFF3D_EINVAL;
    }
    if (overlap(gT0, fb, gCi, fb)) return DIFF3D_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (overlap(workspace, need, ins[i], fb)) return DIFF3D_EINVAL;

    hipStream_t st = as_stream(stream);
    const int C = ckpt_every;
    const size_t stride = align256(fb);
    char* ws = static_cast<char*>(workspace);
    const int nck = nck_of(nt, C);
    auto slot = [&](int j) -> void* { return ws + (size_t)(j - 1) * stride; };   // T_{jC}, j >= 1
    const int nseg = recompute_fields(dtype, nt, C, c);
    char* seg0 = ws + (size_t)(nck > 1 ? nck - 1 : 0) * stride;                  // recompute fields
    auto seg = [&](int i) -> void* { return seg0 + (size_t)i * stride; };
    void* W = seg0 + (size_t)nseg * stride;                                      // adjoint ping-pong

    int rc = zero_bytes(gCi, fb, st);
    if (rc) return rc;
    if (nt == 0) return copy_bytes(gT0, gTnt, fb, st);

    if (!ckpt_ready && nck > 1) {
        // forward from T0 on the two scratch fields W and gT0, filling the slots
        rc = copy_bytes(W, T0, fb, st);
        const int last = (nck - 1) * C;
        if (!rc) rc = run_loop(dtype, W, gT0, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, last, st, ws, C, stride, last,
                               false, c);
        if (rc) return rc;
    }
    // recompute fields need T0's boundary (steps write interior points only)
    for (int i = 0; i < nseg; ++i) {
        rc = boundary_dispatch(dtype, seg(i), T0, nx, ny, nz, st);
        if (rc) return rc;
    }

    if (rev_fused(c)) {
        // Fused reverse passes of P steps (the first pass of a segment takes
        // the remainder): only the states at pass starts are recomputed (by
        // forward passes of the same lengths), the pass recomputes the rest
        // on chip.  lambda alternates between gT0 and W so that the last
        // launch writes gT0.
        const int P = rev_pass_steps(dtype, c);
        auto npass = [&](int len) { return (len + P - 1) / P; };
        long nlaunch = 0;
        for (int j = nck - 1; j >= 0; --j) nlaunch += npass(((j * C + C < nt) ? j * C + C : nt) - j * C);
        long launch = 0;
        const void* lin = gTnt;
        for (int j = nck - 1; j >= 0; --j) {
            const int s = j * C;
            const int len = ((s + C < nt) ? s + C : nt) - s;
            const int m = npass(len);
            const int r = len - (m - 1) * P;      // first pass: 1 .. P steps
            const void* base = j == 0 ? T0 : slot(j);
            // states at the starts of passes 1 .. m-1 into seg(0) .. seg(m-2)
            const void* src = base;
            for (int i = 1; i < m; ++i) {
                rc = pass_dispatch(dtype, seg(i - 1), src, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, i == 1 ? r : P, 0,
                                   c, st);
                if (rc) return rc;
                src = seg(i - 1);
            }
            for (int i = m - 1; i >= 0; --i) {
                const int n = i == 0 ? r : P;
                const void* Tk = i == 0 ? base : seg(i - 1);
                void* out = ((nlaunch - 1 - launch) % 2 == 0) ? gT0 : W;
                rc = n >= 2 ? rev_dispatch(dtype, n, out, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st)
                            : adj_dispatch(dtype, out, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
                if (rc) return rc;
                lin = out;
                ++launch;
            }
        }
        return DIFF3D_OK;
    }

    // adjoint launches (two steps per launch inside a segment where enabled);
    // lambda alternates between gT0 and W so that the last launch writes gT0
    const bool apairs = c.kernel == DIFF3D_KERNEL_TB2;
    long nlaunch = 0;
    for (int j = nck - 1; j >= 0; --j) {
        const int len = ((j * C + C < nt) ? j * C + C : nt) - j * C;
        nlaunch += apairs ? (len + 1) / 2 : len;
    }
    long launch = 0;
    const void* lin = gTnt;
    for (int j = nck - 1; j >= 0; --j) {
        const int s = j * C;
        const int e = (s + C < nt) ? s + C : nt;
        const void* base = j == 0 ? T0 : slot(j);
        // states T_{s+1} .. T_{e-1} into seg(0) .. seg(e-s-2), two at a time
        // where possible (one pass writing both the intermediate and the
        // second state), the two-step kernel unless single steps are selected
        const void* src = base;
        const bool pairs = c.kernel == DIFF3D_KERNEL_TB2;
        for (int k = s; k < e - 1;) {
            if (pairs && k + 2 <= e - 1) {
                rc = pair_mid_dispatch(dtype, seg(k - s + 1), seg(k - s), src, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz,
                                       c, st);
                src = seg(k - s + 1);
                k += 2;
            } else {
                rc = step_dispatch(dtype, seg(k - s), src, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, 0, c, st);
                src = seg(k - s);
                k += 1;
            }
            if (rc) return rc;
        }
        auto state = [&](int k) -> const void* { return k == s ? base : seg(k - s - 1); };
        for (int k = e - 1; k >= s;) {
            void* out = ((nlaunch - 1 - launch) % 2 == 0) ? gT0 : W;
            if (apairs && k - 1 >= s) {
                rc = adj2_dispatch(dtype, out, lin, Ci, state(k), state(k - 1), gCi, nx, ny, nz, lam, dt, rdx, rdy,
                                   rdz, c, st);
                k -= 2;
            } else {
                rc = adj_dispatch(dtype, out, lin, Ci, state(k), gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
                k -= 1;
            }
            if (rc) return rc;
            lin = out;
            ++launch;
        }
    }
    return DIFF3D_OK;
}

// ------------------------------------------------------------- 2-D form

static int check2d(const void* T2, const void* T, const void* Ci, int nx, int ny, int dtype)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T2 || !T || !Ci || nx < 3 || ny < 3 || (size_t)nx * (size_t)ny >= kMaxPoints) return DIFF3D_EINVAL;
    const size_t fb = (size_t)nx * ny * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb)) return DIFF3D_EINVAL;
    return DIFF3D_OK;
}

int diff2d_step(void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt, double rdx,
                double rdy, int dtype, void* stream, const diff3d_config* cfg)
{
    const int rc = check2d(T2, T, Ci, nx, ny, dtype);
    if (rc) return rc;
    const diff3d_config c = config_of(cfg);
    return step2dn_dispatch(dtype, 1, T2, T, Ci, nx, ny, lam, dt, rdx, rdy, c.sr_seed, c.sr_step,
                            as_stream(stream));
}

int diff2d_stepn(void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt, double rdx,
                 double rdy, int nsteps, int dtype, void* stream, const diff3d_config* cfg)
{
    const int rc = check2d(T2, T, Ci, nx, ny, dtype);
    if (rc) return rc;
    if (nsteps < 1 || nsteps > kMaxSteps2d) return DIFF3D_EINVAL;
    const diff3d_config c = config_of(cfg);
    return step2dn_dispatch(dtype, nsteps, T2, T, Ci, nx, ny, lam, dt, rdx, rdy, c.sr_seed,
                            c.sr_step + (uint64_t)(nsteps - 1), as_stream(stream));
}

int diff2d_run(void* T, void* T2, const void* Ci, int nx, int ny, double lam, double dt, double rdx, double rdy,
               int nt, int dtype, void* stream, const diff3d_config* cfg)
{
    int rc = check2d(T2, T, Ci, nx, ny, dtype);
    if (rc) return rc;
    const size_t fb = (size_t)nx * ny * elem_size(dtype);
    if (nt < 0 || overlap(T, fb, Ci, fb)) return DIFF3D_EINVAL;
    if (nt == 0) return DIFF3D_OK;
    const diff3d_config c = config_of(cfg);
    hipStream_t st = as_stream(stream);
    // passes of near-equal length, at most P steps each, ping-ponging; the
    // state a pass stores draws with the index of its last step.  Both
    // buffers carry T's boundary: an even number of passes starts from T
    // (T2 needs only the boundary), an odd number from T2 = copy(T), so the
    // last pass always writes T
    const int P = run2d_pass_steps(dtype);
    const int m = (nt + P - 1) / P;
    void* a = T;
    void* b = T2;
    if (m % 2) {
        rc = copy_bytes(T2, T, fb, st);
        a = T2;
        b = T;
    } else {
        rc = boundary2d_dispatch(dtype, T2, T, nx, ny, st);
    }
    for (int i = 0, done = 0; i < m && !rc; ++i) {
        const int n = (nt - done + (m - i) - 1) / (m - i);
        rc = step2dn_dispatch(dtype, n, b, a, Ci, nx, ny, lam, dt, rdx, rdy, c.sr_seed,
                              c.sr_step + (uint64_t)(done + n - 1), st);
        done += n;
        void* s = a;
        a = b;
        b = s;
    }
    if (!rc && a != T) rc = copy_bytes(T, a, fb, st);
    return rc;
}

// ------------------------------------------------------------- operators

int diff3d_apply(int op, void* out, const void* in, int nx, int ny, int nz, double rdx, double rdy, double rdz,
                 int dtype, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (op < DIFF3D_OP_INN || op > DIFF3D_OP_LAP) return DIFF3D_EINVAL;
    if (!out || !in || nx < 3 || ny < 3 || nz < 1 || nz == 2) return DIFF3D_EINVAL;
    if (nz == 1 && op == DIFF3D_OP_D2_ZI) return DIFF3D_EINVAL;
    if (npoints(nx, ny, nz) >= kMaxPoints) return DIFF3D_EINVAL;
    const size_t ib = npoints(nx, ny, nz) * elem_size(dtype);
    const size_t ob = npoints(nx - 2, ny - 2, nz == 1 ? 1 : nz - 2) * (dtype == DIFF3D_F64 ? 8 : 4);
    if (overlap(out, ob, in, ib)) return DIFF3D_EINVAL;
    return apply_dispatch(dtype, op, out, in, nx, ny, nz, rdx, rdy, rdz, as_stream(stream));
}

void diff3d_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const u32x4 r = philox4x32_10(u32x4{ctr[0], ctr[1], ctr[2], ctr[3]}, key[0], key[1]);
    out[0] = r.x;
    out[1] = r.y;
    out[2] = r.z;
    out[3] = r.w;
}

}  // extern "C"
