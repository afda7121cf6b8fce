// Forward step launches: tile configuration tables and defaults per dtype,
// the single-step, two-step and S-step launchers, their dispatch, the pass
// plan of the time loop and the validation of the caller's overrides.
#pragma once

#include "launch_plan.hpp"
#include "step_kernels.hpp"
#include "tb_kernels.hpp"
#include "tbs_kernels.hpp"

namespace diff3d {
namespace {

// ------------------------------------------------------------------ forward
// Arguments of a forward launch.  `draw_step` is the step index of the
// stochastic rounding of the state the launch stores (the index of the last
// step it takes).
template <int DT>
StepArgs<DT> make_step_args(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                            double rdx, double rdy, double rdz, uint64_t sr_seed, uint64_t draw_step)
{
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    StepArgs<DT> a;
    a.T2 = static_cast<S*>(T2);
    a.T = static_cast<const S*>(T);
    a.Ci = static_cast<const S*>(Ci);
    a.Tmid = nullptr;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.lam = (C)lam;
    a.dt = (C)dt;
    a.cx = (C)(rdx * rdx);
    a.cy = (C)(rdy * rdy);
    a.cz = (C)(rdz * rdz);
    a.sr.k0 = (uint32_t)sr_seed;
    a.sr.k1 = (uint32_t)(sr_seed >> 32);
    a.sr.s0 = (uint32_t)draw_step;
    a.sr.s1 = (uint32_t)(draw_step >> 32);
    return a;
}

template <int DT>
int launch_naive(const StepArgs<DT>& a, hipStream_t st)
{
    dim3 grid((unsigned)((a.nx - 2 + 63) / 64), (unsigned)((a.ny - 2 + 3) / 4), (unsigned)min(a.nz - 2, 65535));
    step_naive<DT><<<grid, 256, 0, st>>>(a);
    return hip_status();
}

// Instantiated forward configurations per storage size (V*sizeof(S) <= 16).
#define DIFF3D_FWD_CFGS_8(X) X(1, 4, 4, 0) X(1, 8, 4, 0) X(1, 4, 8, 0) X(2, 4, 4, 0) X(2, 8, 4, 0) X(2, 2, 8, 0) \
    X(2, 4, 8, 0) X(2, 4, 4, 1) X(2, 8, 4, 1) X(2, 4, 8, 1)
#define DIFF3D_FWD_CFGS_4(X) X(1, 4, 4, 0) X(2, 4, 4, 0) X(2, 8, 4, 0) X(2, 4, 8, 0) X(4, 2, 4, 0) X(4, 4, 4, 0) \
    X(4, 2, 8, 0) X(4, 2, 8, 1) X(4, 4, 4, 1) X(2, 8, 4, 1)
#define DIFF3D_FWD_CFGS_2(X) X(1, 4, 4, 0) X(2, 4, 4, 0) X(2, 8, 4, 0) X(4, 2, 4, 0) X(4, 4, 4, 0) X(4, 2, 8, 0) \
    X(4, 1, 8, 0) X(8, 1, 8, 0) X(8, 2, 4, 0) X(4, 4, 4, 1) X(2, 8, 4, 1) X(4, 2, 8, 1)

template <int DT>
struct FwdDefaults;
template <> struct FwdDefaults<DIFF3D_F64> { static constexpr ZKey wide{2, 4, 4, 1}; static constexpr int zdef = 128; };
template <> struct FwdDefaults<DIFF3D_F32> { static constexpr ZKey wide{4, 4, 4, 1}; static constexpr int zdef = 32; };
template <> struct FwdDefaults<DIFF3D_BF16> { static constexpr ZKey wide{4, 1, 8, 0}; static constexpr int zdef = 32; };
template <> struct FwdDefaults<DIFF3D_BF16_RNE> {
    static constexpr ZKey wide{4, 1, 8, 0};
    static constexpr int zdef = 64;
};
constexpr ZKey kNarrow{1, 4, 4, 0};

// Is a (V, R, NW, NT) key instantiated for storage of `size` bytes?
inline bool fwd_has(int size, const ZKey& k)
{
#define DIFF3D_HAS(v, r, nw, nt) || key_eq(k, v, r, nw, nt)
    switch (size) {
    case 8: return false DIFF3D_FWD_CFGS_8(DIFF3D_HAS);
    case 4: return false DIFF3D_FWD_CFGS_4(DIFF3D_HAS);
    case 2: return false DIFF3D_FWD_CFGS_2(DIFF3D_HAS);
    default: return false;
    }
#undef DIFF3D_HAS
}

template <int DT, int V, int R, int NW, int NT>
int launch_zmarch_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz - 2, 64 * V, R * NW, zlen_req, zdef);
    step_zmarch<DT, V, R, NW, NT != 0><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT>
int launch_zmarch(const StepArgs<DT>& a, const diff3d_config& c, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    ZKey k = zkey_of(c.zmarch, FwdDefaults<DT>::wide);
    if (c.narrow || !vec_ok<S>(a.nx, k.V, a.T, a.T2, a.Ci)) k = kNarrow;
    const int zdef = FwdDefaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw, nt) \
    if (key_eq(k, v, r, nw, nt)) return launch_zmarch_cfg<DT, v, r, nw, nt>(a, st, c.zmarch.zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_FWD_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(S) == 4) {
        DIFF3D_FWD_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_FWD_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;   // not reached: overrides are validated before any launch
}

// Two-step (temporal-blocked) configurations.
#define DIFF3D_TB2_CFGS_8(X) X(1, 4, 4, 1) X(2, 2, 4, 1) X(1, 2, 8, 1) X(2, 2, 8, 1) X(2, 1, 8, 1) X(1, 4, 8, 1)
#define DIFF3D_TB2_CFGS_4(X) X(1, 4, 4, 1) X(2, 2, 4, 1) X(4, 1, 8, 1) X(2, 2, 8, 1) X(4, 2, 4, 1) X(2, 1, 8, 1)
#define DIFF3D_TB2_CFGS_2(X) X(1, 4, 4, 1) X(4, 1, 8, 1) X(4, 2, 4, 1) X(8, 1, 8, 1) X(2, 2, 8, 1) X(8, 1, 4, 1)

template <int DT>
struct Tb2Defaults;
template <> struct Tb2Defaults<DIFF3D_F64> { static constexpr ZKey wide{2, 2, 8, 1}; static constexpr int zdef = 256; };
template <> struct Tb2Defaults<DIFF3D_F32> { static constexpr ZKey wide{2, 2, 8, 1}; static constexpr int zdef = 128; };
template <> struct Tb2Defaults<DIFF3D_BF16> {
    static constexpr ZKey wide{4, 2, 4, 1};
    static constexpr int zdef = 128;
};
template <> struct Tb2Defaults<DIFF3D_BF16_RNE> {
    static constexpr ZKey wide{4, 2, 4, 1};
    static constexpr int zdef = 128;
};
constexpr ZKey kNarrowTb2{1, 4, 4, 1};

inline bool tb2_has(int size, const ZKey& k)
{
#define DIFF3D_HAS(v, r, nw, nt) || key_eq(k, v, r, nw, nt)
    switch (size) {
    case 8: return false DIFF3D_TB2_CFGS_8(DIFF3D_HAS);
    case 4: return false DIFF3D_TB2_CFGS_4(DIFF3D_HAS);
    case 2: return false DIFF3D_TB2_CFGS_2(DIFF3D_HAS);
    default: return false;
    }
#undef DIFF3D_HAS
}

template <int DT, int V, int R, int NW, int NT, bool MID>
int launch_tb2_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz - 2, 64 * V, R * NW, zlen_req, zdef);
    step_tb2<DT, V, R, NW, NT != 0, MID><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT, bool MID>
int launch_tb2(const StepArgs<DT>& a, const diff3d_config& c, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    ZKey k = zkey_of(c.tb2, Tb2Defaults<DT>::wide);
    if (c.narrow || !vec_ok<S>(a.nx, k.V, a.T, a.T2, a.Ci)) k = kNarrowTb2;
    const int zdef = Tb2Defaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw, nt) \
    if (key_eq(k, v, r, nw, nt)) return launch_tb2_cfg<DT, v, r, nw, nt, MID>(a, st, c.tb2.zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_TB2_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(S) == 4) {
        DIFF3D_TB2_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_TB2_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

// Two steps T -> T2 (T^{k+2}); the stored state draws with `draw_step`.
template <int DT>
int launch_pair(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, uint64_t draw_step, const diff3d_config& c, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c.sr_seed, draw_step);
    return launch_tb2<DT, false>(a, c, st);
}

// Two steps T -> Tmid (T^{k+1}) and T2 (T^{k+2}), interior points of both.
template <int DT>
int launch_pair_mid(void* T2, void* Tmid, const void* T, const void* Ci, int nx, int ny, int nz, double lam,
                    double dt, double rdx, double rdy, double rdz, const diff3d_config& c, hipStream_t st)
{
    StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, 0, 0);
    a.Tmid = static_cast<typename Traits<DT>::S*>(Tmid);
    return launch_tb2<DT, true>(a, c, st);
}

int pair_mid_dispatch(int dtype, void* T2, void* Tmid, const void* T, const void* Ci, int nx, int ny, int nz,
                      double lam, double dt, double rdx, double rdy, double rdz, const diff3d_config& c,
                      hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_pair_mid<DIFF3D_F64>(T2, Tmid, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    case DIFF3D_F32:
        return launch_pair_mid<DIFF3D_F32>(T2, Tmid, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    default: return DIFF3D_EDTYPE;
    }
}

int pair_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, uint64_t draw_step, const diff3d_config& c, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_pair<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    case DIFF3D_F32:
        return launch_pair<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    case DIFF3D_BF16:
        return launch_pair<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    case DIFF3D_BF16_RNE:
        return launch_pair<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    default: return DIFF3D_EDTYPE;
    }
}

#define DIFF3D_TBS_CFGS_8(X) X(2, 64, 16, 512, 1) X(2, 64, 32, 512, 0) X(3, 64, 32, 512, 0) X(3, 64, 32, 1024, 0) \
    X(4, 64, 32, 512, 0) X(4, 64, 32, 1024, 0)
#define DIFF3D_TBS_CFGS_4(X) X(2, 64, 32, 512, 1) X(2, 64, 64, 1024, 0) X(3, 64, 32, 512, 0) X(3, 128, 32, 1024, 0) \
    X(4, 64, 32, 512, 0) X(4, 64, 48, 768, 0) X(4, 64, 32, 1024, 0)
#define DIFF3D_TBS_CFGS_2(X) X(2, 64, 32, 512, 1) X(2, 64, 32, 1024, 0) X(3, 64, 32, 1024, 0) X(4, 64, 32, 1024, 0)

template <int DT>
struct TbsDefaults;
template <> struct TbsDefaults<DIFF3D_F64> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 512, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};
// FP32 four-step passes on 64 x 32 regions of 1024 threads (62 VGPRs, 70 KB
// of LDS: two workgroups per CU) are an override, not the default: 6-18%
// faster than 64 x 48 / 768 on grids from 192^3 to 768^2 x 128, but 8% slower
// at 512^3 with the automatic z-chunks.
template <> struct TbsDefaults<DIFF3D_F32> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 64, 1024, 0}, {3, 128, 32, 1024, 0}, {4, 64, 48, 768, 0}};
};
template <> struct TbsDefaults<DIFF3D_BF16> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 1024, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};
template <> struct TbsDefaults<DIFF3D_BF16_RNE> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 1024, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};

inline bool tbs_has(int size, const SKey& k)
{
#define DIFF3D_HAS(s, w0, h0, nth, nt) || skey_eq(k, s, w0, h0, nth, nt)
    switch (size) {
    case 8: return false DIFF3D_TBS_CFGS_8(DIFF3D_HAS);
    case 4: return false DIFF3D_TBS_CFGS_4(DIFF3D_HAS);
    case 2: return false DIFF3D_TBS_CFGS_2(DIFF3D_HAS);
    default: return false;
    }
#undef DIFF3D_HAS
}

template <int DT, int S, int W0, int H0, int NTH, int NT>
int launch_tbs_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req)
{
    static std::atomic<long long> cache{0};
    auto kernel = step_tbs<DT, S, W0, H0, NTH, NT != 0>;
    const long slots = resident_slots(kernel, NTH, cache);
    const ZPlan p = plan_rounds(edge_tiles(a.nx, W0, W0 - 2 * S), edge_tiles(a.ny, H0, H0 - 2 * S), a.nz - 2,
                                zlen_req, 2 * S, slots);
    kernel<<<p.blocks, NTH, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

// S steps T -> T2 in one pass (2 <= S <= DIFF3D_MAX_PASS_STEPS).
template <int DT>
int launch_tbs(const StepArgs<DT>& a, int nsteps, const diff3d_config& c, hipStream_t st)
{
    using Sz = typename Traits<DT>::S;
    if (nsteps < 2 || nsteps > DIFF3D_MAX_PASS_STEPS) return DIFF3D_EINVAL;
    const SKey k = skey_of(c.tbs, nsteps, TbsDefaults<DT>::key[nsteps]);
    const int zlen = szlen_of(c.tbs, nsteps);
#define DIFF3D_TRY(s, w0, h0, nth, nt) \
    if (skey_eq(k, s, w0, h0, nth, nt)) return launch_tbs_cfg<DT, s, w0, h0, nth, nt>(a, st, zlen);
    if constexpr (sizeof(Sz) == 8) {
        DIFF3D_TBS_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(Sz) == 4) {
        DIFF3D_TBS_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_TBS_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

template <int DT>
int launch_multi(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, int nsteps, uint64_t draw_step, const diff3d_config& c, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c.sr_seed, draw_step);
    return launch_tbs<DT>(a, nsteps, c, st);
}

int multi_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                   double rdx, double rdy, double rdz, int nsteps, uint64_t draw_step, const diff3d_config& c,
                   hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_multi<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, draw_step, c, st);
    case DIFF3D_F32:
        return launch_multi<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, draw_step, c, st);
    case DIFF3D_BF16:
        return launch_multi<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, draw_step, c, st);
    case DIFF3D_BF16_RNE:
        return launch_multi<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, draw_step, c,
                                             st);
    default: return DIFF3D_EDTYPE;
    }
}

template <int DT>
int launch_step(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, uint64_t draw_step, const diff3d_config& c, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, c.sr_seed, draw_step);
    if (c.kernel == DIFF3D_KERNEL_NAIVE) return launch_naive<DT>(a, st);
    return launch_zmarch<DT>(a, c, st);
}

int step_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, uint64_t draw_step, const diff3d_config& c, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_step<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    case DIFF3D_F32:
        return launch_step<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    case DIFF3D_BF16:
        return launch_step<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    case DIFF3D_BF16_RNE:
        return launch_step<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw_step, c, st);
    default: return DIFF3D_EDTYPE;
    }
}

// n steps in one pass: a single step, the two-step kernel, or the S-step
// kernel (always for n >= 3; for n = 2 when it is selected, and under AUTO
// for the BF16 forms, where it is about twice as fast per step at 512^3;
// for FP64 and FP32 the two-step kernel is faster).  `first_step` is the
// index of the pass's first step; the stored state draws with the index of
// its last.
int pass_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, int n, uint64_t first_step, const diff3d_config& c,
                  hipStream_t st)
{
    const uint64_t draw = first_step + (uint64_t)(n - 1);
    if (n == 1) return step_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw, c, st);
    const bool tbs2 = c.kernel == DIFF3D_KERNEL_TBS ||
                      (c.kernel == DIFF3D_KERNEL_AUTO && (dtype == DIFF3D_BF16 || dtype == DIFF3D_BF16_RNE));
    if (n == 2 && !tbs2) return pair_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, draw, c, st);
    return multi_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, n, draw, c, st);
}

// FP32 four-step passes lose to three-step ones on large x-y planes
// (us per step, S = 3 / S = 4: 512^2 138 / 135, 768^2 497 / 461,
// 896^2 732 / 755, 1024^2 1101 / 1410): three steps above 768^2 points.
constexpr size_t kF32FourStepMaxPlane = (size_t)768 * 768;
// FP64 on small grids, where a launch holds few workgroups and each z-chunk
// is short, is faster with three-step passes (us per step, S = 3 / S = 4:
// 64^3 3.80 / 4.14, 96^3 5.17 / 5.34, 128^3 7.35 / 7.43, 160^3 9.68 / 10.26;
// 192^3 15.1 / 14.4, 256^3 33.1 / 32.8): three steps on x-y planes of at
// most 160^2 points.
constexpr size_t kF64ThreeStepMaxPlane = (size_t)160 * 160;

int tbs_default_steps(int dtype, int nx, int ny)
{
    switch (dtype) {
    case DIFF3D_F64:
        return (size_t)nx * (size_t)ny <= kF64ThreeStepMaxPlane ? 3 : TbsDefaults<DIFF3D_F64>::S;
    case DIFF3D_F32:
        return (size_t)nx * (size_t)ny > kF32FourStepMaxPlane ? 3 : TbsDefaults<DIFF3D_F32>::S;
    case DIFF3D_BF16: return TbsDefaults<DIFF3D_BF16>::S;
    default: return TbsDefaults<DIFF3D_BF16_RNE>::S;
    }
}

// Steps per pass of diff3d_run for the selected kernel.  AUTO uses the
// S-step kernel's measured best pass length for the dtype (and, for FP32,
// the plane size).
int run_pass_steps(int dtype, int nx, int ny, const diff3d_config& c)
{
    switch (c.kernel) {
    case DIFF3D_KERNEL_NAIVE:
    case DIFF3D_KERNEL_ZMARCH: return 1;
    case DIFF3D_KERNEL_TB2: return 2;
    case DIFF3D_KERNEL_TBS: return c.pass_steps ? c.pass_steps : tbs_default_steps(dtype, nx, ny);
    default: return tbs_default_steps(dtype, nx, ny);
    }
}

// The pass lengths of the time loop (diff3d_pass_plan): passes of at most P
// steps that never cross a checkpointed state (multiples of C at or below
// klast; C = 0: none); with the default pass length each stretch between
// checkpoints is split into passes of near-equal length (14 steps with
// P = 4 as 4, 4, 3, 3 rather than 4, 4, 4, 2: short passes cost more per
// step), with a set length into passes of exactly that length.  Calls
// f(first_step, length) for each pass in order.
template <class F>
void for_each_pass(int dtype, int nx, int ny, int nt, int C, int klast, const diff3d_config& c, F&& f)
{
    const int P = run_pass_steps(dtype, nx, ny, c);
    const bool even = !(c.kernel == DIFF3D_KERNEL_TBS && c.pass_steps);
    for (int it = 0; it < nt;) {
        int end = nt;
        if (C > 0) {
            const int next = (it / C + 1) * C;   // next checkpointed step
            if (next <= klast && next < end) end = next;
        }
        const int rem = end - it;
        const int m = (rem + P - 1) / P;
        const int n = even ? (rem + m - 1) / m : min(P, rem);
        f(it, n);
        it += n;
    }
}

// ------------------------------------------------------------------ validation
// The caller's configuration must name a known kernel, a pass length the
// S-step kernel has and only instantiated tile overrides for this storage
// size; nothing is launched otherwise.
int check_forward_config(const diff3d_config& c, int dtype)
{
    if (c.kernel < DIFF3D_KERNEL_AUTO || c.kernel > DIFF3D_KERNEL_TBS) return DIFF3D_EINVAL;
    if (c.pass_steps != 0 && (c.pass_steps < 2 || c.pass_steps > DIFF3D_MAX_PASS_STEPS)) return DIFF3D_EINVAL;
    if (c.narrow != 0 && c.narrow != 1) return DIFF3D_EINVAL;
    if (c.reserved != 0) return DIFF3D_EINVAL;
    const int size = (int)elem_size(dtype);
    const diff3d_tile* zt[2] = {&c.zmarch, &c.tb2};
    for (int i = 0; i < 2; ++i) {
        if (zt[i]->steps != 0 || zt[i]->zlen < 0) return DIFF3D_EINVAL;
    }
    if (tile_set(c.zmarch) && !fwd_has(size, zkey_of(c.zmarch, kNarrow))) return DIFF3D_EINVAL;
    if (tile_set(c.tb2) && !tb2_has(size, zkey_of(c.tb2, kNarrowTb2))) return DIFF3D_EINVAL;
    if (c.tbs.zlen < 0) return DIFF3D_EINVAL;
    if (c.tbs.steps != 0 && (c.tbs.steps < 2 || c.tbs.steps > DIFF3D_MAX_PASS_STEPS)) return DIFF3D_EINVAL;
    if (tile_set(c.tbs) && (c.tbs.steps == 0 || !tbs_has(size, skey_of(c.tbs, c.tbs.steps, SKey{0, 0, 0, 0, 0}))))
        return DIFF3D_EINVAL;
    return DIFF3D_OK;
}

}  // namespace
}  // namespace diff3d
