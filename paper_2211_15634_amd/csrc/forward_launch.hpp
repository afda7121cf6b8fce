// Forward step launches: tile configuration tables and defaults per dtype,
// the single-step, two-step and S-step launchers and their dispatch.
#pragma once

#include "launch_plan.hpp"
#include "step_kernels.hpp"
#include "tb_kernels.hpp"
#include "tbs_kernels.hpp"

namespace diff3d {
namespace {

// ------------------------------------------------------------------ forward
template <int DT>
StepArgs<DT> make_step_args(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                            double rdx, double rdy, double rdz, uint64_t step_index)
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
    a.sr.k0 = (uint32_t)g_sr_seed;
    a.sr.k1 = (uint32_t)(g_sr_seed >> 32);
    a.sr.s0 = (uint32_t)step_index;
    a.sr.s1 = (uint32_t)(step_index >> 32);
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

template <int DT, int V, int R, int NW, int NT>
int launch_zmarch_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz - 2, 64 * V, R * NW, zlen_req, zdef);
    step_zmarch<DT, V, R, NW, NT != 0><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT>
int launch_zmarch(const StepArgs<DT>& a, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    ZKey k = FwdDefaults<DT>::wide;
    env_key("DIFF3D_ZCFG", k);
    if (env_int("DIFF3D_NARROW", 0) || !vec_ok<S>(a.nx, k.V, a.T, a.T2, a.Ci)) k = kNarrow;
    const int zlen = env_int("DIFF3D_ZLEN", 0);
    const int zdef = FwdDefaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw, nt) \
    if (key_eq(k, v, r, nw, nt)) return launch_zmarch_cfg<DT, v, r, nw, nt>(a, st, zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_FWD_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(S) == 4) {
        DIFF3D_FWD_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_FWD_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;   // configuration not instantiated (tuning override only)
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

template <int DT, int V, int R, int NW, int NT, bool MID>
int launch_tb2_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz - 2, 64 * V, R * NW, zlen_req, zdef);
    step_tb2<DT, V, R, NW, NT != 0, MID><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT, bool MID>
int launch_tb2(const StepArgs<DT>& a, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    ZKey k = Tb2Defaults<DT>::wide;
    env_key("DIFF3D_TCFG", k);
    if (env_int("DIFF3D_NARROW", 0) || !vec_ok<S>(a.nx, k.V, a.T, a.T2, a.Ci)) k = kNarrowTb2;
    const int zlen = env_int("DIFF3D_TZLEN", 0);
    const int zdef = Tb2Defaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw, nt) \
    if (key_eq(k, v, r, nw, nt)) return launch_tb2_cfg<DT, v, r, nw, nt, MID>(a, st, zlen, zdef);
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

// Two steps T -> T2 (T^{k+2}); SR step indices step_index and step_index+1.
template <int DT>
int launch_pair(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index);
    return launch_tb2<DT, false>(a, st);
}

// Two steps T -> Tmid (T^{k+1}) and T2 (T^{k+2}), interior points of both.
template <int DT>
int launch_pair_mid(void* T2, void* Tmid, const void* T, const void* Ci, int nx, int ny, int nz, double lam,
                    double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, 0);
    a.Tmid = static_cast<typename Traits<DT>::S*>(Tmid);
    return launch_tb2<DT, true>(a, st);
}

int pair_mid_dispatch(int dtype, void* T2, void* Tmid, const void* T, const void* Ci, int nx, int ny, int nz,
                      double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_pair_mid<DIFF3D_F64>(T2, Tmid, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    case DIFF3D_F32: return launch_pair_mid<DIFF3D_F32>(T2, Tmid, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    default: return DIFF3D_EDTYPE;
    }
}

int pair_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_pair<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_F32: return launch_pair<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16: return launch_pair<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16_RNE:
        return launch_pair<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    default: return DIFF3D_EDTYPE;
    }
}

#define DIFF3D_TBS_CFGS_8(X) X(2, 64, 16, 512, 1) X(2, 64, 32, 512, 0) X(3, 64, 32, 512, 0) X(3, 64, 32, 1024, 0) \
    X(4, 64, 32, 512, 0) X(4, 64, 32, 1024, 0)
#define DIFF3D_TBS_CFGS_4(X) X(2, 64, 32, 512, 1) X(2, 64, 64, 1024, 0) X(3, 64, 32, 512, 0) X(3, 128, 32, 1024, 0) \
    X(4, 64, 32, 512, 0) X(4, 64, 48, 768, 0)
#define DIFF3D_TBS_CFGS_2(X) X(2, 64, 32, 512, 1) X(2, 64, 32, 1024, 0) X(3, 64, 32, 1024, 0) X(4, 64, 32, 1024, 0)

template <int DT>
struct TbsDefaults;
template <> struct TbsDefaults<DIFF3D_F64> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 512, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};
template <> struct TbsDefaults<DIFF3D_F32> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 64, 1024, 0}, {3, 128, 32, 1024, 0}, {4, 64, 48, 768, 0}};
};
template <> struct TbsDefaults<DIFF3D_BF16> {
    static constexpr int S = 3;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 1024, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};
template <> struct TbsDefaults<DIFF3D_BF16_RNE> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 1024, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};

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
int launch_tbs(const StepArgs<DT>& a, int nsteps, hipStream_t st)
{
    using Sz = typename Traits<DT>::S;
    if (nsteps < 2 || nsteps > DIFF3D_MAX_PASS_STEPS) return DIFF3D_EINVAL;
    SKey k = TbsDefaults<DT>::key[nsteps];
    env_skey("DIFF3D_SCFG", k);
    const int zlen = env_int("DIFF3D_SZLEN", 0);
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
                 double rdy, double rdz, int nsteps, uint64_t step_index, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index);
    return launch_tbs<DT>(a, nsteps, st);
}

int multi_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                   double rdx, double rdy, double rdz, int nsteps, uint64_t step_index, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_multi<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    case DIFF3D_F32:
        return launch_multi<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    case DIFF3D_BF16:
        return launch_multi<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    case DIFF3D_BF16_RNE:
        return launch_multi<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    default: return DIFF3D_EDTYPE;
    }
}

template <int DT>
int launch_step(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index);
    if (g_kernel == DIFF3D_KERNEL_NAIVE) return launch_naive<DT>(a, st);
    return launch_zmarch<DT>(a, st);
}

int step_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_step<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_F32: return launch_step<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16: return launch_step<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16_RNE:
        return launch_step<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    default: return DIFF3D_EDTYPE;
    }
}

// n steps in one pass: a single step, the two-step kernel, or the S-step
// kernel (always for n >= 3; for n = 2 when it is selected, and under AUTO
// for the BF16 forms, where it is about twice as fast per step at 512^3;
// for FP64 and FP32 the two-step kernel is faster).
int pass_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, int n, uint64_t step_index, hipStream_t st)
{
    if (n == 1) return step_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    const bool tbs2 = g_kernel == DIFF3D_KERNEL_TBS ||
                      (g_kernel == DIFF3D_KERNEL_AUTO && (dtype == DIFF3D_BF16 || dtype == DIFF3D_BF16_RNE));
    if (n == 2 && !tbs2)
        return pair_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    return multi_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, n, step_index, st);
}

// FP32 four-step passes lose to three-step ones on large x-y planes
// (us per step, S = 3 / S = 4: 512^2 138 / 135, 768^2 497 / 461,
// 896^2 732 / 755, 1024^2 1101 / 1410): three steps above 768^2 points.
constexpr size_t kF32FourStepMaxPlane = (size_t)768 * 768;

int tbs_default_steps(int dtype, int nx, int ny)
{
    switch (dtype) {
    case DIFF3D_F64: return TbsDefaults<DIFF3D_F64>::S;
    case DIFF3D_F32:
        return (size_t)nx * (size_t)ny > kF32FourStepMaxPlane ? 3 : TbsDefaults<DIFF3D_F32>::S;
    case DIFF3D_BF16: return TbsDefaults<DIFF3D_BF16>::S;
    default: return TbsDefaults<DIFF3D_BF16_RNE>::S;
    }
}

// Steps per pass of diff3d_run for the selected kernel.  AUTO uses the
// S-step kernel's measured best pass length: 4 for FP64 and FP32 (3 for
// FP32 on planes above 768^2 points), 4 for
// BF16 with round-to-nearest (two workgroups per CU: 103 us per step against
// 207 for single steps at 512^3), 3 for BF16 with stochastic rounding (bound
// by the Philox draws: 253 against 300 us).
int run_pass_steps(int dtype, int nx, int ny)
{
    switch (g_kernel) {
    case DIFF3D_KERNEL_NAIVE:
    case DIFF3D_KERNEL_ZMARCH: return 1;
    case DIFF3D_KERNEL_TB2: return 2;
    case DIFF3D_KERNEL_TBS: return g_pass_steps ? g_pass_steps : tbs_default_steps(dtype, nx, ny);
    default: return tbs_default_steps(dtype, nx, ny);
    }
}

}  // namespace
}  // namespace diff3d
