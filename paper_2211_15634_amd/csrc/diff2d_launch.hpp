// Launch of the 2-D form of the step.
#pragma once

#include "host_common.hpp"
#include "step2d_kernels.hpp"

namespace diff3d {
namespace {

constexpr int kStep2dWaves = 4;                   // waves per workgroup (independent)

// Kernel arguments; the stored state draws its rounding bits (stochastically
// rounded BF16) with key sr_seed and step index draw_step.
template <int DT>
Step2dArgs<DT> make_step2d_args(void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt,
                                double rdx, double rdy, uint64_t sr_seed, uint64_t draw_step)
{
    using Sz = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    Step2dArgs<DT> a;
    a.T2 = static_cast<Sz*>(T2);
    a.T = static_cast<const Sz*>(T);
    a.Ci = static_cast<const Sz*>(Ci);
    a.nx = nx;
    a.ny = ny;
    a.lam = (C)lam;
    a.dt = (C)dt;
    a.cx = (C)(rdx * rdx);
    a.cy = (C)(rdy * rdy);
    a.sr.k0 = (uint32_t)sr_seed;
    a.sr.k1 = (uint32_t)(sr_seed >> 32);
    a.sr.s0 = (uint32_t)draw_step;
    a.sr.s1 = (uint32_t)(draw_step >> 32);
    return a;
}

template <int DT>
int launch_step2d(const Step2dArgs<DT>& a, hipStream_t st)
{
    const int nx = a.nx, ny = a.ny;
    // y-chunks for about 128 waves per CU (several rounds of resident waves),
    // each at least 16 rows long.  Measured at 8192^2, us per step for a target
    // of 16 / 32 / 64 / 128 waves per CU: FP64 299 / 346 / 346 / 285, FP32
    // 210 / 154 / 211 / 159 (non-monotonic: the chunk starts' spacing in
    // memory matters as much as the count).
    const int nstrips = (nx + 63) / 64;
    const int rows = ny - 2;
    const int want = (256 * 128 + nstrips - 1) / nstrips;
    const int nchunks = max(1, min(want, (rows + 15) / 16));
    // an odd chunk length keeps chunk starts from lying a power of two rows
    // apart (FP64 at 4096^2: 79 against 101 us per step; FP32 at 8192^2: 148
    // against 159); chunks past the last row exit at once
    int ylen = (rows + nchunks - 1) / nchunks;
    if (ylen > 1) ylen |= 1;
    const long waves = (long)nstrips * nchunks;
    const unsigned blocks = (unsigned)((waves + kStep2dWaves - 1) / kStep2dWaves);
    step2d_ymarch<DT, kStep2dWaves><<<blocks, 64 * kStep2dWaves, 0, st>>>(a, nstrips, nchunks, ylen);
    return hip_status();
}

// S steps in one pass (2 <= S <= kMaxSteps2d): regions of 64 points every
// 64 - 2S along x, chunks of rows along y long enough that the 2S - 2 rows
// of warm-up per chunk stay a small part of a wave's work.  The chunk count
// aims at 64 waves per CU (us per step at S = 7 FP64 / 8 FP32, targets of
// 16 / 32 / 64 / 128 waves per CU: 8192^2 81.0 / 73.9 / 75.9 / 75.4 and
// 47.6 / 43.7 / 42.9 / 42.1; 16384^2 329.7 / 290.6 / 274.8 / 276.0 and
// 180.9 / 163.9 / 151.7 / 152.0).
constexpr int kStep2dMinRowsPerWarmup = 8;        // chunk rows >= 8 x (2S - 2)
constexpr int kStep2dWavesPerCU = 64;             // waves per CU the chunk count aims at

// Steps per pass of diff2d_run (us per step at 8192^2 for S = 1 / 4 / 6 / 7 /
// 8: FP64 282 / 112 / 77 / 74 / 78, FP32 146 / 62 / 44 / 43 / 45, BF16 with
// stochastic rounding 191 / 75 / 62 / 61 / 60, BF16 with round-to-nearest
// 105 / 45 / 40 / 40 / 42; at 16384^2 FP32 S = 8 beats S = 7 by 6%).  The
// BF16 forms share FP32's arithmetic and, at these pass lengths, its speed.
inline int run2d_pass_steps(int dtype)
{
    return dtype == DIFF3D_F64 ? 7 : 8;
}

template <int DT, int S>
int launch_step2d_s(const Step2dArgs<DT>& a, hipStream_t st)
{
    const int nx = a.nx, ny = a.ny;
    constexpr int TX = 64 - 2 * S;
    const int nstrips = nx <= 64 ? 1 : (nx - 64 + TX - 1) / TX + 1;
    const int rows = ny - 2;
    const int want = (256 * kStep2dWavesPerCU + nstrips - 1) / nstrips;
    const int minlen = kStep2dMinRowsPerWarmup * (2 * S - 2);
    const int nchunks = max(1, min(want, (rows + minlen - 1) / minlen));
    int ylen = (rows + nchunks - 1) / nchunks;
    if (ylen > 1) ylen |= 1;                      // chunk starts not a power of two rows apart
    const long waves = (long)nstrips * nchunks;
    const unsigned blocks = (unsigned)((waves + kStep2dWaves - 1) / kStep2dWaves);
    step2d_ymarch_s<DT, S, kStep2dWaves><<<blocks, 64 * kStep2dWaves, 0, st>>>(a, nstrips, nchunks, ylen);
    return hip_status();
}

template <int DT>
int launch_step2d_n(int n, void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt,
                    double rdx, double rdy, uint64_t sr_seed, uint64_t draw_step, hipStream_t st)
{
    const Step2dArgs<DT> a = make_step2d_args<DT>(T2, T, Ci, nx, ny, lam, dt, rdx, rdy, sr_seed, draw_step);
    switch (n) {
    case 1: return launch_step2d<DT>(a, st);
    case 2: return launch_step2d_s<DT, 2>(a, st);
    case 3: return launch_step2d_s<DT, 3>(a, st);
    case 4: return launch_step2d_s<DT, 4>(a, st);
    case 5: return launch_step2d_s<DT, 5>(a, st);
    case 6: return launch_step2d_s<DT, 6>(a, st);
    case 7: return launch_step2d_s<DT, 7>(a, st);
    case 8: return launch_step2d_s<DT, 8>(a, st);
    default: return DIFF3D_EINVAL;
    }
}

// n steps (1 <= n <= kMaxSteps2d) in one pass of the 2-D form; the stored
// state draws with step index draw_step (stochastically rounded BF16).
int step2dn_dispatch(int dtype, int n, void* T2, const void* T, const void* Ci, int nx, int ny, double lam,
                     double dt, double rdx, double rdy, uint64_t sr_seed, uint64_t draw_step, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_step2d_n<DIFF3D_F64>(n, T2, T, Ci, nx, ny, lam, dt, rdx, rdy, sr_seed, draw_step, st);
    case DIFF3D_F32:
        return launch_step2d_n<DIFF3D_F32>(n, T2, T, Ci, nx, ny, lam, dt, rdx, rdy, sr_seed, draw_step, st);
    case DIFF3D_BF16:
        return launch_step2d_n<DIFF3D_BF16>(n, T2, T, Ci, nx, ny, lam, dt, rdx, rdy, sr_seed, draw_step, st);
    case DIFF3D_BF16_RNE:
        return launch_step2d_n<DIFF3D_BF16_RNE>(n, T2, T, Ci, nx, ny, lam, dt, rdx, rdy, sr_seed, draw_step, st);
    default: return DIFF3D_EDTYPE;
    }
}

}  // namespace
}  // namespace diff3d
