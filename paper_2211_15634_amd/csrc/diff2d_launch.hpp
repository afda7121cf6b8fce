// Launch of the 2-D form of the step.
#pragma once

#include "host_common.hpp"
#include "step2d_kernels.hpp"

namespace diff3d {
namespace {

constexpr int kStep2dWaves = 4;                   // waves per workgroup (independent)

template <int DT>
int launch_step2d(void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt, double rdx,
                  double rdy, hipStream_t st)
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

int step2d_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, double lam, double dt,
                    double rdx, double rdy, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_step2d<DIFF3D_F64>(T2, T, Ci, nx, ny, lam, dt, rdx, rdy, st);
    case DIFF3D_F32: return launch_step2d<DIFF3D_F32>(T2, T, Ci, nx, ny, lam, dt, rdx, rdy, st);
    default: return DIFF3D_EDTYPE;
    }
}

}  // namespace
}  // namespace diff3d
