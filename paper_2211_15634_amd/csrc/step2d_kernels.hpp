// The 2-D form of the step: the Fig. 1 expression without the z term,
//   T2 = T + dt*((lam*Ci)*(d2x(T)*cx + d2y(T)*cy))   on interior points,
// on an nx x ny grid (index x + nx*y), boundary values never written.
#pragma once

#include "common.hpp"
#include "fd_ops.hpp"

namespace diff3d {

template <int DT>
struct Step2dArgs {
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    S* __restrict__ T2;
    const S* __restrict__ T;
    const S* __restrict__ Ci;
    int nx, ny;
    C lam, dt, cx, cy;
};

// One wave64 owns a strip of 64 consecutive x points (lane l: x = 64*strip
// + l) and marches along y over `ylen` output rows.  Rows y-1, y, y+1 of its
// point live in registers and rows y+2, y+3 are in flight, so the y
// neighbours never leave the thread; the x neighbours are the adjacent
// lanes' values (cross-lane moves), the strip's two outer neighbours one
// extra load per row (lanes 1..63 all load the same address, lane 0 the
// point left of the strip).  Ci is read and T2 written non-temporally
// (neither is touched again by the launch).  Waves are independent: no LDS,
// no barrier.  Loads are clamped into the grid; values of points outside it
// are never used by an interior update.  Measured at 8192^2: one point per
// lane with 8-byte accesses beats 16-byte vector loads and stores (352
// against 631 and 384 us per FP64 step), and the non-temporal hints gain 3%
// (FP64) and 7% (FP32).
template <int DT, int WPB>
__global__ __launch_bounds__(64 * WPB) void step2d_ymarch(Step2dArgs<DT> a, int nstrips, int nchunks, int ylen)
{
    using Tr = Traits<DT>;
    using S_ = typename Tr::S;
    using C = typename Tr::C;
    const int lane = (int)(threadIdx.x & 63);
    const int wid = (int)blockIdx.x * WPB + (int)(threadIdx.x >> 6);
    if (wid >= nstrips * nchunks) return;         // whole waves
    const int nx = a.nx, ny = a.ny;
    const int strip = wid % nstrips, chunk = wid / nstrips;
    const int ys = 1 + chunk * ylen, ye = min(ny - 1, ys + ylen);   // output rows ys .. ye-1
    if (ys >= ye) return;                         // whole waves
    const int x = strip * 64 + lane;
    const int xc = min(x, nx - 1);
    const int xh = lane == 0 ? max(x - 1, 0) : min(strip * 64 + 64, nx - 1);
    const bool interior_x = x >= 1 && x <= nx - 2;
    const size_t sy = (size_t)nx;
    auto ld = [&](const S_* p, int y, int xx) __attribute__((always_inline)) -> C {
        return Tr::load(p[(size_t)xx + sy * (size_t)y]);
    };
    auto ldnt = [&](const S_* p, int y, int xx) __attribute__((always_inline)) -> C {
        return Tr::load(__builtin_nontemporal_load(p + (size_t)xx + sy * (size_t)y));
    };
    // rows y-1 .. y+1 in use, rows y+2 and y+3 (and Ci, halo of y+1, y+2) in flight
    C rm = ld(a.T, ys - 1, xc), rc = ld(a.T, ys, xc), rp = ld(a.T, ys + 1, xc);
    C r2 = ld(a.T, min(ys + 2, ny - 1), xc);
    C hc = ld(a.T, ys, xh), h1 = ld(a.T, ys + 1, xh);
    C cc = ldnt(a.Ci, ys, xc), c1 = ldnt(a.Ci, ys + 1, xc);
    for (int y = ys; y < ye; ++y) {
        const C r3 = ld(a.T, min(y + 3, ny - 1), xc);
        const C h2 = ld(a.T, min(y + 2, ny - 1), xh);
        const C c2 = ldnt(a.Ci, min(y + 2, ny - 1), xc);
        C xm = __shfl_up(rc, 1);
        C xp = __shfl_down(rc, 1);
        if (lane == 0) xm = hc;
        if (lane == 63) xp = hc;
        const C t = rc;
        const C l = fd::lap2(t, xm, xp, rm, rp, a.cx, a.cy);
        const C w = fd::update(t, a.dt, a.lam * cc, l);
        if (interior_x) __builtin_nontemporal_store(Tr::store(w, 0), a.T2 + (size_t)x + sy * (size_t)y);
        rm = rc;
        rc = rp;
        rp = r2;
        r2 = r3;
        hc = h1;
        h1 = h2;
        cc = c1;
        c1 = c2;
    }
}

}  // namespace diff3d
