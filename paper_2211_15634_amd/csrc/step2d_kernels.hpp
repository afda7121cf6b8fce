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
    SrState sr;                                   // stochastic rounding of the stored state (BF16)
};

// The 16 random bits that round point i = x + nx*y of the stored state
// (stochastically rounded BF16 only; the same counter layout as the 3-D
// steps, with the 2-D linear index).
template <int DT>
__device__ inline uint32_t rounding2d(const Step2dArgs<DT>& a, size_t i)
{
    if constexpr (Traits<DT>::sr)
        return sr_word(sr_block(a.sr, i >> 3), (unsigned)(i & 7));
    else
        return 0u;
}

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
        if (interior_x) {
            const size_t i = (size_t)x + sy * (size_t)y;
            __builtin_nontemporal_store(Tr::store(w, rounding2d(a, i)), a.T2 + i);
        }
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

// S steps per pass over HBM (S = 2 .. kMaxSteps2d).  A wave owns a region
// of 64 consecutive x points (origin strip * (64 - 2S): regions start at the
// grid's edge and the last one reaches its far edge) and marches along y
// over the output rows of its chunk.  Level s (s = 0 .. S, level 0 = T^k) is
// computed on the region's lanes s .. 63-s (a side on the grid's boundary
// does not shrink: the boundary values are the same at every level), at row
// y + 1 - s in iteration y, from level s-1 at rows y - s .. y + 2 - s: the
// two older rows in registers, the newest just computed; x neighbours are
// the adjacent lanes' values.  Every lane computes every level and keeps
// the result only at interior grid points (elsewhere the level keeps the
// fixed boundary value); values of a level outside its lanes are read by no
// needed point.  Level S is stored on lanes S .. 63-S (from x = 1 and up to
// x = nx-2 at the grid's edges) and the chunk's rows.  Intermediate levels
// stay in the compute type (FP64, or FP32 for FP32 and BF16), so a pass is
// bit-identical to S single steps; BF16 rounds once per pass.  No LDS and
// no barrier.
constexpr int kMaxSteps2d = 8;

template <int DT, int S, int WPB>
__global__ __launch_bounds__(64 * WPB) void step2d_ymarch_s(Step2dArgs<DT> a, int nstrips, int nchunks, int ylen)
{
    using Tr = Traits<DT>;
    using C = typename Tr::C;
    static_assert(S >= 2 && S <= kMaxSteps2d, "two to eight steps per pass");
    constexpr int TX = 64 - 2 * S;
    const int lane = (int)(threadIdx.x & 63);
    const int wid = (int)blockIdx.x * WPB + (int)(threadIdx.x >> 6);
    if (wid >= nstrips * nchunks) return;         // whole waves
    const int nx = a.nx, ny = a.ny;
    const int strip = wid % nstrips, chunk = wid / nstrips;
    const int ys = 1 + chunk * ylen, ye = min(ny - 1, ys + ylen);   // output rows ys .. ye-1
    if (ys >= ye) return;                         // whole waves
    const int xr = strip * TX;
    const int x = xr + lane;
    const int xc = min(x, nx - 1);
    const bool ex0 = xr == 0, ex1 = xr + 64 >= nx;
    const bool interior_x = x >= 1 && x <= nx - 2;
    const bool out_lane = interior_x && (lane >= S || ex0) && (lane <= 63 - S || ex1);
    const size_t sy = (size_t)nx;
    auto row = [&](int y) __attribute__((always_inline)) { return (size_t)min(max(y, 0), ny - 1); };
    auto ld = [&](int y) __attribute__((always_inline)) -> C { return Tr::load(a.T[(size_t)xc + sy * row(y)]); };
    auto ldc = [&](int y) __attribute__((always_inline)) -> C {
        return Tr::load(__builtin_nontemporal_load(a.Ci + (size_t)xc + sy * row(y)));
    };

    const int y0 = ys - S + 1;                    // level 1 reaches its first needed row
    const int ylast = ye + S - 2;                 // level S reaches the chunk's last row
    // level s-1's two rows below its newest one (lm: row - 2, lc: row - 1)
    C lm[S], lc[S];
    // lam*Ci at rows y, y-1, .., y-S+1 (level s uses cr[s-1]); loads in flight
    C cr[S];
#pragma unroll
    for (int s = 1; s < S; ++s) lm[s] = lc[s] = C(0);
    lm[0] = ld(y0 - 1);
    lc[0] = ld(y0);
    C tA = ld(y0 + 1), tB = ld(y0 + 2);           // level 0 at rows y+1 and y+2
#pragma unroll
    for (int j = 0; j < S; ++j) cr[j] = a.lam * ldc(y0 - j);
    C cA = ldc(y0 + 1);                           // Ci at row y+1
    for (int y = y0; y <= ylast; ++y) {
        const C tC = ld(y + 3);
        const C cB = ldc(y + 2);
        C fresh = tA;                             // level s-1 at row y + 2 - s
#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int r = y + 1 - s;
            const C ce = lc[s - 1];
            const C xm = lane_shift<C, false>(ce);
            const C xp = lane_shift<C, true>(ce);
            const C l = fd::lap2(ce, xm, xp, lm[s - 1], fresh, a.cx, a.cy);
            const C w = fd::update(ce, a.dt, cr[s - 1], l);
            lm[s - 1] = ce;
            lc[s - 1] = fresh;
            if (s < S) {
                fresh = (r >= 1 && r <= ny - 2 && interior_x) ? w : ce;
            } else if (r >= ys && r < ye && out_lane) {
                const size_t i = (size_t)x + sy * (size_t)r;
                __builtin_nontemporal_store(Tr::store(w, rounding2d(a, i)), a.T2 + i);
            }
        }
#pragma unroll
        for (int j = S - 1; j >= 1; --j) cr[j] = cr[j - 1];
        cr[0] = a.lam * cA;
        cA = cB;
        tA = tB;
        tB = tC;
    }
}

}  // namespace diff3d
