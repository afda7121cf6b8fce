// Reverse (adjoint) step of the explicit 3-D heat-diffusion scheme.
//
// The forward step is T_{k+1} = A T_k with A = I + diag(c) L on interior rows
// (c = dt*lam*Ci) and identity rows on the boundary, L the weighted 7-point
// second-difference operator, which is symmetric.  Hence
//   A^T lambda = lambda + L mu,   mu = c*lambda on interior points, 0 elsewhere,
// evaluated at every point (faces receive one inward term, edges and corners
// none), and dLoss/dCi accumulates dt*lam*lambda_{k+1}*(L T_k) on interior
// points.  Operation order (no contraction):
//   mu   = ((dt*lam)*Ci)*lambda
//   gCi  = gCi + ((dt*lam)*lambda)*((d2x(T)*cx + d2y(T)*cy) + d2z(T)*cz)
//   lout = lambda + ((d2x(mu)*cx + d2y(mu)*cy) + d2z(mu)*cz)
#pragma once

#include "common.hpp"
#include "fd_ops.hpp"

namespace diff3d {

template <int DT>
struct AdjArgs {
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    S* __restrict__ lout;         // lambda_k (all points)
    const S* __restrict__ lin;    // lambda_{k+1}
    const S* __restrict__ Ci;
    const S* __restrict__ Tk;     // forward state T_k
    const S* __restrict__ Tk1;    // two-step kernel only: forward state T_{k-1}
    S* __restrict__ gCi;          // accumulated in place (interior points)
    int nx, ny, nz;
    C dtlam, cx, cy, cz;
};

template <int DT>
__device__ inline typename Traits<DT>::C lap7(typename Traits<DT>::C t, typename Traits<DT>::C xm,
                                              typename Traits<DT>::C xp, typename Traits<DT>::C ym,
                                              typename Traits<DT>::C yp, typename Traits<DT>::C zm,
                                              typename Traits<DT>::C zp, const AdjArgs<DT>& a)
{
    return fd::lap3(t, xm, xp, ym, yp, zm, zp, a.cx, a.cy, a.cz);
}

// ------------------------------------------------------------------ naive
// One thread per grid point (boundary included); neighbours through caches.
template <int DT>
__global__ __launch_bounds__(256) void adj_naive(AdjArgs<DT> a)
{
    using Tr = Traits<DT>;
    using C = typename Tr::C;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ix >= nx || iy >= ny) return;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    auto mu = [&](int x, int y, int z) __attribute__((always_inline)) -> C {
        if (x < 1 || x > nx - 2 || y < 1 || y > ny - 2 || z < 1 || z > nz - 2) return C(0);
        const size_t i = (size_t)x + sy * y + sz * z;
        return a.dtlam * Tr::load(a.Ci[i]) * Tr::load(a.lin[i]);
    };
    for (int iz = blockIdx.z; iz < nz; iz += gridDim.z) {
        const size_t i = (size_t)ix + sy * iy + sz * iz;
        const C l = Tr::load(a.lin[i]);
        const C lm = lap7<DT>(mu(ix, iy, iz), mu(ix - 1, iy, iz), mu(ix + 1, iy, iz), mu(ix, iy - 1, iz),
                              mu(ix, iy + 1, iz), mu(ix, iy, iz - 1), mu(ix, iy, iz + 1), a);
        a.lout[i] = Tr::store(l + lm, 0);
        if (ix >= 1 && ix <= nx - 2 && iy >= 1 && iy <= ny - 2 && iz >= 1 && iz <= nz - 2) {
            const C lt = lap7<DT>(Tr::load(a.Tk[i]), Tr::load(a.Tk[i - 1]), Tr::load(a.Tk[i + 1]),
                                  Tr::load(a.Tk[i - sy]), Tr::load(a.Tk[i + sy]), Tr::load(a.Tk[i - sz]),
                                  Tr::load(a.Tk[i + sz]), a);
            a.gCi[i] = Tr::store(Tr::load(a.gCi[i]) + a.dtlam * l * lt, 0);
        }
    }
}

// ------------------------------------------------------------------ z-march
// Same tiling as the forward z-march (NW wave64s, tile 64*V x R*NW, march
// along z over `zlen` output planes, all planes 0..nz-1 are outputs).  Two
// fields are staged per plane in double-buffered LDS: mu (built on the fly
// from Ci and lambda) and T_k.  Registers hold mu and T_k for planes z-1..z+2
// and lambda for z..z+2; gCi of plane z is read just before it is updated.
template <int DT, int V, int R, int NW>
__global__ __launch_bounds__(64 * NW) void adj_zmarch(AdjArgs<DT> a, int ntx, int nty, int zlen)
{
    using Tr = Traits<DT>;
    using S = typename Tr::S;
    using C = typename Tr::C;
    constexpr int TX = 64 * V, TY = R * NW, LW = TX + 2;
    constexpr int WYL = 0, WYH = NW - 1, WXL = 1, WXR = 2;
    static_assert(TY <= 64, "x-halo columns are loaded by one lane per row");
    static_assert(NW >= 4, "the four halo roles need four distinct waves");
    __shared__ C lmu[2][TY + 2][LW];
    __shared__ C lt[2][TY + 2][LW];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)ntx);
    const int rest = (int)(t / (unsigned)ntx);
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY;
    const int zb = tz * zlen;
    const int ze = min(nz, zb + zlen);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xl = x0 + lane * V;
    const bool xin = xl < nx;
    const int yw = y0 + wave * R;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;

    // a point is interior if all three coordinates are
    auto inner = [&](int x, int y, int z) __attribute__((always_inline)) {
        return x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
    };
    // mu and T at V consecutive points starting at (x, y, z); lambda too.
    auto fetch = [&](int x, int y, int z, C (&m)[V], C (&tv)[V], C (&lv)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) m[v] = tv[v] = lv[v] = C(0);
        if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) return;
        const size_t i = (size_t)x + sy * y + sz * z;
        S rl[V], rc[V], rt[V];
        vload<S, V>(a.lin + i, rl);
        vload<S, V>(a.Ci + i, rc);
        vload<S, V>(a.Tk + i, rt);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            lv[v] = Tr::load(rl[v]);
            tv[v] = Tr::load(rt[v]);
            m[v] = inner(x + v, y, z) ? a.dtlam * Tr::load(rc[v]) * lv[v] : C(0);
        }
    };
    auto fetch1 = [&](int x, int y, int z, C& m, C& tv) __attribute__((always_inline)) {
        m = tv = C(0);
        if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) return;
        const size_t i = (size_t)x + sy * y + sz * z;
        tv = Tr::load(a.Tk[i]);
        m = inner(x, y, z) ? a.dtlam * Tr::load(a.Ci[i]) * Tr::load(a.lin[i]) : C(0);
    };

    // Halo roles as in the forward z-march: one wave per role, so a thread
    // holds at most one halo row (mu and T) and one halo column value.
    const bool yrole = wave == WYL || wave == WYH;
    const int yh = wave == WYL ? y0 - 1 : y0 + TY;
    const int yrow = wave == WYL ? 0 : TY + 1;
    const bool xrole = (wave == WXL || wave == WXR) && lane < TY;
    const int xh = wave == WXL ? x0 - 1 : x0 + TX;
    const int xcol = wave == WXL ? 0 : TX + 1;

    struct Plane {
        C m[R][V], tk[R][V], l[R][V];
        C ym[V], yt[V], xm, xt;
    };
    auto load_plane = [&](int z, Plane& p) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (xin && yw + r < ny) {
                fetch(xl, yw + r, z, p.m[r], p.tk[r], p.l[r]);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) p.m[r][v] = p.tk[r][v] = p.l[r][v] = C(0);
            }
        }
        C dummy[V];
        if (yrole && xin) {
            fetch(xl, yh, z, p.ym, p.yt, dummy);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) p.ym[v] = p.yt[v] = C(0);
        }
        if (xrole) {
            fetch1(xh, y0 + lane, z, p.xm, p.xt);
        } else {
            p.xm = p.xt = C(0);
        }
    };
    auto stage = [&](int buf, const Plane& p) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                lmu[buf][1 + wave * R + r][1 + lane * V + v] = p.m[r][v];
                lt[buf][1 + wave * R + r][1 + lane * V + v] = p.tk[r][v];
            }
        if (yrole)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                lmu[buf][yrow][1 + lane * V + v] = p.ym[v];
                lt[buf][yrow][1 + lane * V + v] = p.yt[v];
            }
        if (xrole) {
            lmu[buf][1 + lane][xcol] = p.xm;
            lt[buf][1 + lane][xcol] = p.xt;
        }
    };

    // One output plane z from planes z-1 (p0), z (p1, staged in LDS buffer
    // buf) and z+1 (p2); plane z+2 is prefetched into p3 and p2 is staged.
    auto body = [&](int z, int buf, const Plane& p0, const Plane& p1, const Plane& p2,
                    Plane& p3) __attribute__((always_inline)) {
        const bool more = z + 1 < ze;
        if (more) load_plane(z + 2, p3);
        lds_barrier();
        if (more) stage(buf ^ 1, p2);

#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yw + r;
            if (!(xin && y < ny)) continue;
            const int row = 1 + wave * R + r;
            const size_t i0 = (size_t)xl + sy * y + sz * z;
            const bool rowin = y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
            S gr[V];
            if (rowin) vload<S, V>(a.gCi + i0, gr);
            S lo[V], go[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int col = 1 + lane * V + v;
                const C mxm = v > 0 ? p1.m[r][v - 1] : lmu[buf][row][col - 1];
                const C mxp = v < V - 1 ? p1.m[r][v + 1] : lmu[buf][row][col + 1];
                const C mym = r > 0 ? p1.m[r - 1][v] : lmu[buf][row - 1][col];
                const C myp = r < R - 1 ? p1.m[r + 1][v] : lmu[buf][row + 1][col];
                const C lm = lap7<DT>(p1.m[r][v], mxm, mxp, mym, myp, p0.m[r][v], p2.m[r][v], a);
                lo[v] = Tr::store(p1.l[r][v] + lm, 0);
                if (rowin) {
                    const C txm = v > 0 ? p1.tk[r][v - 1] : lt[buf][row][col - 1];
                    const C txp = v < V - 1 ? p1.tk[r][v + 1] : lt[buf][row][col + 1];
                    const C tym = r > 0 ? p1.tk[r - 1][v] : lt[buf][row - 1][col];
                    const C typ = r < R - 1 ? p1.tk[r + 1][v] : lt[buf][row + 1][col];
                    const C ltk = lap7<DT>(p1.tk[r][v], txm, txp, tym, typ, p0.tk[r][v], p2.tk[r][v], a);
                    go[v] = Tr::store(Tr::load(gr[v]) + a.dtlam * p1.l[r][v] * ltk, 0);
                }
            }
            vstore<S, V>(a.lout + i0, lo);
            if (rowin) {
                if (xl >= 1 && xl + V - 1 <= nx - 2) {
                    vstore<S, V>(a.gCi + i0, go);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (xl + v >= 1 && xl + v <= nx - 2) a.gCi[i0 + v] = go[v];
                }
            }
        }
    };

    // plane z sits in LDS buffer (z - zb) & 1; the plane sets shift down by
    // one after each plane
    Plane P0, P1, P2, P3;
    load_plane(zb - 1, P0);
    load_plane(zb, P1);
    stage(0, P1);
    load_plane(zb + 1, P2);
    load_plane(-1, P3);   // zero-filled: plane -1 is outside the grid
    int buf = 0;
    for (int z = zb; z < ze; ++z) {
        body(z, buf, P0, P1, P2, P3);
        P0 = P1;
        P1 = P2;
        P2 = P3;
        buf ^= 1;
    }
}

}  // namespace diff3d
