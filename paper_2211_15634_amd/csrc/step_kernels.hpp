// Forward time-step kernels of the explicit 3-D heat-diffusion scheme
// (Fig. 1, `step!`): on interior points
//   T2 = T + dt*((lam*Ci)*((d2x*cx + d2y*cy) + d2z*cz)),
//   d2x = (T[x+1] - T[x]) - (T[x] - T[x-1])  (likewise y, z),
// composed of the operators of fd_ops.hpp, evaluated in this order with no
// contraction (the library is built with -ffp-contract=off), so the FP64
// form reproduces a plain loop bit for bit.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "fd_ops.hpp"

namespace diff3d {

template <int DT>
struct StepArgs {
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    S* __restrict__ T2;
    const S* __restrict__ T;
    const S* __restrict__ Ci;
    S* __restrict__ Tmid;    // two-step kernel only: optional output of the intermediate state
    int nx, ny, nz;
    C lam, dt, cx, cy, cz;
    SrState sr;
};

template <int DT>
__device__ inline typename Traits<DT>::C stencil_point(typename Traits<DT>::C t, typename Traits<DT>::C xm,
                                                       typename Traits<DT>::C xp, typename Traits<DT>::C ym,
                                                       typename Traits<DT>::C yp, typename Traits<DT>::C zm,
                                                       typename Traits<DT>::C zp, typename Traits<DT>::C ci,
                                                       const StepArgs<DT>& a)
{
    const auto l = fd::lap3(t, xm, xp, ym, yp, zm, zp, a.cx, a.cy, a.cz);
    return fd::update(t, a.dt, a.lam * ci, l);
}

// The same update with lam*Ci already formed (identical rounding).
template <int DT>
__device__ inline typename Traits<DT>::C stencil_point_lc(typename Traits<DT>::C t, typename Traits<DT>::C xm,
                                                          typename Traits<DT>::C xp, typename Traits<DT>::C ym,
                                                          typename Traits<DT>::C yp, typename Traits<DT>::C zm,
                                                          typename Traits<DT>::C zp, typename Traits<DT>::C lamci,
                                                          const StepArgs<DT>& a)
{
    const auto l = fd::lap3(t, xm, xp, ym, yp, zm, zp, a.cx, a.cy, a.cz);
    return fd::update(t, a.dt, lamci, l);
}

// ------------------------------------------------------------------ naive
// One thread per interior point; the seven reads of T go through the
// caches.  Block 64 x 4 over (x, y); grid z strides over interior planes.
template <int DT>
__global__ __launch_bounds__(256) void step_naive(StepArgs<DT> a)
{
    using Tr = Traits<DT>;
    using C = typename Tr::C;
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63) + 1;
    const int iy = blockIdx.y * 4 + (threadIdx.x >> 6) + 1;
    if (ix > a.nx - 2 || iy > a.ny - 2) return;
    const size_t sy = (size_t)a.nx, sz = (size_t)a.nx * a.ny;
    for (int iz = blockIdx.z + 1; iz < a.nz - 1; iz += gridDim.z) {
        const size_t i = (size_t)ix + sy * iy + sz * iz;
        const C t = Tr::load(a.T[i]);
        const C r = stencil_point<DT>(t, Tr::load(a.T[i - 1]), Tr::load(a.T[i + 1]), Tr::load(a.T[i - sy]),
                                      Tr::load(a.T[i + sy]), Tr::load(a.T[i - sz]), Tr::load(a.T[i + sz]),
                                      Tr::load(a.Ci[i]), a);
        uint32_t rnd = 0;
        if constexpr (Tr::sr) rnd = sr_word(sr_block(a.sr, i >> 3), (unsigned)(i & 7));
        a.T2[i] = Tr::store(r, rnd);
    }
}

// ------------------------------------------------------------------ z-march
// A workgroup of NW wave64s owns an x-y tile of TX = 64*V by TY = R*NW
// points and marches along z over `zlen` output planes.  Lane l of wave w
// holds V consecutive x points (one load of V*sizeof(S) <= 16 bytes) of the
// R consecutive rows y0 + w*R .. y0 + w*R + R-1.
//  - z neighbours: three planes (z-1, z, z+1) of the thread's points live in
//    registers, and the plane z+2 is loaded one iteration ahead;
//  - x and y neighbours inside the thread come from registers, the others
//    from the current plane staged in LDS (double-buffered, one LDS-only
//    barrier per plane); halo rows and columns of the tile are loaded by
//    designated waves;
//  - each element of T and Ci is read from HBM about once per step (halo
//    re-reads of neighbouring tiles are L2 hits when they share an XCD);
//  - with NT, Ci is loaded and T2 stored non-temporally (neither is touched
//    again by this launch).
template <int DT, int V, int R, int NW, bool NT>
__global__ __launch_bounds__(64 * NW) void step_zmarch(StepArgs<DT> a, int ntx, int nty, int zlen)
{
    using Tr = Traits<DT>;
    using S = typename Tr::S;
    using C = typename Tr::C;
    constexpr int TX = 64 * V, TY = R * NW, LW = TX + 2;
    constexpr int WYL = 0, WYH = NW - 1, WXL = 1, WXR = 2;
    static_assert(TY <= 64, "x-halo columns are loaded by one lane per row");
    static_assert(NW >= 4, "the four halo roles need four distinct waves");
    __shared__ C lds[2][TY + 2][LW];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)ntx);
    const int rest = (int)(t / (unsigned)ntx);
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY;
    const int zb = 1 + tz * zlen;
    const int ze = min(nz - 1, zb + zlen);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xl = x0 + lane * V;
    const bool xin = xl < nx;            // nx % V == 0: a vector is wholly in or out
    const int yw = y0 + wave * R;        // first row of this thread
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;

    // Each halo role belongs to one wave (NW >= 4): wave WYL loads the row
    // below the tile, WYH the row above, WXL and WXR the columns left and
    // right of it; so a thread holds at most one halo row vector and one
    // halo column value.
    struct Halo {
        C y[V], x;
    };
    using Rows = C[R][V];
    const bool yrole = wave == WYL || wave == WYH;
    const int yh = wave == WYL ? y0 - 1 : y0 + TY;             // halo row of a y-role wave
    const int yrow = wave == WYL ? 0 : TY + 1;                 // its LDS row
    const bool xrole = (wave == WXL || wave == WXR) && lane < TY;
    const int xh = wave == WXL ? x0 - 1 : x0 + TX;              // halo column of an x-role wave
    const int xcol = wave == WXL ? 0 : TX + 1;                  // its LDS column
    const bool yload = yrole && xin && yh >= 0 && yh < ny;
    const bool xload = xrole && y0 + lane < ny && xh >= 0 && xh < nx;

    auto load_rows = [&](const S* base, int z, Rows& dst, auto nt) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (xin && yw + r < ny) {
                S raw[V];
                vload<S, V, decltype(nt)::value>(base + (size_t)xl + sy * (yw + r) + sz * z, raw);
#pragma unroll
                for (int v = 0; v < V; ++v) dst[r][v] = Tr::load(raw[v]);
            }
        }
    };
    auto load_halo = [&](int z, Halo& h) __attribute__((always_inline)) {
        if (yload) {
            S raw[V];
            vload<S, V>(a.T + (size_t)xl + sy * yh + sz * z, raw);
#pragma unroll
            for (int v = 0; v < V; ++v) h.y[v] = Tr::load(raw[v]);
        }
        if (xload) h.x = Tr::load(a.T[(size_t)xh + sy * (y0 + lane) + sz * z]);
    };
    auto stage = [&](int buf, const Rows& c, const Halo& h) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) lds[buf][1 + wave * R + r][1 + lane * V + v] = c[r][v];
        if (yrole)
#pragma unroll
            for (int v = 0; v < V; ++v) lds[buf][yrow][1 + lane * V + v] = h.y[v];
        if (xrole) lds[buf][1 + lane][xcol] = h.x;
    };
    auto compute = [&](int z, int buf, const Rows& prev, const Rows& cur, const Rows& nxt,
                       const Rows& ci) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yw + r;
            if (!(xin && y >= 1 && y <= ny - 2)) continue;
            const int row = 1 + wave * R + r;
            C out[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int col = 1 + lane * V + v;
                const C xm = v > 0 ? cur[r][v - 1] : lds[buf][row][col - 1];
                const C xp = v < V - 1 ? cur[r][v + 1] : lds[buf][row][col + 1];
                const C ym = r > 0 ? cur[r - 1][v] : lds[buf][row - 1][col];
                const C yp = r < R - 1 ? cur[r + 1][v] : lds[buf][row + 1][col];
                out[v] = stencil_point<DT>(cur[r][v], xm, xp, ym, yp, prev[r][v], nxt[r][v], ci[r][v], a);
            }
            const size_t i0 = (size_t)xl + sy * y + sz * z;
            S st[V];
            if constexpr (Tr::sr) {
                const u32x4 rb = sr_block(a.sr, i0 >> 3);
#pragma unroll
                for (int v = 0; v < V; ++v) st[v] = Tr::store(out[v], sr_word(rb, (unsigned)((i0 + v) & 7)));
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) st[v] = Tr::store(out[v], 0);
            }
            if (xl >= 1 && xl + V - 1 <= nx - 2) {
                vstore<S, V, NT>(a.T2 + i0, st);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (xl + v >= 1 && xl + v <= nx - 2) a.T2[i0 + v] = st[v];
            }
        }
    };
    using Tmp = std::false_type;
    using Str = std::integral_constant<bool, NT>;
    // One plane z: prefetch plane z+2 (into nn, hn) and Ci of z+1 (into ci2),
    // barrier, stage plane z+1 (nxt, hc) into the other LDS buffer, compute z.
    auto body = [&](int z, int buf, const Rows& prev, const Rows& cur, const Rows& nxt, Rows& nn, const Rows& ci,
                    Rows& ci2, const Halo& hc, Halo& hn) __attribute__((always_inline)) {
        const bool more = z + 1 < ze;
        if (more) {
            load_rows(a.T, z + 2, nn, Tmp{});
            load_halo(z + 2, hn);
            load_rows(a.Ci, z + 1, ci2, Str{});
        }
        lds_barrier();
        if (more) stage(buf ^ 1, nxt, hc);
        compute(z, buf, prev, cur, nxt, ci);
    };

    Rows pa, pb, pc, pd, ca, cb;
    Halo ha, hb;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < V; ++v) pa[r][v] = pb[r][v] = pc[r][v] = pd[r][v] = ca[r][v] = cb[r][v] = C(0);
#pragma unroll
    for (int v = 0; v < V; ++v) ha.y[v] = hb.y[v] = C(0);
    ha.x = hb.x = C(0);

    // prologue: planes zb-1, zb (staged in LDS buffer 0), zb+1 with its halo, Ci at zb
    load_rows(a.T, zb - 1, pa, Tmp{});
    load_rows(a.T, zb, pb, Tmp{});
    {
        Halo h0;
#pragma unroll
        for (int v = 0; v < V; ++v) h0.y[v] = C(0);
        h0.x = C(0);
        load_halo(zb, h0);
        stage(0, pb, h0);
    }
    load_rows(a.T, zb + 1, pc, Tmp{});
    load_halo(zb + 1, ha);
    load_rows(a.Ci, zb, ca, Str{});

    // plane z sits in LDS buffer (z - zb) & 1; after each plane the buffers
    // shift down by one (a single loop body keeps the kernel small enough
    // for the instruction cache)
    int buf = 0;
    for (int z = zb; z < ze; ++z) {
        body(z, buf, pa, pb, pc, pd, ca, cb, ha, hb);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                pa[r][v] = pb[r][v];
                pb[r][v] = pc[r][v];
                pc[r][v] = pd[r][v];
                ca[r][v] = cb[r][v];
            }
#pragma unroll
        for (int v = 0; v < V; ++v) ha.y[v] = hb.y[v];
        ha.x = hb.x;
        buf ^= 1;
    }
}

}  // namespace diff3d
