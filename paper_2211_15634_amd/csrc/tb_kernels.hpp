// Two time steps per pass over HBM (temporal blocking) for the explicit 3-D
// heat-diffusion step.  T^{k+2} is computed from T^k with the same
// operations, in the same order, as two single steps; the intermediate
// T^{k+1} stays in the compute type on chip, so FP64 and FP32 results are
// bit-identical to two launches of the single-step kernel and BF16 rounds
// once per pass (the stored state draws with the step index in a.sr).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "step_kernels.hpp"

namespace diff3d {

// Tiling as in step_zmarch: NW wave64s, tile TX = 64*V by TY = R*NW in x-y,
// marching along z.  Per plane p the workgroup
//   1. computes T^{k+1}(p) on the tile and on a one-point ring around it
//      (without corners), from T^k(p) staged in LDS with a two-point ring
//      and T^k(p-1), T^k(p+1) in registers;
//   2. computes T^{k+2}(p-1) on the tile from T^{k+1}(p-2 .. p) (registers
//      for z, LDS for x and y) and stores it.
// The ring rows are owned by waves WYL (below the tile) and WYH (above), the
// ring columns by waves WXL (left) and WXR (right); those waves also load the
// second ring of T^k and the four corners of the first.  One LDS-only
// barrier per plane; loads run one plane ahead.
// With MID, the intermediate state of the workgroup's own planes is also
// stored (interior points) into a.Tmid: the reverse sweep recomputes every
// state of a checkpoint segment this way at two field passes per step.
template <int DT, int V, int R, int NW, bool NT, bool MID>
__global__ __launch_bounds__(64 * NW) void step_tb2(StepArgs<DT> a, int ntx, int nty, int zlen)
{
    using Tr = Traits<DT>;
    using S = typename Tr::S;
    using C = typename Tr::C;
    constexpr int TX = 64 * V, TY = R * NW;
    constexpr int WYL = 0, WYH = NW - 1, WXL = 1, WXR = 2;
    static_assert(NW >= 4, "the four ring roles need four distinct waves");
    static_assert(TY + 2 <= 64, "ring columns are held one point per lane");
    static_assert(!MID || DT == DIFF3D_F64 || DT == DIFF3D_F32, "the intermediate is stored exactly only for FP64/FP32");
    __shared__ C lA[2][TY + 4][TX + 4];   // T^k plane, origin (y0 - 2, x0 - 2)
    __shared__ C lB[2][TY + 2][TX + 2];   // T^{k+1} plane, origin (y0 - 1, x0 - 1)

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)ntx);
    const int rest = (int)(t / (unsigned)ntx);
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY;
    const int zb = 1 + tz * zlen;                 // output planes zb .. ze-1
    const int ze = min(nz - 1, zb + zlen);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xl = x0 + lane * V;
    const bool xin = xl < nx;
    const int yw = y0 + wave * R;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;

    // ring roles
    const bool yrole = wave == WYL || wave == WYH;
    const int yr1 = wave == WYL ? y0 - 1 : y0 + TY;        // first-ring row
    const int yr2 = wave == WYL ? y0 - 2 : y0 + TY + 1;    // second-ring row
    const int ay1 = wave == WYL ? 1 : TY + 2;              // their rows in lA
    const int ay2 = wave == WYL ? 0 : TY + 3;
    const int by1 = wave == WYL ? 0 : TY + 1;              // first-ring row in lB
    const bool xrole = (wave == WXL || wave == WXR) && lane < TY + 2;
    const int xc1 = wave == WXL ? x0 - 1 : x0 + TX;        // first-ring column
    const int xc2 = wave == WXL ? x0 - 2 : x0 + TX + 1;    // second-ring column
    const int ax1 = wave == WXL ? 1 : TX + 2;
    const int ax2 = wave == WXL ? 0 : TX + 3;
    const int bx1 = wave == WXL ? 0 : TX + 1;
    const int yx = y0 - 1 + lane;                          // row of an x-role lane
    const bool xmid = lane >= 1 && lane <= TY;             // x-role lanes on ring points (not corners)

    const bool yload1 = yrole && xin && yr1 >= 0 && yr1 < ny;
    const bool yload2 = yrole && xin && yr2 >= 0 && yr2 < ny;
    const bool xload1 = xrole && xc1 >= 0 && xc1 < nx && yx >= 0 && yx < ny;
    const bool xload2 = xrole && xmid && xc2 >= 0 && xc2 < nx && yx >= 0 && yx < ny;

    using Rows = C[R][V];
    using Vec = C[V];
    auto interior = [&](int x, int y, int z) __attribute__((always_inline)) {
        return x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
    };
    auto vld = [&](const S* base, int x, int y, int z, Vec& dst, bool ok, auto nt) __attribute__((always_inline)) {
        if (ok && z >= 0 && z < nz) {
            S raw[V];
            vload<S, V, decltype(nt)::value>(base + (size_t)x + sy * y + sz * z, raw);
#pragma unroll
            for (int v = 0; v < V; ++v) dst[v] = Tr::load(raw[v]);
        }
    };
    auto sld = [&](const S* base, int x, int y, int z, C& dst, bool ok) __attribute__((always_inline)) {
        if (ok && z >= 0 && z < nz) dst = Tr::load(base[(size_t)x + sy * y + sz * z]);
    };
    using Tmp = std::false_type;
    using Str = std::integral_constant<bool, NT>;

    // plane-indexed state; suffix 0..3 = planes p-1 .. p+2 of T^k
    Rows t0, t1, t2, t3;          // owned T^k
    Rows u0, u1, u2;              // owned T^{k+1} at p-2, p-1, p
    Rows cm, c0, c1;              // owned Ci at p-1, p, p+1
    Vec y0v, y1v, y2v, y3v;       // first-ring row T^k (y roles)
    Vec ycv0, ycv1;               // first-ring row Ci at p, p+1
    Vec l2a, l2b;                 // second-ring row T^k at p+1, p+2
    C x0s = C(0), x1s = C(0), x2s = C(0), x3s = C(0);   // first-ring column T^k (x roles)
    C xcs0 = C(0), xcs1 = C(0);   // first-ring column Ci at p, p+1
    C l2xa = C(0), l2xb = C(0);   // second-ring column T^k at p+1, p+2
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < V; ++v)
            t0[r][v] = t1[r][v] = t2[r][v] = t3[r][v] = u0[r][v] = u1[r][v] = u2[r][v] = cm[r][v] = c0[r][v] =
                c1[r][v] = C(0);
#pragma unroll
    for (int v = 0; v < V; ++v) y0v[v] = y1v[v] = y2v[v] = y3v[v] = ycv0[v] = ycv1[v] = l2a[v] = l2b[v] = C(0);

    auto load_owned = [&](const S* base, int z, Rows& dst, auto nt) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) vld(base, xl, yw + r, z, dst[r], xin && yw + r < ny, nt);
    };
    // T^k of plane z: owned points, first ring (rows and columns with corners)
    auto load_plane = [&](int z, Rows& own, Vec& yv, C& xs) __attribute__((always_inline)) {
        load_owned(a.T, z, own, Tmp{});
        vld(a.T, xl, yr1, z, yv, yload1, Tmp{});
        sld(a.T, xc1, yx, z, xs, xload1);
    };
    auto load_ring2 = [&](int z, Vec& yv, C& xs) __attribute__((always_inline)) {
        vld(a.T, xl, yr2, z, yv, yload2, Tmp{});
        sld(a.T, xc2, yx, z, xs, xload2);
    };
    auto load_ci = [&](int z, Rows& own, Vec& yv, C& xs) __attribute__((always_inline)) {
        load_owned(a.Ci, z, own, Str{});
        vld(a.Ci, xl, yr1, z, yv, yload1, Str{});
        sld(a.Ci, xc1, yx, z, xs, xload1 && xmid);
    };
    auto stage_A = [&](int buf, const Rows& own, const Vec& yv, const Vec& y2, C xs,
                       C x2) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) lA[buf][2 + wave * R + r][2 + lane * V + v] = own[r][v];
        if (yrole) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                lA[buf][ay1][2 + lane * V + v] = yv[v];
                lA[buf][ay2][2 + lane * V + v] = y2[v];
            }
        }
        if (xrole) {
            lA[buf][1 + lane][ax1] = xs;
            if (xmid) lA[buf][1 + lane][ax2] = x2;
        }
    };

    const int p0 = zb - 1;
    // prologue: T^k planes p0-1 .. p0+1, plane p0 staged with both rings,
    // the second ring of p0+1, Ci at p0
    {
        load_plane(p0 - 1, t0, y0v, x0s);
        load_plane(p0, t1, y1v, x1s);
        Vec r2;
        C r2x = C(0);
#pragma unroll
        for (int v = 0; v < V; ++v) r2[v] = C(0);
        load_ring2(p0, r2, r2x);
        stage_A(0, t1, y1v, r2, x1s, r2x);
        load_plane(p0 + 1, t2, y2v, x2s);
        load_ring2(p0 + 1, l2a, l2xa);
        load_ci(p0, c0, ycv0, xcs0);
    }

    int bA = 0, bB = 0;
    for (int p = p0; p <= ze; ++p) {
        // 1. loads one plane ahead
        if (p + 1 <= ze) {
            load_plane(p + 2, t3, y3v, x3s);
            if (p + 2 <= ze) load_ring2(p + 2, l2b, l2xb);
            load_ci(p + 1, c1, ycv1, xcs1);
        }
        lds_barrier();
        // 2. stage T^k(p+1) for the next plane
        if (p + 1 <= ze) stage_A(bA ^ 1, t2, y2v, l2a, x2s, l2xa);

        // 3. T^{k+1}(p) on the tile and the first ring
        const bool zin = p >= 1 && p <= nz - 2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yw + r;
            const int row = 2 + wave * R + r;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int x = xl + v, col = 2 + lane * V + v;
                C u = t1[r][v];
                if (zin && xin && interior(x, y, p)) {
                    const C xm = v > 0 ? t1[r][v - 1] : lA[bA][row][col - 1];
                    const C xp = v < V - 1 ? t1[r][v + 1] : lA[bA][row][col + 1];
                    const C ym = r > 0 ? t1[r - 1][v] : lA[bA][row - 1][col];
                    const C yp = r < R - 1 ? t1[r + 1][v] : lA[bA][row + 1][col];
                    u = stencil_point<DT>(t1[r][v], xm, xp, ym, yp, t0[r][v], t2[r][v], c0[r][v], a);
                }
                u2[r][v] = u;
                lB[bB][1 + wave * R + r][1 + lane * V + v] = u;
            }
            if constexpr (MID) {
                // own planes only (the halo planes belong to the neighbouring chunks)
                if (p >= zb && p < ze && xin && y >= 1 && y <= ny - 2 && zin) {
                    const size_t i0 = (size_t)xl + sy * y + sz * p;
                    S st[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) st[v] = Tr::store(u2[r][v], 0);   // FP64/FP32 only: exact
                    if (xl >= 1 && xl + V - 1 <= nx - 2) {
                        vstore<S, V>(a.Tmid + i0, st);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            if (xl + v >= 1 && xl + v <= nx - 2) a.Tmid[i0 + v] = st[v];
                    }
                }
            }
        }
        if (yrole) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int x = xl + v, col = 2 + lane * V + v;
                C u = y1v[v];
                if (zin && xin && interior(x, yr1, p)) {
                    const C xm = v > 0 ? y1v[v - 1] : lA[bA][ay1][col - 1];
                    const C xp = v < V - 1 ? y1v[v + 1] : lA[bA][ay1][col + 1];
                    const C ym = lA[bA][ay1 - 1][col];
                    const C yp = lA[bA][ay1 + 1][col];
                    u = stencil_point<DT>(y1v[v], xm, xp, ym, yp, y0v[v], y2v[v], ycv0[v], a);
                }
                lB[bB][by1][1 + lane * V + v] = u;
            }
        }
        if (xrole && xmid) {
            C u = x1s;
            if (zin && interior(xc1, yx, p)) {
                const C xm = lA[bA][1 + lane][ax1 - 1];
                const C xp = lA[bA][1 + lane][ax1 + 1];
                const C ym = lA[bA][lane][ax1];
                const C yp = lA[bA][2 + lane][ax1];
                u = stencil_point<DT>(x1s, xm, xp, ym, yp, x0s, x2s, xcs0, a);
            }
            lB[bB][lane][bx1] = u;
        }

        // 4. T^{k+2}(p-1) on the tile from T^{k+1}(p-2 .. p)
        if (p >= zb + 1) {
            const int q = p - 1;
            const int bq = bB ^ 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int y = yw + r;
                if (!(xin && y >= 1 && y <= ny - 2)) continue;
                const int row = 1 + wave * R + r;
                C out[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int col = 1 + lane * V + v;
                    const C xm = v > 0 ? u1[r][v - 1] : lB[bq][row][col - 1];
                    const C xp = v < V - 1 ? u1[r][v + 1] : lB[bq][row][col + 1];
                    const C ym = r > 0 ? u1[r - 1][v] : lB[bq][row - 1][col];
                    const C yp = r < R - 1 ? u1[r + 1][v] : lB[bq][row + 1][col];
                    out[v] = stencil_point<DT>(u1[r][v], xm, xp, ym, yp, u0[r][v], u2[r][v], cm[r][v], a);
                }
                const size_t i0 = (size_t)xl + sy * y + sz * q;
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
        }

        // 5. shift the plane window
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                t0[r][v] = t1[r][v];
                t1[r][v] = t2[r][v];
                t2[r][v] = t3[r][v];
                u0[r][v] = u1[r][v];
                u1[r][v] = u2[r][v];
                cm[r][v] = c0[r][v];
                c0[r][v] = c1[r][v];
            }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            y0v[v] = y1v[v];
            y1v[v] = y2v[v];
            y2v[v] = y3v[v];
            ycv0[v] = ycv1[v];
            l2a[v] = l2b[v];
        }
        x0s = x1s;
        x1s = x2s;
        x2s = x3s;
        xcs0 = xcs1;
        l2xa = l2xb;
        bA ^= 1;
        bB ^= 1;
    }
}

}  // namespace diff3d

#include "adjoint_kernels.hpp"

namespace diff3d {

// Two adjoint steps per pass: from lambda_{k+1} (a.lin), T_k (a.Tk) and
// T_{k-1} (a.Tk1) to lambda_{k-1} (a.lout), adding both steps' terms to gCi
// in the order of two single adjoint steps (bit-identical for FP64/FP32).
// Per plane p the workgroup
//   A. computes lambda_k(p) on the tile and on the one-point ring (no
//      corners) from mu_{k+1} = dt*lam*Ci*lambda_{k+1} staged in LDS with a
//      two-point ring, then mu_k = dt*lam*Ci*lambda_k (LDS, registers), and
//      the partial gCi(p) + dt*lam*lambda_{k+1}*Lap(T_k) on the tile;
//   B. computes lambda_{k-1}(p-1) = lambda_k + Lap(mu_k) on the tile (every
//      point, boundary included) and gCi(p-1) += dt*lam*lambda_k*Lap(T_{k-1})
//      on interior points, and stores both.
// Outputs cover planes zb .. ze-1 of all nz planes; mu is 0 outside the
// interior.  Ring roles and the pipeline follow step_tb2.
template <int DT, int V, int R, int NW>
__global__ __launch_bounds__(64 * NW) void adj_tb2(AdjArgs<DT> a, int ntx, int nty, int zlen)
{
    using Tr = Traits<DT>;
    using S = typename Tr::S;
    using C = typename Tr::C;
    constexpr int TX = 64 * V, TY = R * NW;
    constexpr int WYL = 0, WYH = NW - 1, WXL = 1, WXR = 2;
    static_assert(NW >= 4, "the four ring roles need four distinct waves");
    static_assert(TY + 2 <= 64, "ring columns are held one point per lane");
    __shared__ C lM1[2][TY + 4][TX + 4];   // mu_{k+1}, origin (y0 - 2, x0 - 2)
    __shared__ C lTA[2][TY + 2][TX + 2];   // T_k, origin (y0 - 1, x0 - 1)
    __shared__ C lM0[2][TY + 2][TX + 2];   // mu_k
    __shared__ C lTB[2][TY + 2][TX + 2];   // T_{k-1}

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)ntx);
    const int rest = (int)(t / (unsigned)ntx);
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY;
    const int zb = tz * zlen;                    // output planes zb .. ze-1
    const int ze = min(nz, zb + zlen);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xl = x0 + lane * V;
    const bool xin = xl < nx;
    const int yw = y0 + wave * R;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;

    const bool yrole = wave == WYL || wave == WYH;
    const int yr1 = wave == WYL ? y0 - 1 : y0 + TY;
    const int yr2 = wave == WYL ? y0 - 2 : y0 + TY + 1;
    const int ay1 = wave == WYL ? 1 : TY + 2;
    const int ay2 = wave == WYL ? 0 : TY + 3;
    const int by1 = wave == WYL ? 0 : TY + 1;
    const bool xrole = (wave == WXL || wave == WXR) && lane < TY + 2;
    const int xc1 = wave == WXL ? x0 - 1 : x0 + TX;
    const int xc2 = wave == WXL ? x0 - 2 : x0 + TX + 1;
    const int ax1 = wave == WXL ? 1 : TX + 2;
    const int ax2 = wave == WXL ? 0 : TX + 3;
    const int bx1 = wave == WXL ? 0 : TX + 1;
    const int yx = y0 - 1 + lane;
    const bool xmid = lane >= 1 && lane <= TY;

    const bool yin1 = yrole && xin && yr1 >= 0 && yr1 < ny;
    const bool yin2 = yrole && xin && yr2 >= 0 && yr2 < ny;
    const bool xin1 = xrole && xc1 >= 0 && xc1 < nx && yx >= 0 && yx < ny;
    const bool xin2 = xrole && xmid && xc2 >= 0 && xc2 < nx && yx >= 0 && yx < ny;

    using Rows = C[R][V];
    using Vec = C[V];
    auto inner = [&](int x, int y, int z) __attribute__((always_inline)) {
        return x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
    };
    // V points from (x, y, z) of one field, zero outside the grid
    auto vld = [&](const S* base, int x, int y, int z, Vec& dst, bool ok) __attribute__((always_inline)) {
        if (ok && z >= 0 && z < nz) {
            S raw[V];
            vload<S, V>(base + (size_t)x + sy * y + sz * z, raw);
#pragma unroll
            for (int v = 0; v < V; ++v) dst[v] = Tr::load(raw[v]);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) dst[v] = C(0);
        }
    };
    auto sld = [&](const S* base, int x, int y, int z, C& dst, bool ok) __attribute__((always_inline)) {
        dst = (ok && z >= 0 && z < nz) ? Tr::load(base[(size_t)x + sy * y + sz * z]) : C(0);
    };
    // mu = dt*lam*Ci*lambda on interior points, 0 elsewhere
    auto muv = [&](int x, int y, int z, const Vec& ci, const Vec& l, Vec& m) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < V; ++v) m[v] = inner(x + v, y, z) ? a.dtlam * ci[v] * l[v] : C(0);
    };

    // ---- register state; index 0 = oldest plane
    Rows m1[4];     // tile mu_{k+1} at p-1 .. p+2
    Rows l1[3];     // tile lambda_{k+1} at p .. p+2
    Rows c1[3];     // tile Ci at p .. p+2
    Rows ta[4];     // tile T_k at p-1 .. p+2
    Rows tb[4];     // tile T_{k-1} at p-2 .. p+1
    Rows g[2];      // tile gCi at p, p+1
    Rows g1m;       // tile gCi + step-k term at p-1
    Rows m0[3];     // tile mu_k at p-2 .. p
    Rows lkm;       // tile lambda_k at p-1
    Vec ym1[4], yl1[3], yc1[3], yta[2], ytb[2], ym2[2];   // y roles: ring row
    C xm1[4], xl1[3], xc1v[3], xta[2], xtb[2], xm2[2];    // x roles: ring column (lanes 0..TY+1)

    auto zero_rows = [&](Rows& r_) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) r_[r][v] = C(0);
    };
    auto copy_rows = [&](Rows& d, const Rows& s_) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) d[r][v] = s_[r][v];
    };
    auto copy_vec = [&](Vec& d, const Vec& s_) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = s_[v];
    };
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        zero_rows(m1[i]);
        zero_rows(ta[i]);
        zero_rows(tb[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        zero_rows(l1[i]);
        zero_rows(c1[i]);
        zero_rows(m0[i]);
    }
    zero_rows(g[0]);
    zero_rows(g[1]);
    zero_rows(g1m);
    zero_rows(lkm);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        for (int i = 0; i < 4; ++i) ym1[i][v] = C(0);
        for (int i = 0; i < 3; ++i) yl1[i][v] = yc1[i][v] = C(0);
        for (int i = 0; i < 2; ++i) yta[i][v] = ytb[i][v] = ym2[i][v] = C(0);
    }
    for (int i = 0; i < 4; ++i) xm1[i] = C(0);
    for (int i = 0; i < 3; ++i) xl1[i] = xc1v[i] = C(0);
    for (int i = 0; i < 2; ++i) xta[i] = xtb[i] = xm2[i] = C(0);

    // lambda_{k+1}, Ci and mu_{k+1} of plane z: tile and first ring;
    // second-ring mu_{k+1} into (r2y, r2x)
    auto load_lam = [&](int z, Rows& m, Rows& l, Rows& c, Vec& ym, Vec& yl, Vec& yc, C& xm, C& xl_, C& xc,
                        Vec& r2y, C& r2x) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool ok = xin && yw + r < ny;
            vld(a.lin, xl, yw + r, z, l[r], ok);
            vld(a.Ci, xl, yw + r, z, c[r], ok);
            muv(xl, yw + r, z, c[r], l[r], m[r]);
        }
        vld(a.lin, xl, yr1, z, yl, yin1);
        vld(a.Ci, xl, yr1, z, yc, yin1);
        muv(xl, yr1, z, yc, yl, ym);
        sld(a.lin, xc1, yx, z, xl_, xin1);
        sld(a.Ci, xc1, yx, z, xc, xin1);
        xm = inner(xc1, yx, z) ? a.dtlam * xc * xl_ : C(0);
        Vec l2, c2;
        vld(a.lin, xl, yr2, z, l2, yin2);
        vld(a.Ci, xl, yr2, z, c2, yin2);
        muv(xl, yr2, z, c2, l2, r2y);
        C l2x, c2x;
        sld(a.lin, xc2, yx, z, l2x, xin2);
        sld(a.Ci, xc2, yx, z, c2x, xin2);
        r2x = inner(xc2, yx, z) ? a.dtlam * c2x * l2x : C(0);
    };
    // a forward state of plane z: tile and first ring (no corners)
    auto load_state = [&](const S* base, int z, Rows& tile, Vec& yv, C& xv) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) vld(base, xl, yw + r, z, tile[r], xin && yw + r < ny);
        vld(base, xl, yr1, z, yv, yin1);
        sld(base, xc1, yx, z, xv, xin1 && xmid);
    };
    auto load_g = [&](int z, Rows& dst) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) vld(a.gCi, xl, yw + r, z, dst[r], xin && yw + r < ny);
    };
    auto stage_m1 = [&](int buf, const Rows& m, const Vec& ym, C xm, const Vec& r2y, C r2x)
        __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) lM1[buf][2 + wave * R + r][2 + lane * V + v] = m[r][v];
        if (yrole) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                lM1[buf][ay1][2 + lane * V + v] = ym[v];
                lM1[buf][ay2][2 + lane * V + v] = r2y[v];
            }
        }
        if (xrole) {
            lM1[buf][1 + lane][ax1] = xm;
            if (xmid) lM1[buf][1 + lane][ax2] = r2x;
        }
    };
    auto stage_ring1 = [&](C (&L)[2][TY + 2][TX + 2], int buf, const Rows& tile, const Vec& yv, C xv)
        __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < V; ++v) L[buf][1 + wave * R + r][1 + lane * V + v] = tile[r][v];
        if (yrole)
#pragma unroll
            for (int v = 0; v < V; ++v) L[buf][by1][1 + lane * V + v] = yv[v];
        if (xrole && xmid) L[buf][lane][bx1] = xv;
    };

    const int p0 = zb - 1;
    // prologue: mu_{k+1} at p0-1 .. p0+1 (plane p0 staged with both rings),
    // second ring of p0+1, T_k at p0-1 .. p0+1 (p0 staged), T_{k-1} at
    // p0-1, p0, gCi at p0
    {
        Vec r2y;
        C r2x;
        Rows ldum, cdum;
        Vec yldum, ycdum;
        C xldum, xcdum;
        load_lam(p0 - 1, m1[0], ldum, cdum, ym1[0], yldum, ycdum, xm1[0], xldum, xcdum, r2y, r2x);
        load_lam(p0, m1[1], l1[0], c1[0], ym1[1], yl1[0], yc1[0], xm1[1], xl1[0], xc1v[0], r2y, r2x);
        stage_m1(0, m1[1], ym1[1], xm1[1], r2y, r2x);
        load_lam(p0 + 1, m1[2], l1[1], c1[1], ym1[2], yl1[1], yc1[1], xm1[2], xl1[1], xc1v[1], ym2[0], xm2[0]);
        Vec ydum;
        C xdum;
        load_state(a.Tk, p0 - 1, ta[0], ydum, xdum);
        load_state(a.Tk, p0, ta[1], yta[0], xta[0]);
        stage_ring1(lTA, 0, ta[1], yta[0], xta[0]);
        load_state(a.Tk, p0 + 1, ta[2], yta[1], xta[1]);
        load_state(a.Tk1, p0 - 1, tb[1], ydum, xdum);
        load_state(a.Tk1, p0, tb[2], ytb[0], xtb[0]);
        load_g(p0, g[0]);
    }

    int b = 0;
    for (int p = p0; p <= ze; ++p) {
        const bool more = p + 1 <= ze;
        // 1. loads one plane ahead
        if (more) {
            load_lam(p + 2, m1[3], l1[2], c1[2], ym1[3], yl1[2], yc1[2], xm1[3], xl1[2], xc1v[2], ym2[1], xm2[1]);
            load_state(a.Tk, p + 2, ta[3], yta[0], xta[0]);   // ring T_k of p+2 (index 0 is free)
            load_state(a.Tk1, p + 1, tb[3], ytb[1], xtb[1]);
            load_g(p + 1, g[1]);
        }
        lds_barrier();
        // 2. stage mu_{k+1} and T_k of plane p+1, T_{k-1} of plane p
        if (more) {
            stage_m1(b ^ 1, m1[2], ym1[2], xm1[2], ym2[0], xm2[0]);
            stage_ring1(lTA, b ^ 1, ta[2], yta[1], xta[1]);
        }
        stage_ring1(lTB, b, tb[2], ytb[0], xtb[0]);

        // A. lambda_k(p) and mu_k(p) on tile and ring; partial gCi on the tile
        const bool pin = p >= 0 && p <= nz - 1;
        Rows lk, mk, g1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yw + r;
            const int rowA = 2 + wave * R + r, rowB = 1 + wave * R + r;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int x = xl + v, colA = 2 + lane * V + v, colB = 1 + lane * V + v;
                const C mxm = v > 0 ? m1[1][r][v - 1] : lM1[b][rowA][colA - 1];
                const C mxp = v < V - 1 ? m1[1][r][v + 1] : lM1[b][rowA][colA + 1];
                const C mym = r > 0 ? m1[1][r - 1][v] : lM1[b][rowA - 1][colA];
                const C myp = r < R - 1 ? m1[1][r + 1][v] : lM1[b][rowA + 1][colA];
                const C lm = lap7<DT>(m1[1][r][v], mxm, mxp, mym, myp, m1[0][r][v], m1[2][r][v], a);
                const C l = pin ? Tr::load(Tr::store(l1[0][r][v] + lm, 0)) : C(0);
                lk[r][v] = l;
                mk[r][v] = (pin && inner(x, y, p)) ? a.dtlam * c1[0][r][v] * l : C(0);
                lM0[b][rowB][colB] = mk[r][v];
                g1[r][v] = g[0][r][v];
                if (xin && inner(x, y, p)) {
                    const C txm = v > 0 ? ta[1][r][v - 1] : lTA[b][rowB][colB - 1];
                    const C txp = v < V - 1 ? ta[1][r][v + 1] : lTA[b][rowB][colB + 1];
                    const C tym = r > 0 ? ta[1][r - 1][v] : lTA[b][rowB - 1][colB];
                    const C typ = r < R - 1 ? ta[1][r + 1][v] : lTA[b][rowB + 1][colB];
                    const C ltk = lap7<DT>(ta[1][r][v], txm, txp, tym, typ, ta[0][r][v], ta[2][r][v], a);
                    g1[r][v] = Tr::load(Tr::store(g[0][r][v] + a.dtlam * l1[0][r][v] * ltk, 0));
                }
            }
        }
        if (yrole) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int x = xl + v, colA = 2 + lane * V + v;
                const C mxm = v > 0 ? ym1[1][v - 1] : lM1[b][ay1][colA - 1];
                const C mxp = v < V - 1 ? ym1[1][v + 1] : lM1[b][ay1][colA + 1];
                const C lm = lap7<DT>(ym1[1][v], mxm, mxp, lM1[b][ay1 - 1][colA], lM1[b][ay1 + 1][colA], ym1[0][v],
                                      ym1[2][v], a);
                const C l = pin ? Tr::load(Tr::store(yl1[0][v] + lm, 0)) : C(0);
                lM0[b][by1][1 + lane * V + v] = (pin && inner(x, yr1, p)) ? a.dtlam * yc1[0][v] * l : C(0);
            }
        }
        if (xrole && xmid) {
            const C lm = lap7<DT>(xm1[1], lM1[b][1 + lane][ax1 - 1], lM1[b][1 + lane][ax1 + 1], lM1[b][lane][ax1],
                                  lM1[b][2 + lane][ax1], xm1[0], xm1[2], a);
            const C l = pin ? Tr::load(Tr::store(xl1[0] + lm, 0)) : C(0);
            lM0[b][lane][bx1] = (pin && inner(xc1, yx, p)) ? a.dtlam * xc1v[0] * l : C(0);
        }

        // B. lambda_{k-1}(p-1) and gCi(p-1) on the tile
        if (p >= zb + 1) {
            const int q = p - 1;
            const int bq = b ^ 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int y = yw + r;
                if (!(xin && y < ny)) continue;
                const int row = 1 + wave * R + r;
                const size_t i0 = (size_t)xl + sy * y + sz * q;
                S lo[V], go[V];
                bool anyin = false;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int col = 1 + lane * V + v;
                    const C mxm = v > 0 ? m0[1][r][v - 1] : lM0[bq][row][col - 1];
                    const C mxp = v < V - 1 ? m0[1][r][v + 1] : lM0[bq][row][col + 1];
                    const C mym = r > 0 ? m0[1][r - 1][v] : lM0[bq][row - 1][col];
                    const C myp = r < R - 1 ? m0[1][r + 1][v] : lM0[bq][row + 1][col];
                    const C lm = lap7<DT>(m0[1][r][v], mxm, mxp, mym, myp, m0[0][r][v], mk[r][v], a);
                    lo[v] = Tr::store(lkm[r][v] + lm, 0);
                    go[v] = Tr::store(g1m[r][v], 0);
                    if (inner(xl + v, y, q)) {
                        anyin = true;
                        const C txm = v > 0 ? tb[1][r][v - 1] : lTB[bq][row][col - 1];
                        const C txp = v < V - 1 ? tb[1][r][v + 1] : lTB[bq][row][col + 1];
                        const C tym = r > 0 ? tb[1][r - 1][v] : lTB[bq][row - 1][col];
                        const C typ = r < R - 1 ? tb[1][r + 1][v] : lTB[bq][row + 1][col];
                        const C ltk = lap7<DT>(tb[1][r][v], txm, txp, tym, typ, tb[0][r][v], tb[2][r][v], a);
                        go[v] = Tr::store(g1m[r][v] + a.dtlam * lkm[r][v] * ltk, 0);
                    }
                }
                vstore<S, V>(a.lout + i0, lo);
                if (anyin) {
                    if (xl >= 1 && xl + V - 1 <= nx - 2) {
                        vstore<S, V>(a.gCi + i0, go);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            if (xl + v >= 1 && xl + v <= nx - 2) a.gCi[i0 + v] = go[v];
                    }
                }
            }
        }

        // shift the plane window
        copy_rows(m1[0], m1[1]);
        copy_rows(m1[1], m1[2]);
        copy_rows(m1[2], m1[3]);
        copy_rows(l1[0], l1[1]);
        copy_rows(l1[1], l1[2]);
        copy_rows(c1[0], c1[1]);
        copy_rows(c1[1], c1[2]);
        copy_rows(ta[0], ta[1]);
        copy_rows(ta[1], ta[2]);
        copy_rows(ta[2], ta[3]);
        copy_rows(tb[0], tb[1]);
        copy_rows(tb[1], tb[2]);
        copy_rows(tb[2], tb[3]);
        copy_rows(g[0], g[1]);
        copy_rows(g1m, g1);
        copy_rows(m0[0], m0[1]);
        copy_rows(m0[1], mk);
        copy_rows(lkm, lk);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            ym1[0][v] = ym1[1][v];
            ym1[1][v] = ym1[2][v];
            ym1[2][v] = ym1[3][v];
            yl1[0][v] = yl1[1][v];
            yl1[1][v] = yl1[2][v];
            yc1[0][v] = yc1[1][v];
            yc1[1][v] = yc1[2][v];
            ym2[0][v] = ym2[1][v];
        }
        copy_vec(ytb[0], ytb[1]);
        // yta: index 1 holds plane p+1's ring (staged this iteration); the
        // ring of p+2 was loaded into index 0 and moves to index 1
        copy_vec(yta[1], yta[0]);
        xm1[0] = xm1[1];
        xm1[1] = xm1[2];
        xm1[2] = xm1[3];
        xl1[0] = xl1[1];
        xl1[1] = xl1[2];
        xc1v[0] = xc1v[1];
        xc1v[1] = xc1v[2];
        xm2[0] = xm2[1];
        xtb[0] = xtb[1];
        xta[1] = xta[0];
        b ^= 1;
    }
}

}  // namespace diff3d
