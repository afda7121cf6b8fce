// Two time steps per pass over HBM (temporal blocking) for the explicit 3-D
// heat-diffusion step.  T^{k+2} is computed from T^k with the same
// operations, in the same order, as two single steps: the intermediate
// T^{k+1} is rounded exactly as storing it would round it (stochastic
// rounding draws the same Philox bits for the same point and step), so the
// result is bit-identical to two launches of the single-step kernel.
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

    SrState sr1 = a.sr, sr2 = a.sr;
    sr2.s0 = a.sr.s0 + 1u;
    sr2.s1 = a.sr.s1 + (sr2.s0 == 0u ? 1u : 0u);

    using Rows = C[R][V];
    using Vec = C[V];
    auto interior = [&](int x, int y, int z) __attribute__((always_inline)) {
        return x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
    };
    // the value a single step would have stored and the next step loaded
    auto as_stored = [&](C v, size_t idx, const SrState& sr) __attribute__((always_inline)) -> C {
        uint32_t rnd = 0;
        if constexpr (Tr::sr) rnd = sr_word(sr_block(sr, idx >> 3), (unsigned)(idx & 7));
        return Tr::load(Tr::store(v, rnd));
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
    auto stage_A = [&](int buf, const Rows& own, const Vec& yv, const Vec& y2, C xs, C x2) __attribute__((always_inline)) {
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
                    u = as_stored(stencil_point<DT>(t1[r][v], xm, xp, ym, yp, t0[r][v], t2[r][v], c0[r][v], a),
                                  (size_t)x + sy * y + sz * p, sr1);
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
                    for (int v = 0; v < V; ++v) st[v] = Tr::store(u2[r][v], 0);   // exact: u2 is already rounded
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
                    u = as_stored(stencil_point<DT>(y1v[v], xm, xp, ym, yp, y0v[v], y2v[v], ycv0[v], a),
                                  (size_t)x + sy * yr1 + sz * p, sr1);
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
                u = as_stored(stencil_point<DT>(x1s, xm, xp, ym, yp, x0s, x2s, xcs0, a),
                              (size_t)xc1 + sy * yx + sz * p, sr1);
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
                    const u32x4 rb = sr_block(sr2, i0 >> 3);
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
