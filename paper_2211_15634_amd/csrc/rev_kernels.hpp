// Fused reverse pass over S steps: the forward states are recomputed on chip
// from one stored state, so the pass reads T_k, lambda_{k+S}, Ci and gCi once
// and writes lambda_k and gCi once, for S adjoint steps.
//
// The adjoint step (derivation with the single-step kernels):
//   gCi  = gCi + ((dt*lam)*lambda_{k+1})*Lap(T_k)          interior points
//   mu   = ((dt*lam)*Ci)*lambda_{k+1}                       interior, 0 elsewhere
//   lambda_k = lambda_{k+1} + Lap(mu)                       every point
// with Lap(A) = (d2x(A)*cx + d2y(A)*cy) + d2z(A)*cz.  Lap(T_k) is the same
// expression the forward update T_{k+1} = T_k + dt*((lam*Ci)*Lap(T_k)) forms,
// so recomputing T_{k+1} also yields Lap(T_k), bit for bit.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "fd_ops.hpp"

namespace diff3d {

template <int DT>
struct RevArgs {
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    S* __restrict__ lout;        // lambda_k (every point of the grid)
    const S* __restrict__ lin;   // lambda_{k+S}
    const S* __restrict__ Ci;
    const S* __restrict__ Tk;    // forward state T_k
    S* __restrict__ gCi;         // accumulated in place (interior points)
    int nx, ny, nz;
    C lam, dt, dtlam, cx, cy, cz;
};

// A workgroup owns a W0 x H0 region (origin tx*TX, ty*TY; TX = W0-2S,
// TY = H0-2S) and outputs lambda_k and gCi on its tile, the region without a
// border of S points (region sides on the grid's boundary do not shrink: the
// forward boundary values are fixed and mu is zero beyond the interior, so
// points next to the boundary are computable at every level).  It marches
// along z over chunks of `zlen` output planes (all planes 0..nz-1 are
// outputs).  Levels, each on the region without a border of its index:
//   F_f = T_{k+f}, f = 0..S-1 (F_0 loaded), computed at plane p-f+1 in plane
//         iteration p, together with Lap(F_{f-1}) at the same plane; the
//         last stencil (f = S) forms only Lap(F_{S-1});
//   L_j = lambda_{k+S-j}, j = 0..S (L_0 loaded), computed at plane p-S-j+2,
//         from mu_{j-1} = dt*lam*Ci*L_{j-1}, adding to gCi on the tile
//         dt*lam*L_{j-1}*Lap(F_{S-j}) (steps k+S-1 down to k, in that order).
// Lap(F_{S-j}) is formed 2j-2 iterations before level j uses it and waits in
// a register ring.  x/y neighbours of F_f and mu_j come from their planes
// staged in double-buffered LDS in the previous iteration (one barrier per
// plane; with two points per thread on adjacent rows, the y neighbour across
// the pair from the other point's registers); z neighbours from registers.
// Loads are issued one or two plane
// iterations before the one that uses them, from addresses clamped into the
// grid (values outside the grid are never used).
template <int DT, int S, int W0, int H0, int NTH>
__global__ __launch_bounds__(NTH) void rev_tbs(RevArgs<DT> a, int ntx, int nty, int zlen)
{
    using Tr = Traits<DT>;
    using S_ = typename Tr::S;
    using C = typename Tr::C;
    constexpr int TX = W0 - 2 * S, TY = H0 - 2 * S, A0 = W0 * H0;
    static_assert(S >= 2, "single reverse steps use the adjoint step kernels");
    static_assert(TX > 0 && TY > 0, "region too small for S steps");
    static_assert(W0 % 64 == 0 && NTH % 64 == 0, "a wave must cover whole region rows");
    constexpr int K = (A0 + NTH - 1) / NTH;       // region points per thread
    constexpr int NCI = 2 * S - 2;                // Ci planes held: p .. p-2S+3
    __shared__ C lf[S][2][A0];                    // F_0 .. F_{S-1}
    // mu planes carry a border of zeros (one row above and below, one column
    // left and right): mu is zero beyond the grid, so a lambda stencil at the
    // grid's edge reads its missing neighbours as stored zeros
    constexpr int WP = W0 + 2, AP = WP * (H0 + 2);
    __shared__ C lm[S][2][AP];                    // mu_0 .. mu_{S-1}

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)ntx);
    const int rest = (int)(t / (unsigned)ntx);
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY;
    const bool ex0 = x0 == 0, ex1 = x0 + W0 >= nx, ey0 = y0 == 0, ey1 = y0 + H0 >= ny;
    const int ox0 = ex0 ? 0 : x0 + S, ox1 = ex1 ? nx : x0 + W0 - S;
    const int oy0 = ey0 ? 0 : y0 + S, oy1 = ey1 ? ny : y0 + H0 - S;
    const int zb = tz * zlen;                     // output planes zb .. ze-1
    const int ze = min(nz, zb + zlen);
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;

    // two points per thread (FP32) on adjacent region rows of one wave (rows
    // 2w and 2w+1): the y neighbour across the pair comes from the other
    // point's registers, the outer two from LDS (256^3 FP32 reverse sweep
    // 13.6 -> 13.4 ms)
    constexpr bool kRowsY = K == 2 && W0 == 64 && A0 == K * NTH;
    int rr[K], cc[K], gx[K], gy[K];
    size_t base[K];
    bool live[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = kRowsY ? ((((int)threadIdx.x >> 6) * K + k) << 6) + ((int)threadIdx.x & 63)
                               : (int)threadIdx.x + k * NTH;
        live[k] = idx < A0;
        rr[k] = live[k] ? idx / W0 : 0;
        cc[k] = live[k] ? idx % W0 : 0;
        gx[k] = x0 + cc[k];
        gy[k] = y0 + rr[k];
        base[k] = (size_t)min(max(gx[k], 0), nx - 1) + sy * (size_t)min(max(gy[k], 0), ny - 1);
    }
    auto in_level = [&](int k, int s) __attribute__((always_inline)) {
        return live[k] && (rr[k] >= s || ey0) && (rr[k] < H0 - s || ey1) && (cc[k] >= s || ex0) &&
               (cc[k] < W0 - s || ex1);
    };
    auto in_grid = [&](int k) __attribute__((always_inline)) {
        return gx[k] >= 0 && gx[k] < nx && gy[k] >= 0 && gy[k] < ny;
    };
    auto inner_xy = [&](int k) __attribute__((always_inline)) {
        return gx[k] >= 1 && gx[k] <= nx - 2 && gy[k] >= 1 && gy[k] <= ny - 2;
    };
    auto on_tile = [&](int k) __attribute__((always_inline)) {
        return gx[k] >= ox0 && gx[k] < ox1 && gy[k] >= oy0 && gy[k] < oy1;
    };
    auto gidx = [&](int k, int z) __attribute__((always_inline)) {
        return (size_t)gx[k] + sy * gy[k] + sz * z;
    };
    auto load = [&](const S_* f, int z, C (&dst)[K]) __attribute__((always_inline)) {
        const size_t zo = sz * (size_t)min(max(z, 0), nz - 1);
#pragma unroll
        for (int k = 0; k < K; ++k) dst[k] = Tr::load(f[base[k] + zo]);
    };
    auto lap = [&](C t, C xm, C xp, C ym, C yp, C zm, C zp) __attribute__((always_inline)) -> C {
        return fd::lap3(t, xm, xp, ym, yp, zm, zp, a.cx, a.cy, a.cz);
    };
    auto stage = [&](C (&buf)[A0], const C (&src)[K]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (live[k]) buf[rr[k] * W0 + cc[k]] = src[k];
    };
    auto stage_mu = [&](C (&buf)[AP], const C (&src)[K]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (live[k]) buf[(rr[k] + 1) * WP + cc[k] + 1] = src[k];
    };
    // the zero border, written once (staging writes only the region's cells)
    for (int i = (int)threadIdx.x; i < S * 2 * AP; i += NTH) {
        const int q = i % AP, r = q / WP, c = q % WP;
        if (r == 0 || r == H0 + 1 || c == 0 || c == WP - 1) (&lm[0][0][0])[i] = C(0);
    }
    // per-point conditions that do not change along z, one bit each
    constexpr int G_BIT = 2 * S, O_BIT = 2 * S + 1, M_BIT = 2 * S + 2;
    unsigned act[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        unsigned b = 0;
#pragma unroll
        for (int f = 1; f <= S; ++f) b |= (in_level(k, f) && inner_xy(k)) ? 1u << (f - 1) : 0u;
#pragma unroll
        for (int j = 1; j <= S; ++j) b |= (in_level(k, j) && in_grid(k)) ? 1u << (S + j - 1) : 0u;
        b |= (live[k] && inner_xy(k) && on_tile(k)) ? 1u << G_BIT : 0u;
        b |= (in_level(k, S) && in_grid(k) && on_tile(k)) ? 1u << O_BIT : 0u;
        b |= (live[k] && inner_xy(k)) ? 1u << M_BIT : 0u;
        act[k] = b;
    }
    auto bit = [&](int k, int b) __attribute__((always_inline)) { return ((act[k] >> b) & 1u) != 0; };
    // z in [lo, hi) as one unsigned comparison (every range below has
    // lo <= hi: chunks start inside the grid, zb < ze, nz >= 3)
    auto in_range = [](int z, int lo, int hi) __attribute__((always_inline)) {
        return (unsigned)(z - lo) < (unsigned)(hi - lo);
    };
    const int zi0 = max(zb, 1), zi1 = min(ze, nz - 1);   // chunk planes that are interior
    // gCi is read only where this workgroup writes it (tile, interior, plane
    // of this chunk): other workgroups update the rest concurrently
    auto load_g = [&](int z, C (&dst)[K]) __attribute__((always_inline)) {
        const bool zok = in_range(z, zi0, zi1);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            dst[k] = C(0);
            if (zok && bit(k, G_BIT)) dst[k] = Tr::load(a.gCi[gidx(k, z)]);
        }
    };
    // mu of a point at plane z from lambda and Ci there (0 off the interior)
    auto mu_of = [&](int k, int z, C l, C ci) __attribute__((always_inline)) -> C {
        const bool in = bit(k, M_BIT) && in_range(z, 1, nz - 1);
        return in ? (a.dtlam * ci) * l : C(0);
    };

    // registers (per point)
    C t0[3][K];                                   // F_0 at planes p-1, p, p+1
    C uf[S - 1][2][K];                            // F_f (f = 1..S-1): the two planes below the fresh one
    C cr[NCI][K];                                 // Ci at planes p, p-1, .., p-2S+3
    C lpr[S][2 * S - 1][K];                       // Lap(F_{S-j}) for level j, by age (slots 0..2j-2)
    C lh[S][K];                                   // L_{j-1} at the centre plane of level j
    C mh[S][2][K];                                // mu_{j-1} at the two planes below the fresh one
    C g[S][K];                                    // gCi partial sum of the plane level j+1 works on
    C lt[2][K], lc[2][K], ll[2][K], lg[2][K];     // loads in flight: T, Ci, lambda, gCi
    // FP64: lambda and gCi are loaded two plane iterations before their use
    // (the waves otherwise wait on them: 256^3 reverse sweep 22.0 -> 20.8
    // ms); FP32 at two points per thread would spill with the longer
    // lifetimes (13.4 -> 14.6 ms) and keeps one iteration.
    constexpr bool kFar = sizeof(C) == 8;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int f = 0; f < S - 1; ++f) uf[f][0][k] = uf[f][1][k] = C(0);
#pragma unroll
        for (int i = 0; i < NCI; ++i) cr[i][k] = C(0);
#pragma unroll
        for (int j = 0; j < S; ++j) {
#pragma unroll
            for (int i = 0; i < 2 * S - 1; ++i) lpr[j][i][k] = C(0);
            lh[j][k] = mh[j][0][k] = mh[j][1][k] = g[j][k] = C(0);
        }
    }

    // First iteration: forward level 1 starts at plane zb-S+1, and mu_0 is
    // needed from plane zb-S (below level 1's first plane), which arrives in
    // iteration zb-2.  Level S's last plane ze-1 is reached in iteration
    // ze+2S-3.
    const int p0 = min(zb - S + 1, zb - 2);
    const int plast = ze + 2 * S - 3;
    // prologue: what the first iteration reads
    load(a.Tk, p0 - 1, t0[0]);
    load(a.Tk, p0, t0[1]);
    load(a.Tk, p0 + 1, t0[2]);
    load(a.Tk, p0 + 2, lt[0]);
#pragma unroll
    for (int i = 0; i < NCI; ++i) load(a.Ci, p0 - i, cr[i]);
    load(a.Ci, p0 + 1, lc[0]);
    load(a.lin, p0 - S + 2, ll[0]);
    load_g(p0 - S + 1, lg[0]);
    if constexpr (kFar) {
        load(a.lin, p0 - S + 3, ll[1]);
        load_g(p0 - S + 2, lg[1]);
    }
    stage(lf[0][1], t0[1]);

    auto iteration = [&](auto par, int p) __attribute__((always_inline)) {
        constexpr int PAR = decltype(par)::value;
        constexpr int buf = PAR, rbuf = PAR ^ 1;
        // T and Ci two iterations ahead; lambda and gCi one ahead (or two,
        // issued below, with kFar)
        load(a.Tk, p + 3, lt[PAR ^ 1]);
        load(a.Ci, p + 2, lc[PAR ^ 1]);
        if constexpr (!kFar) {
            load(a.lin, p - S + 3, ll[PAR ^ 1]);
            load_g(p - S + 2, lg[PAR ^ 1]);
        }
        lds_barrier();
        stage(lf[0][buf], t0[2]);                 // F_0 at p+1

        // ---- forward: stencil f at plane z = p-f+1 on F_{f-1}
        C prev[K];                                // F_{f-1} at z+1
#pragma unroll
        for (int k = 0; k < K; ++k) prev[k] = t0[2][k];
#pragma unroll
        for (int f = 1; f <= S; ++f) {
            const int z = p - f + 1;
            // F_f is needed on planes [zb-(S-f), ze+(S-f)); Lap(F_{S-1}) on [zb, ze)
            const bool zact = in_range(z, max(zb - (S - f), 1), min(ze + (S - f), nz - 1));
            C out[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const C zm = f == 1 ? t0[0][k] : uf[f - 2][0][k];
                const C ce = f == 1 ? t0[1][k] : uf[f - 2][1][k];
                const C zp = prev[k];
                C v = ce, lp = C(0);
                if (zact && bit(k, f - 1)) {
                    const int i = rr[k] * W0 + cc[k];
                    const C ceo = f == 1 ? t0[1][k ^ 1] : uf[f - 2][1][k ^ 1];
                    const C ym = (kRowsY && k == 1) ? ceo : lf[f - 1][rbuf][i - W0];
                    const C yp = (kRowsY && k == 0) ? ceo : lf[f - 1][rbuf][i + W0];
                    lp = lap(ce, lf[f - 1][rbuf][i - 1], lf[f - 1][rbuf][i + 1], ym, yp, zm, zp);
                    if (f < S) v = fd::update(ce, a.dt, a.lam * cr[f - 1][k], lp);
                }
                out[k] = v;
                lpr[S - f][0][k] = lp;            // Lap(F_{f-1}) serves level j = S-f+1
            }
            if (f > 1) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    uf[f - 2][0][k] = uf[f - 2][1][k];
                    uf[f - 2][1][k] = prev[k];
                }
            }
            if (f < S) {
                stage(lf[f][buf], out);
#pragma unroll
                for (int k = 0; k < K; ++k) prev[k] = out[k];
            }
        }

        // ---- adjoint: L_0 arrives at plane p-S+2; mu_0 there
        C lprev[K], mprev[K];                     // L_{j-1}, mu_{j-1} at the fresh plane
        {
            const int z = p - S + 2;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                lprev[k] = ll[PAR][k];
                mprev[k] = mu_of(k, z, lprev[k], cr[S - 2][k]);
            }
            stage_mu(lm[0][buf], mprev);
        }
        // gCi of plane p-S+1 enters the partial sums
#pragma unroll
        for (int k = 0; k < K; ++k) g[0][k] = lg[PAR][k];
        if constexpr (kFar) {
            // lambda and gCi two iterations ahead, into the slots just consumed
            load(a.lin, p - S + 4, ll[PAR]);
            load_g(p - S + 3, lg[PAR]);
        }
#pragma unroll
        for (int j = 1; j <= S; ++j) {
            const int z = p - S - j + 2;
            const bool zact = in_range(z, max(zb - (S - j), 0), min(ze + (S - j), nz));
            const bool zin = in_range(z, 1, nz - 1);
            const bool zout = in_range(z, zb, ze);
            C out[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const C lc0 = lh[j - 1][k];       // L_{j-1} at z
                C v = lc0;
                if (zact && bit(k, S + j - 1)) {
                    const int i = (rr[k] + 1) * WP + cc[k] + 1;
                    const C mc = mh[j - 1][1][k];
                    const C xm = lm[j - 1][rbuf][i - 1];
                    const C xp = lm[j - 1][rbuf][i + 1];
                    const C mco = mh[j - 1][1][k ^ 1];
                    const C ym = (kRowsY && k == 1) ? mco : lm[j - 1][rbuf][i - WP];
                    const C yp = (kRowsY && k == 0) ? mco : lm[j - 1][rbuf][i + WP];
                    v = lc0 + lap(mc, xm, xp, ym, yp, mh[j - 1][0][k], mprev[k]);
                    if (in_range(z, zi0, zi1) && bit(k, G_BIT))
                        g[j - 1][k] = g[j - 1][k] + (a.dtlam * lc0) * lpr[j - 1][2 * j - 2][k];
                }
                out[k] = v;
            }
            // mu_{j-1} history moves up; L_{j-1}'s centre becomes the fresh plane
#pragma unroll
            for (int k = 0; k < K; ++k) {
                mh[j - 1][0][k] = mh[j - 1][1][k];
                mh[j - 1][1][k] = mprev[k];
                lh[j - 1][k] = lprev[k];
            }
            if (j < S) {
                const int ci_slot = S + j - 2;    // Ci at plane z
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    lprev[k] = out[k];
                    mprev[k] = mu_of(k, z, out[k], cr[ci_slot][k]);
                }
                stage_mu(lm[j][buf], mprev);
            } else if (zout) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (bit(k, O_BIT)) {
                        a.lout[gidx(k, z)] = Tr::store(out[k], 0);
                        if (zin && bit(k, M_BIT)) a.gCi[gidx(k, z)] = Tr::store(g[S - 1][k], 0);
                    }
                }
            }
        }

        // ---- shifts for the next plane
#pragma unroll
        for (int k = 0; k < K; ++k) {
            t0[0][k] = t0[1][k];
            t0[1][k] = t0[2][k];
            t0[2][k] = lt[PAR][k];
#pragma unroll
            for (int i = NCI - 1; i >= 1; --i) cr[i][k] = cr[i - 1][k];
            cr[0][k] = lc[PAR][k];
#pragma unroll
            for (int j = S - 1; j >= 1; --j) g[j][k] = g[j - 1][k];
#pragma unroll
            for (int j = 2; j <= S; ++j)
#pragma unroll
                for (int i = 2 * j - 2; i >= 1; --i) lpr[j - 1][i][k] = lpr[j - 1][i - 1][k];
        }
    };
    // Plane iterations, unrolled far enough that the z-history rings (up to
    // six planes long) mostly rotate by renaming registers instead of
    // copying them: four-way, except for two points per thread with three
    // steps per pass, where four-way would exceed 128 VGPRs (two-way).
    constexpr int UNR = (K > 1 && S > 2) ? 2 : 4;
    for (int p = p0; p <= plast; p += UNR) {
        iteration(std::integral_constant<int, 0>{}, p);
        if constexpr (UNR == 2) {
            if (p + 1 <= plast) iteration(std::integral_constant<int, 1>{}, p + 1);
        } else {
            // leaving the loop (rather than skipping the remaining copies)
            // keeps the rings' register assignment fixed across the body
            if (p + 1 > plast) break;
            iteration(std::integral_constant<int, 1>{}, p + 1);
            if (p + 2 > plast) break;
            iteration(std::integral_constant<int, 0>{}, p + 2);
            if (p + 3 > plast) break;
            iteration(std::integral_constant<int, 1>{}, p + 3);
        }
    }
}

}  // namespace diff3d
