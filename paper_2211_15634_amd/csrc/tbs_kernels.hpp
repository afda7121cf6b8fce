// The S-step temporal-blocked forward kernel (S = 2..4 steps per pass over
// HBM).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "step_kernels.hpp"

namespace diff3d {

// S time steps per pass over HBM.  A workgroup of NTH threads owns a W0 x H0
// region in x-y; its output tile is the region without a border of S points
// (TX = W0 - 2S by TY = H0 - 2S).  Level s (s = 0 .. S, level 0 = the input
// T^k) is computed on the region without a border of s points, so level S
// is the tile.  A region side that reaches the grid's boundary plane does
// not shrink: the boundary values are the same at every level, so the
// points next to it are computable at every level.  Regions therefore start
// at the grid's edge (origin tx*TX, ty*TY) and the first and last tile of a
// row or column output up to S-1 more points.  With W0 = 64 each wave holds
// whole region rows (coalesced).  Every thread keeps the same region points
// at every level, so the z-history of a point (three planes per level, four
// for the input with its prefetch) stays in that thread's registers; x and y
// neighbours come from the level's plane staged in LDS (with whole rows per
// wave, x neighbours from the adjacent lanes instead, and for FP64 the y
// neighbour inside a wave's pair of rows from the thread's other point).
// Per plane iteration
// p, level s is computed at plane p - s + 1 from level s-1 (its planes
// p-s .. p-s+2), which is one LDS barrier per plane.
// Intermediate levels stay in the compute type (FP64 or FP32) on chip; only
// the output level is rounded to the storage type, so FP64 and FP32 results
// are bit-identical to S single steps and BF16 rounds once per pass.
//
// BF16 on 1024 threads and S >= 3 asks for eight waves per SIMD (at most 64
// VGPRs, two workgroups per CU; its LDS allows it): round to nearest fits
// without spills, and four-step passes at 512^3 take 100 us per step against
// 147 us at one workgroup per CU (two-step passes: 136 us); stochastic
// rounding fits with its raw-value rings, 136 us per step (one workgroup
// per CU: 174 us).
template <int DT, int S, int W0, int H0, int NTH>
constexpr int tbs_min_waves()
{
    return ((DT == DIFF3D_BF16_RNE || DT == DIFF3D_BF16) && NTH == 1024 && S >= 3) ? 8 : 1;
}

template <int DT, int S, int W0, int H0, int NTH, bool NT>
__global__ __launch_bounds__(NTH, (tbs_min_waves<DT, S, W0, H0, NTH>())) void step_tbs(StepArgs<DT> a, int ntx,
                                                                                     int nty, int zlen)
{
    using Tr = Traits<DT>;
    using S_ = typename Tr::S;
    using C = typename Tr::C;
    constexpr int TX = W0 - 2 * S, TY = H0 - 2 * S, A0 = W0 * H0;
    static_assert(TX > 0 && TY > 0, "region too small for S steps");
    constexpr int K = (A0 + NTH - 1) / NTH;       // region points per thread
    // levels 0 .. S-1, double-buffered; region row r is array row r + 1
    __shared__ C lds[S][2][H0 + 2][W0];
    // Stochastic rounding of the stored level: the 64 points a wave holds
    // for one point slot k are consecutive in x, so they lie in at most 9
    // Philox blocks of 8 consecutive points; a wave evaluates all 9*K blocks
    // it needs in one Philox call (one block per lane) per plane iteration
    // and passes the words through LDS.  Without room for them every lane
    // draws its own block.
    // With lanes to spare, one call covers the planes of two consecutive
    // iterations (NP = 2: half the Philox evaluations; BF16 four-step passes
    // at 512^3 143 -> 136 us per step).
    constexpr int NB = 9;
    constexpr bool SR_BATCH = Tr::sr && NB * K <= 64;
    constexpr int NP = (SR_BATCH && 2 * NB * K <= 64) ? 2 : 1;
    constexpr int NWAVE = NTH / 64;
    __shared__ uint32_t srw[SR_BATCH ? NWAVE : 1][SR_BATCH ? NP * NB * K : 1][4];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = (int)(t % (unsigned)ntx);
    const int rest = (int)(t / (unsigned)ntx);
    const int ty = rest % nty, tz = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY;         // region origin
    const bool ex0 = x0 == 0, ex1 = x0 + W0 >= nx, ey0 = y0 == 0, ey1 = y0 + H0 >= ny;
    // output tile: [ox0, ox1) x [oy0, oy1)
    const int ox0 = ex0 ? 1 : x0 + S, ox1 = ex1 ? nx - 1 : x0 + W0 - S;
    const int oy0 = ey0 ? 1 : y0 + S, oy1 = ey1 ? ny - 1 : y0 + H0 - S;
    const int zb = 1 + tz * zlen;                 // output planes zb .. ze-1
    const int ze = min(nz - 1, zb + zlen);
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;

    // This thread's region points: region coordinates (r, c), global (x, y).
    // Loads use addresses clamped into the grid (T) or onto a point the
    // level-1 region needs (Ci), so they need no branch; values at points
    // outside the grid are never used by an interior update.
    // FP64 (W0 = 64, every slot live): wave w holds the K consecutive region
    // rows K*w .. K*w+K-1 (one per point slot), so a point's y neighbours
    // inside that group come from the thread's own registers and only the
    // group's outer two from LDS (512^3 four-step passes 3% faster).  FP32
    // and BF16 run 1-7% slower that way (BF16 with stochastic rounding 13-18%:
    // it spills) and keep slot k on row w + k*NTH/64.
    constexpr bool kRowsY = DT == DIFF3D_F64 && W0 == 64 && A0 == K * NTH && K >= 2;
    int rr[K], cc[K], gx[K], gy[K];
    size_t base[K], cbase[K];
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
        const int lx = min(max(gx[k], 0), nx - 1), ly = min(max(gy[k], 0), ny - 1);
        base[k] = (size_t)lx + sy * (size_t)ly;
        const int cx = min(max(x0 + min(max(cc[k], 1), W0 - 2), 0), nx - 1);
        const int cy = min(max(y0 + min(max(rr[k], 1), H0 - 2), 0), ny - 1);
        cbase[k] = (size_t)cx + sy * (size_t)cy;
    }
    // point k belongs to the region of level s (border of s points removed
    // except on sides at the grid's boundary)
    auto in_level = [&](int k, int s) __attribute__((always_inline)) {
        return live[k] && (rr[k] >= s || ey0) && (rr[k] < H0 - s || ey1) && (cc[k] >= s || ex0) &&
               (cc[k] < W0 - s || ex1);
    };
    auto interior_xy = [&](int k) __attribute__((always_inline)) {
        return gx[k] >= 1 && gx[k] <= nx - 2 && gy[k] >= 1 && gy[k] <= ny - 2;
    };
    // The same conditions as a table of lane masks formed once outside the
    // plane loop (combined without short-circuiting): fewer scalar
    // instructions and no SGPR spills.  Measured faster for FP32 (1.5%),
    // BF16 with stochastic rounding (10%) and BF16 with round-to-nearest at
    // two workgroups per CU (8%).  FP64 takes the branch-free levels below
    // and needs neither form.
    constexpr bool kMaskTable = DT == DIFF3D_F32 || DT == DIFF3D_BF16 || DT == DIFF3D_BF16_RNE;
    // x neighbours by cross-lane moves: FP64 and FP32 with W0 = 64 (1.5%
    // faster at 512^3; the BF16 kernels, at 64 VGPRs, are slower with them)
    constexpr bool kLaneX = W0 == 64 && (DT == DIFF3D_F64 || DT == DIFF3D_F32);
    // Branch-free levels for FP64 (512^3 four-step passes 225 -> 217 us per
    // step); FP32 and BF16 run 2-8% slower that way and keep the per-level
    // tests.
    constexpr bool kFlat = DT == DIFF3D_F64;
    static_assert(!kFlat || kLaneX, "branch-free levels take x neighbours by cross-lane moves");
    bool act[S + 1][K];
#pragma unroll
    for (int s = 1; s <= S; ++s)
#pragma unroll
        for (int k = 0; k < K; ++k)
            act[s][k] = live[k] & ((rr[k] >= s) | ey0) & ((rr[k] < H0 - s) | ey1) & ((cc[k] >= s) | ex0) &
                        ((cc[k] < W0 - s) | ex1) & (gx[k] >= 1) & (gx[k] <= nx - 2) & (gy[k] >= 1) & (gy[k] <= ny - 2);
    // Branch-free levels: every lane computes every level, and the result is
    // kept only at interior grid points (elsewhere the level keeps the
    // input's value: the fixed boundary).  Points of a level outside that
    // level's region get values that no needed point reads (a level-s point
    // reads level s-1 only within distance one), so no per-level region
    // test is needed.  The staged planes carry one spare row above and below
    // the region (never written), so that the neighbour reads of the
    // region's outermost rows and columns stay inside the array; what they
    // read there is never used.
    bool ixy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ixy[k] = live[k] && interior_xy(k);
    bool otile[K];                                // on this workgroup's output tile
#pragma unroll
    for (int k = 0; k < K; ++k)
        otile[k] = (gx[k] >= ox0) & (gx[k] < ox1) & (gy[k] >= oy0) & (gy[k] < oy1);
    auto gidx = [&](int k, int z) __attribute__((always_inline)) {
        return (size_t)gx[k] + sy * gy[k] + sz * z;
    };
    auto rounding = [&](size_t i) __attribute__((always_inline)) -> uint32_t {
        uint32_t rnd = 0;
        if constexpr (Tr::sr) rnd = sr_word(sr_block(a.sr, i >> 3), (unsigned)(i & 7));
        return rnd;
    };
    auto load_T = [&](int z, C (&dst)[K]) __attribute__((always_inline)) {
        const size_t zo = sz * (size_t)min(max(z, 0), nz - 1);
#pragma unroll
        for (int k = 0; k < K; ++k) dst[k] = Tr::load(a.T[base[k] + zo]);
    };
    // Ci enters as lam*Ci, the product every update of that point forms
    auto load_Ci = [&](int z, C (&dst)[K]) __attribute__((always_inline)) {
        const size_t zo = sz * (size_t)min(max(z, 0), nz - 1);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const S_* p = a.Ci + cbase[k] + zo;
            dst[k] = Tr::load(NT ? __builtin_nontemporal_load(p) : *p);
        }
    };
    auto lam_ci = [&](C (&v)[K]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = a.lam * v[k];
    };
    auto stage = [&](int lev, int buf, const C (&src)[K]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (live[k]) lds[lev][buf][rr[k] + 1][cc[k]] = src[k];
    };

    // Registers: level-0 planes p-1 .. p+1; for levels 1 .. S-1 the two
    // planes below the one computed in this iteration (u[s-1][0] = z-1,
    // u[s-1][1] = z, the new plane z+1 is the level's fresh output); lam*Ci
    // at planes p, p-1, .., p-S+1 (ci[j] holds plane p+1-j); and two slots
    // each for the loads in flight (T planes p+2 and p+3, Ci planes p+1 and
    // p+2): a load is issued two plane iterations before its use.
    // With stochastically rounded BF16 the loads in flight and the Ci ring
    // hold raw stored values, two slots per 32-bit register, widened (and
    // multiplied by lam) where they are used: the kernel then fits 64 VGPRs
    // (two workgroups per CU) with its random-word exchange.  (Round to
    // nearest fits without, and is 3% slower with it.)
    constexpr bool PK = Tr::sr && K % 2 == 0;
    constexpr int KP = PK ? K / 2 : 1;
    C t0[3][K];
    C u[S > 1 ? S - 1 : 1][2][K];
    C ci[PK ? 1 : S + 1][PK ? 1 : K];
    C lt[PK ? 1 : 2][PK ? 1 : K], lc[PK ? 1 : 2][PK ? 1 : K];
    uint32_t cip[PK ? S + 1 : 1][KP], ltp[PK ? 2 : 1][KP], lcp[PK ? 2 : 1][KP];
    auto widen = [&](uint32_t w, int k) __attribute__((always_inline)) -> C {
        return __uint_as_float((k & 1) ? (w & 0xFFFF0000u) : (w << 16));
    };
    auto load_pairs = [&](const S_* f, const size_t* bs, int z, uint32_t (&dst)[KP]) __attribute__((always_inline)) {
        const size_t zo = sz * (size_t)min(max(z, 0), nz - 1);
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const uint32_t lo = (uint32_t)(uint16_t)f[bs[2 * j] + zo];
            const uint32_t hi = (uint32_t)(uint16_t)f[bs[2 * j + 1] + zo];
            dst[j] = lo | (hi << 16);
        }
    };
    // lam*Ci of slot k at the plane of level s
    auto lamci = [&](int s, int k) __attribute__((always_inline)) -> C {
        if constexpr (PK)
            return a.lam * widen(cip[s][k / 2], k);
        else
            return ci[s][k];
    };
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int s = 0; s < (S > 1 ? S - 1 : 1); ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i) u[s][i][k] = C(0);
        if constexpr (!PK) {
#pragma unroll
            for (int j = 0; j <= S; ++j) ci[j][k] = C(0);
        }
    }

    const int p0 = zb - S + 1;              // first plane of level 1
    const int plast = ze + S - 2;           // last plane of level 1
    load_T(p0 - 1, t0[0]);
    load_T(p0, t0[1]);
    load_T(p0 + 1, t0[2]);
    if constexpr (PK) {
#pragma unroll
        for (int j = 0; j <= S; ++j)
#pragma unroll
            for (int q = 0; q < KP; ++q) cip[j][q] = 0u;
        load_pairs(a.T, base, p0 + 2, ltp[0]);
        load_pairs(a.Ci, cbase, p0, cip[1]);
        load_pairs(a.Ci, cbase, p0 + 1, lcp[0]);
    } else {
        load_T(p0 + 2, lt[0]);
        load_Ci(p0, ci[1]);
        lam_ci(ci[1]);
        load_Ci(p0 + 1, lc[0]);
    }
    stage(0, 1, t0[1]);                     // plane p0 is read as "the previous iteration's" buffer

    // Stochastic rounding words.  A wave's 64 points of slot k are
    // consecutive in memory, from index i0 (lane 0's); lane l's point is
    // i0 + l, in block (i0 % 8 + l) / 8 after lane 0's, at position
    // (i0 % 8 + l) % 8.  Only i0 % 8 (wave-uniform) is kept per slot.
    int i0mod[NP][SR_BATCH ? K : 1];
    auto draw = [&](int p) __attribute__((always_inline)) {
        if constexpr (SR_BATCH) {
            const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
            size_t g0[NP][K];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int z = p + q - S + 1;     // the plane level S reaches in iteration p + q
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const size_t i0 = gidx(k, z) - (size_t)lane;
                    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)i0);
                    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(i0 >> 32));
                    const size_t u = ((size_t)hi << 32) | lo;
                    g0[q][k] = u >> 3;
                    i0mod[q][k] = (int)(lo & 7u);
                }
            }
            // lane L computes block b of slot k for plane q, L = (q*K + k)*NB + b
            if (lane < NP * NB * K) {
                const int qk = lane / NB, b = lane % NB;
                size_t g = 0;
#pragma unroll
                for (int q = 0; q < NP; ++q)
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (qk == q * K + k) g = g0[q][k] + (size_t)b;
                const u32x4 r = sr_block(a.sr, g);
                srw[wv][lane][0] = r.x;
                srw[wv][lane][1] = r.y;
                srw[wv][lane][2] = r.z;
                srw[wv][lane][3] = r.w;
            }
            __builtin_amdgcn_wave_barrier();   // the wave's LDS writes precede its reads (in order per wave)
        }
    };
    // q: which of the draw's planes (the iteration's parity when NP = 2)
    auto rounding_at = [&](int k, int z, int q) __attribute__((always_inline)) -> uint32_t {
        if constexpr (SR_BATCH) {
            const int wv = (int)(threadIdx.x >> 6);
            const int off = i0mod[q][k] + (int)(threadIdx.x & 63);
            const int j = off & 7;
            const uint32_t w = srw[wv][(q * K + k) * NB + (off >> 3)][j >> 1];
            return (j & 1) ? (w & 0xFFFF0000u) : (w << 16);
        } else {
            return rounding(gidx(k, z));
        }
    };

    // One plane iteration; PAR = (p - p0) & 1 selects the load slots.
    auto iteration = [&](auto par, int p) __attribute__((always_inline)) {
        constexpr int PAR = decltype(par)::value;
        constexpr int buf = PAR, rbuf = PAR ^ 1;
        if (NP == 1 || PAR == 0) draw(p);
        // 1. loads two planes ahead
        if constexpr (PK) {
            load_pairs(a.T, base, p + 3, ltp[PAR ^ 1]);
            load_pairs(a.Ci, cbase, p + 2, lcp[PAR ^ 1]);
        } else {
            load_T(p + 3, lt[PAR ^ 1]);
            load_Ci(p + 2, lc[PAR ^ 1]);
        }
        lds_barrier();
        // 2. level 0, plane p+1, for level 1 of the next iteration
        stage(0, buf, t0[2]);
        // 3. levels 1 .. S at planes p, p-1, .., p-S+1
        C prev[K];                          // level s-1 at plane z+1 (fresh output)
#pragma unroll
        for (int k = 0; k < K; ++k) prev[k] = t0[2][k];
        // level s-1 of slot j at the plane level s is computed at
        auto centre = [&](int s, int j) __attribute__((always_inline)) -> C {
            return s == 1 ? t0[1][j] : u[s - 2][1][j];
        };
#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int z = p - s + 1;
            const bool zact = z >= zb - (S - s) && z < ze + (S - s) && z >= 1 && z <= nz - 2;
            C out[K];
            if constexpr (kFlat) {
                const bool zin = z >= 1 && z <= nz - 2;
                const bool zout = z >= zb && z < ze;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const C zm = s == 1 ? t0[0][k] : u[s - 2][0][k];
                    const C ce = s == 1 ? t0[1][k] : u[s - 2][1][k];
                    const C zp = prev[k];
                    C xm, xp;
                    if constexpr (kLaneX) {
                        xm = lane_shift<C, false>(ce);
                        xp = lane_shift<C, true>(ce);
                    } else {
                        xm = (&lds[s - 1][rbuf][rr[k] + 1][0])[cc[k] - 1];
                        xp = (&lds[s - 1][rbuf][rr[k] + 1][0])[cc[k] + 1];
                    }
                    const C ym = (kRowsY && k > 0) ? centre(s, k - 1) : lds[s - 1][rbuf][rr[k]][cc[k]];
                    const C yp = (kRowsY && k < K - 1) ? centre(s, k + 1) : lds[s - 1][rbuf][rr[k] + 2][cc[k]];
                    const C w = stencil_point_lc<DT>(ce, xm, xp, ym, yp, zm, zp, lamci(s, k), a);
                    if (s < S) {
                        out[k] = (zin && ixy[k]) ? w : ce;
                    } else if (zout && otile[k]) {
                        const S_ o = Tr::store(w, rounding_at(k, z, NP == 2 ? PAR : 0));
                        if (NT)
                            __builtin_nontemporal_store(o, a.T2 + gidx(k, z));
                        else
                            a.T2[gidx(k, z)] = o;
                    }
                }
            } else
#pragma unroll
            for (int k = 0; k < K; ++k) {
                // level s-1 at planes z-1, z, z+1 for this point
                const C zm = s == 1 ? t0[0][k] : u[s - 2][0][k];
                const C ce = s == 1 ? t0[1][k] : u[s - 2][1][k];
                const C zp = prev[k];
                C v = ce;
                // FP64/FP32 with whole region rows per wave: the x neighbours
                // are the adjacent lanes' centre values (cross-lane moves,
                // outside the branch so every lane takes part)
                C xmd = ce, xpd = ce;
                if constexpr (kLaneX) {
                    xmd = lane_shift<C, false>(ce);
                    xpd = lane_shift<C, true>(ce);
                }
                if (zact && (kMaskTable ? act[s][k] : in_level(k, s) && interior_xy(k))) {
                    const C xm = kLaneX ? xmd : lds[s - 1][rbuf][rr[k] + 1][cc[k] - 1];
                    const C xp = kLaneX ? xpd : lds[s - 1][rbuf][rr[k] + 1][cc[k] + 1];
                    const C ym = (kRowsY && k > 0) ? centre(s, k - 1) : lds[s - 1][rbuf][rr[k]][cc[k]];
                    const C yp = (kRowsY && k < K - 1) ? centre(s, k + 1) : lds[s - 1][rbuf][rr[k] + 2][cc[k]];
                    const C w = stencil_point_lc<DT>(ce, xm, xp, ym, yp, zm, zp, lamci(s, k), a);
                    if (s < S) {
                        v = w;
                    } else if (z >= zb && z < ze &&
                               (kMaskTable ? otile[k]
                                           : gx[k] >= ox0 && gx[k] < ox1 && gy[k] >= oy0 && gy[k] < oy1)) {
                        const S_ o = Tr::store(w, rounding_at(k, z, NP == 2 ? PAR : 0));
                        if (NT)
                            __builtin_nontemporal_store(o, a.T2 + gidx(k, z));
                        else
                            a.T2[gidx(k, z)] = o;
                    }
                }
                out[k] = v;
            }
            if (s > 1) {
                // level s-1's history moves up by one plane
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    u[s - 2][0][k] = u[s - 2][1][k];
                    u[s - 2][1][k] = prev[k];
                }
            }
            if (s < S) {
                stage(s, buf, out);
#pragma unroll
                for (int k = 0; k < K; ++k) prev[k] = out[k];
            }
        }
        if constexpr (SR_BATCH) __builtin_amdgcn_wave_barrier();   // reads done before a later draw writes
        // 4. shift level 0 and Ci; the older slot (plane p+2, Ci plane p+1) enters
#pragma unroll
        for (int k = 0; k < K; ++k) {
            t0[0][k] = t0[1][k];
            t0[1][k] = t0[2][k];
            if constexpr (PK) {
                t0[2][k] = widen(ltp[PAR][k / 2], k);
            } else {
                t0[2][k] = lt[PAR][k];
#pragma unroll
                for (int j = S; j >= 2; --j) ci[j][k] = ci[j - 1][k];
                ci[1][k] = a.lam * lc[PAR][k];
            }
        }
        if constexpr (PK) {
#pragma unroll
            for (int q = 0; q < KP; ++q) {
#pragma unroll
                for (int j = S; j >= 2; --j) cip[j][q] = cip[j - 1][q];
                cip[1][q] = lcp[PAR][q];
            }
        }
    };
    for (int p = p0; p <= plast; p += 2) {
        iteration(std::integral_constant<int, 0>{}, p);
        if (p + 1 <= plast) iteration(std::integral_constant<int, 1>{}, p + 1);
    }
}

}  // namespace diff3d
