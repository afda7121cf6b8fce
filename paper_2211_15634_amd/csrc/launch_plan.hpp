// Launch planning shared by the kernels: tiles over x-y, z-chunks, rounds
// of resident workgroups, tile configuration keys and the caller's
// overrides of them.
#pragma once

#include <atomic>

#include "host_common.hpp"

namespace diff3d {
namespace {

// z-march launch plan: tiles of TX x TY over x-y, chunks of zlen planes along z
struct ZPlan {
    int ntx, nty, zlen, nchunks;
    unsigned blocks;
};

// zdef: preferred planes per chunk (long chunks amortise the two extra
// planes a chunk reads); the chunk is shortened until the launch has at
// least kMinBlocks workgroups.
constexpr long kMinBlocks = 512;

inline ZPlan plan_tiles(int nx, int ny, int nzout, int TX, int TY, int zlen_req, int zdef, long min_blocks = kMinBlocks)
{
    ZPlan p;
    p.ntx = (nx + TX - 1) / TX;
    p.nty = (ny + TY - 1) / TY;
    const long tiles = (long)p.ntx * p.nty;
    int zlen = zlen_req;
    if (zlen <= 0) {
        long nch = (nzout + zdef - 1) / zdef;
        const long need = (min_blocks + tiles - 1) / tiles;
        if (nch < need) nch = need;
        zlen = (int)((nzout + nch - 1) / nch);
        if (zlen < 4) zlen = 4;
    }
    if (zlen > nzout) zlen = nzout;
    p.zlen = zlen;
    p.nchunks = (nzout + zlen - 1) / zlen;
    p.blocks = (unsigned)(tiles * p.nchunks);
    return p;
}

// A tile configuration: V points per lane along x, R rows per thread, NW
// waves per workgroup, NT non-temporal stream accesses.
struct ZKey {
    int V, R, NW, NT;
};

inline bool key_eq(const ZKey& a, int V, int R, int NW, int NT)
{
    return a.V == V && a.R == R && a.NW == NW && a.NT == NT;
}

// The override of a tile (V, R, NW, NT) family, or the default.
inline ZKey zkey_of(const diff3d_tile& t, const ZKey& dflt)
{
    return tile_set(t) ? ZKey{t.p[0], t.p[1], t.p[2], t.p[3]} : dflt;
}

// Vector width V is usable when rows start on V-element boundaries and all
// three fields are 16-byte aligned.
template <class S>
inline bool vec_ok(int nx, int V, const void* p0, const void* p1, const void* p2)
{
    return V == 1 || (nx % V == 0 && (uintptr_t)p0 % 16 == 0 && (uintptr_t)p1 % 16 == 0 && (uintptr_t)p2 % 16 == 0);
}

// S-step (temporal-blocked) configurations: S steps, W0 x H0 region per
// workgroup (output tile (W0-2S) x (H0-2S)), NTH threads, NT non-temporal.
struct SKey {
    int S, W0, H0, NTH, NT;
};

inline bool skey_eq(const SKey& a, int S, int W0, int H0, int NTH, int NT)
{
    return a.S == S && a.W0 == W0 && a.H0 == H0 && a.NTH == NTH && a.NT == NT;
}

// The override of the S-step or fused reverse kernel for passes of S
// steps (a set override names the pass length it applies to), or the
// default; and the z-chunk length for such passes.
inline SKey skey_of(const diff3d_tile& t, int S, const SKey& dflt)
{
    if (tile_set(t) && t.steps == S) return SKey{S, t.p[0], t.p[1], t.p[2], t.p[3]};
    return dflt;
}

inline int szlen_of(const diff3d_tile& t, int S)
{
    return (t.steps == 0 || t.steps == S) ? t.zlen : 0;
}

// Workgroups of `kernel` (nth threads) resident at once on the current
// device, from the occupancy calculator.  Cached per kernel as one atomic
// word, (device + 1) << 40 | slots, so concurrent callers read a consistent
// pair (a miss recomputes the same value).
template <class F>
long resident_slots(F kernel, int nth, std::atomic<long long>& cache)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    const long long c = cache.load(std::memory_order_relaxed);
    if ((c >> 40) == (long long)dev + 1) return (long)(c & ((1LL << 40) - 1));
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nth, 0) != hipSuccess) per_cu = 1;
    const long slots = (long)max(cus, 1) * max(per_cu, 1);
    cache.store(((long long)dev + 1) << 40 | slots, std::memory_order_relaxed);
    return slots;
}

// Tiles along an axis of n points for regions of width w placed every t
// points from the grid's edge, the last region reaching the far edge.
inline int edge_tiles(int n, int w, int t) { return n <= w ? 1 : (n - w + t - 1) / t + 1; }

// z-chunking for kernels with few resident workgroups: equal-length blocks
// run in rounds of `slots`, so pick the chunk count that minimises
// rounds x (planes per chunk + `extra` halo planes), among counts that fill
// at least 90% of the device (when the grid allows it).
inline ZPlan plan_rounds(int ntx, int nty, int nzout, int zlen_req, int extra, long slots)
{
    ZPlan p;
    p.ntx = ntx;
    p.nty = nty;
    const long tiles = (long)p.ntx * p.nty;
    int zlen = zlen_req > 0 ? min(zlen_req, nzout) : nzout;
    if (zlen_req <= 0) {
        long best = -1;
        const bool can_fill = tiles * nzout >= slots;
        for (int nch = 1; nch <= nzout && nch <= 1024; ++nch) {
            const int zl = (nzout + nch - 1) / nch;
            const long blocks = tiles * ((nzout + zl - 1) / zl);
            if (can_fill && blocks * 10 < slots * 9) continue;
            const long cost = ((blocks + slots - 1) / slots) * (long)(zl + extra);
            if (best < 0 || cost < best) {
                best = cost;
                zlen = zl;
            }
        }
    }
    p.zlen = zlen;
    p.nchunks = (nzout + zlen - 1) / zlen;
    p.blocks = (unsigned)(tiles * p.nchunks);
    return p;
}

}  // namespace
}  // namespace diff3d
