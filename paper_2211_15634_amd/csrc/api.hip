// C ABI of the diff3d library: argument validation, kernel selection and
// launch, the time loop with the buffer swap, and the checkpointed reverse
// sweep.  Everything is enqueued on the caller's stream; no device memory is
// allocated here.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "adjoint_kernels.hpp"
#include "common.hpp"
#include "diff3d.h"
#include "rev_kernels.hpp"
#include "step_kernels.hpp"
#include "tb_kernels.hpp"
#include "util_kernels.hpp"

using namespace diff3d;

namespace {

int g_kernel = DIFF3D_KERNEL_AUTO;
int g_pass_steps = 0;   // steps per pass of the S-step kernel in diff3d_run (0 = dtype default)
uint64_t g_sr_seed = 0x5EEDu;
uint64_t g_sr_step = 0;

constexpr size_t kMaxPoints = (size_t)1 << 40;

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int hip_status()
{
    return hipGetLastError() == hipSuccess ? DIFF3D_OK : DIFF3D_EHIP;
}

inline bool known_dtype(int dt) { return dt >= DIFF3D_F64 && dt <= DIFF3D_BF16_RNE; }

inline size_t elem_size(int dt)
{
    switch (dt) {
    case DIFF3D_F64: return 8;
    case DIFF3D_F32: return 4;
    case DIFF3D_BF16:
    case DIFF3D_BF16_RNE: return 2;
    default: return 0;
    }
}

int check_grid(int nx, int ny, int nz)
{
    if (nx < 3 || ny < 3 || nz < 3) return DIFF3D_EINVAL;
    if ((size_t)nx * (size_t)ny * (size_t)nz >= kMaxPoints) return DIFF3D_EINVAL;
    return DIFF3D_OK;
}

inline size_t npoints(int nx, int ny, int nz) { return (size_t)nx * ny * nz; }

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

int env_int(const char* name, int dflt)
{
    const char* s = getenv(name);
    if (!s || !*s) return dflt;
    return atoi(s);
}

// ------------------------------------------------------------------ forward
template <int DT>
StepArgs<DT> make_step_args(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                            double rdx, double rdy, double rdz, uint64_t step_index)
{
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    StepArgs<DT> a;
    a.T2 = static_cast<S*>(T2);
    a.T = static_cast<const S*>(T);
    a.Ci = static_cast<const S*>(Ci);
    a.Tmid = nullptr;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.lam = (C)lam;
    a.dt = (C)dt;
    a.cx = (C)(rdx * rdx);
    a.cy = (C)(rdy * rdy);
    a.cz = (C)(rdz * rdz);
    a.sr.k0 = (uint32_t)g_sr_seed;
    a.sr.k1 = (uint32_t)(g_sr_seed >> 32);
    a.sr.s0 = (uint32_t)step_index;
    a.sr.s1 = (uint32_t)(step_index >> 32);
    return a;
}

template <int DT>
int launch_naive(const StepArgs<DT>& a, hipStream_t st)
{
    dim3 grid((unsigned)((a.nx - 2 + 63) / 64), (unsigned)((a.ny - 2 + 3) / 4), (unsigned)min(a.nz - 2, 65535));
    step_naive<DT><<<grid, 256, 0, st>>>(a);
    return hip_status();
}

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

// Configuration override "V,R,NW[,NT]" from the environment (tuning only).
inline bool env_key(const char* name, ZKey& k)
{
    const char* s = getenv(name);
    if (!s || !*s) return false;
    ZKey r{0, 0, 0, 0};
    const int got = sscanf(s, "%d,%d,%d,%d", &r.V, &r.R, &r.NW, &r.NT);
    if (got < 3) return false;
    if (got == 3) r.NT = 0;
    k = r;
    return true;
}

// Instantiated forward configurations per storage size (V*sizeof(S) <= 16).
#define DIFF3D_FWD_CFGS_8(X) X(1, 4, 4, 0) X(1, 8, 4, 0) X(1, 4, 8, 0) X(2, 4, 4, 0) X(2, 8, 4, 0) X(2, 2, 8, 0) \
    X(2, 4, 8, 0) X(2, 4, 4, 1) X(2, 8, 4, 1) X(2, 4, 8, 1)
#define DIFF3D_FWD_CFGS_4(X) X(1, 4, 4, 0) X(2, 4, 4, 0) X(2, 8, 4, 0) X(2, 4, 8, 0) X(4, 2, 4, 0) X(4, 4, 4, 0) \
    X(4, 2, 8, 0) X(4, 2, 8, 1) X(4, 4, 4, 1) X(2, 8, 4, 1)
#define DIFF3D_FWD_CFGS_2(X) X(1, 4, 4, 0) X(2, 4, 4, 0) X(2, 8, 4, 0) X(4, 2, 4, 0) X(4, 4, 4, 0) X(4, 2, 8, 0) \
    X(4, 1, 8, 0) X(8, 1, 8, 0) X(8, 2, 4, 0) X(4, 4, 4, 1) X(2, 8, 4, 1) X(4, 2, 8, 1)

template <int DT>
struct FwdDefaults;
template <> struct FwdDefaults<DIFF3D_F64> { static constexpr ZKey wide{2, 4, 4, 1}; static constexpr int zdef = 128; };
template <> struct FwdDefaults<DIFF3D_F32> { static constexpr ZKey wide{4, 4, 4, 1}; static constexpr int zdef = 32; };
template <> struct FwdDefaults<DIFF3D_BF16> { static constexpr ZKey wide{4, 1, 8, 0}; static constexpr int zdef = 32; };
template <> struct FwdDefaults<DIFF3D_BF16_RNE> { static constexpr ZKey wide{4, 1, 8, 0}; static constexpr int zdef = 64; };
constexpr ZKey kNarrow{1, 4, 4, 0};

template <int DT, int V, int R, int NW, int NT>
int launch_zmarch_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz - 2, 64 * V, R * NW, zlen_req, zdef);
    step_zmarch<DT, V, R, NW, NT != 0><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

// Vector width V is usable when rows start on V-element boundaries and all
// three fields are 16-byte aligned.
template <class S>
inline bool vec_ok(int nx, int V, const void* p0, const void* p1, const void* p2)
{
    return V == 1 || (nx % V == 0 && (uintptr_t)p0 % 16 == 0 && (uintptr_t)p1 % 16 == 0 && (uintptr_t)p2 % 16 == 0);
}

template <int DT>
int launch_zmarch(const StepArgs<DT>& a, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    ZKey k = FwdDefaults<DT>::wide;
    env_key("DIFF3D_ZCFG", k);
    if (env_int("DIFF3D_NARROW", 0) || !vec_ok<S>(a.nx, k.V, a.T, a.T2, a.Ci)) k = kNarrow;
    const int zlen = env_int("DIFF3D_ZLEN", 0);
    const int zdef = FwdDefaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw, nt) \
    if (key_eq(k, v, r, nw, nt)) return launch_zmarch_cfg<DT, v, r, nw, nt>(a, st, zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_FWD_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(S) == 4) {
        DIFF3D_FWD_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_FWD_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;   // configuration not instantiated (tuning override only)
}

// Two-step (temporal-blocked) configurations.
#define DIFF3D_TB2_CFGS_8(X) X(1, 4, 4, 1) X(2, 2, 4, 1) X(1, 2, 8, 1) X(2, 2, 8, 1) X(2, 1, 8, 1) X(1, 4, 8, 1)
#define DIFF3D_TB2_CFGS_4(X) X(1, 4, 4, 1) X(2, 2, 4, 1) X(4, 1, 8, 1) X(2, 2, 8, 1) X(4, 2, 4, 1) X(2, 1, 8, 1)
#define DIFF3D_TB2_CFGS_2(X) X(1, 4, 4, 1) X(4, 1, 8, 1) X(4, 2, 4, 1) X(8, 1, 8, 1) X(2, 2, 8, 1) X(8, 1, 4, 1)

template <int DT>
struct Tb2Defaults;
template <> struct Tb2Defaults<DIFF3D_F64> { static constexpr ZKey wide{2, 2, 8, 1}; static constexpr int zdef = 256; };
template <> struct Tb2Defaults<DIFF3D_F32> { static constexpr ZKey wide{2, 2, 8, 1}; static constexpr int zdef = 128; };
template <> struct Tb2Defaults<DIFF3D_BF16> { static constexpr ZKey wide{4, 2, 4, 1}; static constexpr int zdef = 128; };
template <> struct Tb2Defaults<DIFF3D_BF16_RNE> { static constexpr ZKey wide{4, 2, 4, 1}; static constexpr int zdef = 128; };
constexpr ZKey kNarrowTb2{1, 4, 4, 1};

template <int DT, int V, int R, int NW, int NT, bool MID>
int launch_tb2_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz - 2, 64 * V, R * NW, zlen_req, zdef);
    step_tb2<DT, V, R, NW, NT != 0, MID><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT, bool MID>
int launch_tb2(const StepArgs<DT>& a, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    ZKey k = Tb2Defaults<DT>::wide;
    env_key("DIFF3D_TCFG", k);
    if (env_int("DIFF3D_NARROW", 0) || !vec_ok<S>(a.nx, k.V, a.T, a.T2, a.Ci)) k = kNarrowTb2;
    const int zlen = env_int("DIFF3D_TZLEN", 0);
    const int zdef = Tb2Defaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw, nt) \
    if (key_eq(k, v, r, nw, nt)) return launch_tb2_cfg<DT, v, r, nw, nt, MID>(a, st, zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_TB2_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(S) == 4) {
        DIFF3D_TB2_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_TB2_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

// Two steps T -> T2 (T^{k+2}); SR step indices step_index and step_index+1.
template <int DT>
int launch_pair(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index);
    return launch_tb2<DT, false>(a, st);
}

// Two steps T -> Tmid (T^{k+1}) and T2 (T^{k+2}), interior points of both.
template <int DT>
int launch_pair_mid(void* T2, void* Tmid, const void* T, const void* Ci, int nx, int ny, int nz, double lam,
                    double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, 0);
    a.Tmid = static_cast<typename Traits<DT>::S*>(Tmid);
    return launch_tb2<DT, true>(a, st);
}

int pair_mid_dispatch(int dtype, void* T2, void* Tmid, const void* T, const void* Ci, int nx, int ny, int nz,
                      double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_pair_mid<DIFF3D_F64>(T2, Tmid, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    case DIFF3D_F32: return launch_pair_mid<DIFF3D_F32>(T2, Tmid, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    default: return DIFF3D_EDTYPE;
    }
}

int pair_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_pair<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_F32: return launch_pair<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16: return launch_pair<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16_RNE:
        return launch_pair<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    default: return DIFF3D_EDTYPE;
    }
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

// Override "W0,H0,NTH[,NT]" for the S-step kernel from the environment
// (tuning only; S is the pass length).
inline bool env_skey(const char* name, SKey& k)
{
    const char* s = getenv(name);
    if (!s || !*s) return false;
    SKey r{k.S, 0, 0, 0, 1};
    const int got = sscanf(s, "%d,%d,%d,%d", &r.W0, &r.H0, &r.NTH, &r.NT);
    if (got < 3) return false;
    k = r;
    return true;
}

#define DIFF3D_TBS_CFGS_8(X) X(2, 64, 16, 512, 1) X(2, 64, 32, 512, 0) X(3, 64, 32, 512, 0) X(3, 64, 32, 1024, 0) \
    X(4, 64, 32, 512, 0) X(4, 64, 32, 1024, 0)
#define DIFF3D_TBS_CFGS_4(X) X(2, 64, 32, 512, 1) X(2, 64, 64, 1024, 0) X(3, 64, 32, 512, 0) X(3, 128, 32, 1024, 0) \
    X(4, 64, 32, 512, 0) X(4, 64, 48, 768, 0)
#define DIFF3D_TBS_CFGS_2(X) X(2, 64, 32, 512, 1) X(2, 64, 32, 1024, 0) X(3, 64, 32, 1024, 0) X(4, 64, 32, 1024, 0)

template <int DT>
struct TbsDefaults;
template <> struct TbsDefaults<DIFF3D_F64> {
    static constexpr int S = 4;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 512, 0}, {3, 64, 32, 512, 0}, {4, 64, 32, 1024, 0}};
};
template <> struct TbsDefaults<DIFF3D_F32> {
    static constexpr int S = 3;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 64, 1024, 0}, {3, 128, 32, 1024, 0}, {4, 64, 48, 768, 0}};
};
template <> struct TbsDefaults<DIFF3D_BF16> {
    static constexpr int S = 3;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 1024, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};
template <> struct TbsDefaults<DIFF3D_BF16_RNE> {
    static constexpr int S = 2;
    static constexpr SKey key[5] = {{0}, {0}, {2, 64, 32, 1024, 0}, {3, 64, 32, 1024, 0}, {4, 64, 32, 1024, 0}};
};

// Workgroups of `kernel` (nth threads) resident at once on the current
// device, from the occupancy calculator; cached per kernel and device.
template <class F>
long resident_slots(F kernel, int nth, int& cached_dev, long& cached)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev != cached_dev) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nth, 0) != hipSuccess) per_cu = 1;
        cached = (long)max(cus, 1) * max(per_cu, 1);
        cached_dev = dev;
    }
    return cached;
}

// Tiles along an axis of n points for regions of width w placed every t
// points from the grid's edge, the last region reaching the far edge.
inline int edge_tiles(int n, int w, int t) { return n <= w ? 1 : (n - w + t - 1) / t + 1; }

// z-chunking for kernels with few resident workgroups: equal-length blocks
// run in rounds of `slots`, so pick the chunk count that minimises
// rounds x (planes per chunk + `extra` halo planes), among counts that fill
// the device (when the grid allows it).
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
            if (can_fill && blocks < slots) continue;
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

template <int DT, int S, int W0, int H0, int NTH, int NT>
int launch_tbs_cfg(const StepArgs<DT>& a, hipStream_t st, int zlen_req)
{
    static int cdev = -1;
    static long cslots = 0;
    auto kernel = step_tbs<DT, S, W0, H0, NTH, NT != 0>;
    const long slots = resident_slots(kernel, NTH, cdev, cslots);
    const ZPlan p = plan_rounds(edge_tiles(a.nx, W0, W0 - 2 * S), edge_tiles(a.ny, H0, H0 - 2 * S), a.nz - 2,
                                zlen_req, 2 * S, slots);
    kernel<<<p.blocks, NTH, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

// S steps T -> T2 in one pass (2 <= S <= DIFF3D_MAX_PASS_STEPS).
template <int DT>
int launch_tbs(const StepArgs<DT>& a, int nsteps, hipStream_t st)
{
    using Sz = typename Traits<DT>::S;
    if (nsteps < 2 || nsteps > DIFF3D_MAX_PASS_STEPS) return DIFF3D_EINVAL;
    SKey k = TbsDefaults<DT>::key[nsteps];
    env_skey("DIFF3D_SCFG", k);
    const int zlen = env_int("DIFF3D_SZLEN", 0);
#define DIFF3D_TRY(s, w0, h0, nth, nt) \
    if (skey_eq(k, s, w0, h0, nth, nt)) return launch_tbs_cfg<DT, s, w0, h0, nth, nt>(a, st, zlen);
    if constexpr (sizeof(Sz) == 8) {
        DIFF3D_TBS_CFGS_8(DIFF3D_TRY)
    } else if constexpr (sizeof(Sz) == 4) {
        DIFF3D_TBS_CFGS_4(DIFF3D_TRY)
    } else {
        DIFF3D_TBS_CFGS_2(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

template <int DT>
int launch_multi(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, int nsteps, uint64_t step_index, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index);
    return launch_tbs<DT>(a, nsteps, st);
}

int multi_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                   double rdx, double rdy, double rdz, int nsteps, uint64_t step_index, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_multi<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    case DIFF3D_F32:
        return launch_multi<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    case DIFF3D_BF16:
        return launch_multi<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    case DIFF3D_BF16_RNE:
        return launch_multi<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, step_index, st);
    default: return DIFF3D_EDTYPE;
    }
}

template <int DT>
int launch_step(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    const StepArgs<DT> a = make_step_args<DT>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index);
    if (g_kernel == DIFF3D_KERNEL_NAIVE) return launch_naive<DT>(a, st);
    return launch_zmarch<DT>(a, st);
}

int step_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, uint64_t step_index, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_step<DIFF3D_F64>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_F32: return launch_step<DIFF3D_F32>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16: return launch_step<DIFF3D_BF16>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    case DIFF3D_BF16_RNE:
        return launch_step<DIFF3D_BF16_RNE>(T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    default: return DIFF3D_EDTYPE;
    }
}

// n steps in one pass: a single step, the two-step kernel, or the S-step
// kernel (always for n >= 3; for n = 2 when it is selected, and under AUTO
// for the BF16 forms, where it is faster: 140 vs 340 us per step at 512^3
// with round-to-nearest, 305 vs 584 with stochastic rounding; for FP64 and
// FP32 the two-step kernel is faster).
int pass_dispatch(int dtype, void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt,
                  double rdx, double rdy, double rdz, int n, uint64_t step_index, hipStream_t st)
{
    if (n == 1) return step_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    const bool tbs2 = g_kernel == DIFF3D_KERNEL_TBS ||
                      (g_kernel == DIFF3D_KERNEL_AUTO && (dtype == DIFF3D_BF16 || dtype == DIFF3D_BF16_RNE));
    if (n == 2 && !tbs2)
        return pair_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, step_index, st);
    return multi_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, n, step_index, st);
}

int tbs_default_steps(int dtype)
{
    switch (dtype) {
    case DIFF3D_F64: return TbsDefaults<DIFF3D_F64>::S;
    case DIFF3D_F32: return TbsDefaults<DIFF3D_F32>::S;
    case DIFF3D_BF16: return TbsDefaults<DIFF3D_BF16>::S;
    default: return TbsDefaults<DIFF3D_BF16_RNE>::S;
    }
}

// Steps per pass of diff3d_run for the selected kernel.  AUTO uses the
// S-step kernel's measured best pass length: 4 for FP64, 3 for FP32, 2 for
// BF16 with round-to-nearest (bound by ALU work more than bytes: 140 us per
// step against 207 for single steps at 512^3), 3 for BF16 with stochastic
// rounding (bound by the Philox draws: 281 against 300 us).
int run_pass_steps(int dtype)
{
    switch (g_kernel) {
    case DIFF3D_KERNEL_NAIVE:
    case DIFF3D_KERNEL_ZMARCH: return 1;
    case DIFF3D_KERNEL_TB2: return 2;
    case DIFF3D_KERNEL_TBS: return g_pass_steps ? g_pass_steps : tbs_default_steps(dtype);
    default: return tbs_default_steps(dtype);
    }
}

// ------------------------------------------------------------------ helpers
int copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return DIFF3D_OK;
    if ((uintptr_t)dst % 16 || (uintptr_t)src % 16) {
        // fields are at least 2-byte aligned: move 16-bit words
        const size_t n2 = bytes / 2;
        size_t blocks = (n2 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        copy_u16<<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint16_t*>(dst), static_cast<const uint16_t*>(src), n2);
        return hip_status();
    }
    const size_t n16 = bytes / 16, tail = bytes % 16;
    if (n16) {
        const size_t per = 256 * kCopyUnroll;
        const size_t blocks = (n16 + per - 1) / per;   // < 2^31 for any field below 2^40 points
        copy16<<<(unsigned)blocks, 256, 0, st>>>(static_cast<u32v4*>(dst), static_cast<const u32v4*>(src), n16);
    }
    if (tail)
        copy_tail<<<1, 64, 0, st>>>(static_cast<unsigned char*>(dst) + n16 * 16,
                                    static_cast<const unsigned char*>(src) + n16 * 16, tail);
    return hip_status();
}

int zero_bytes(void* p, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return DIFF3D_OK;
    const size_t n16 = bytes / 16, tail = bytes % 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    fill_zero<<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint4*>(p), n16,
                                                 static_cast<unsigned char*>(p) + n16 * 16, tail);
    return hip_status();
}

int boundary_dispatch(int dtype, void* dst, const void* src, int nx, int ny, int nz, hipStream_t st)
{
    const size_t total = 2 * ((size_t)nx * ny + (size_t)nx * nz + (size_t)ny * nz);
    size_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    switch (elem_size(dtype)) {
    case 8:
        boundary_copy<uint64_t><<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint64_t*>(dst),
                                                                   static_cast<const uint64_t*>(src), nx, ny, nz);
        break;
    case 4:
        boundary_copy<uint32_t><<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint32_t*>(dst),
                                                                   static_cast<const uint32_t*>(src), nx, ny, nz);
        break;
    case 2:
        boundary_copy<uint16_t><<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint16_t*>(dst),
                                                                   static_cast<const uint16_t*>(src), nx, ny, nz);
        break;
    default: return DIFF3D_EDTYPE;
    }
    return hip_status();
}

// The time loop of Fig. 1 on two buffers; checkpoint field j-1 receives
// T_{j*C} for every j >= 1 with j*C <= klast.  With want_result the final
// state is left in T.
int run_loop(int dtype, void* T, void* T2, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
             double rdy, double rdz, int nt, hipStream_t st, void* ckpt, int C, size_t field_stride, int klast,
             bool want_result)
{
    int rc = boundary_dispatch(dtype, T2, T, nx, ny, nz, st);
    if (rc) return rc;
    const size_t fbytes = npoints(nx, ny, nz) * elem_size(dtype);
    void* a = T;
    void* b = T2;
    const int P = run_pass_steps(dtype);
    for (int it = 0; it < nt;) {
        // P steps in one pass, shortened at the end and where a checkpoint
        // falls on a state inside the pass
        int n = min(P, nt - it);
        if (ckpt) {
            const int next = (it / C + 1) * C;   // next checkpointed step
            if (next <= klast && next - it < n) n = next - it;
        }
        rc = pass_dispatch(dtype, b, a, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, n, g_sr_step + (uint64_t)it, st);
        if (rc) return rc;
        void* s = a;
        a = b;
        b = s;
        it += n;
        const int k = it;
        if (ckpt && k % C == 0 && k <= klast) {
            rc = copy_bytes(static_cast<char*>(ckpt) + (size_t)(k / C - 1) * field_stride, a, fbytes, st);
            if (rc) return rc;
        }
    }
    g_sr_step += (uint64_t)nt;
    if (want_result && a != T) return copy_bytes(T, a, fbytes, st);
    return DIFF3D_OK;
}

// ------------------------------------------------------------------ adjoint
template <int DT>
AdjArgs<DT> make_adj_args(void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx, int ny,
                          int nz, double lam, double dt, double rdx, double rdy, double rdz)
{
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    AdjArgs<DT> a;
    a.lout = static_cast<S*>(lout);
    a.lin = static_cast<const S*>(lin);
    a.Ci = static_cast<const S*>(Ci);
    a.Tk = static_cast<const S*>(Tk);
    a.Tk1 = nullptr;
    a.gCi = static_cast<S*>(gCi);
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.dtlam = (C)dt * (C)lam;
    a.cx = (C)(rdx * rdx);
    a.cy = (C)(rdy * rdy);
    a.cz = (C)(rdz * rdz);
    return a;
}

#define DIFF3D_ADJ_CFGS_8(X) X(1, 4, 4) X(1, 2, 4) X(1, 2, 8) X(1, 4, 8) X(2, 2, 4) X(2, 1, 8) X(2, 2, 8)
#define DIFF3D_ADJ_CFGS_4(X) X(1, 4, 4) X(1, 2, 4) X(1, 2, 8) X(2, 2, 4) X(2, 2, 8) X(4, 1, 4) X(4, 1, 8) X(2, 1, 8)

template <int DT>
struct AdjDefaults;
template <> struct AdjDefaults<DIFF3D_F64> { static constexpr ZKey wide{2, 1, 8, 0}; static constexpr int zdef = 32; };
template <> struct AdjDefaults<DIFF3D_F32> { static constexpr ZKey wide{4, 1, 8, 0}; static constexpr int zdef = 16; };

template <int DT, int V, int R, int NW>
int launch_adj_cfg(const AdjArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz, 64 * V, R * NW, zlen_req, zdef);
    adj_zmarch<DT, V, R, NW><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT>
int launch_adj(void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx, int ny, int nz,
               double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    const AdjArgs<DT> a = make_adj_args<DT>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz);
    if (g_kernel == DIFF3D_KERNEL_NAIVE) {
        dim3 grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4), (unsigned)min(nz, 65535));
        adj_naive<DT><<<grid, 256, 0, st>>>(a);
        return hip_status();
    }
    ZKey k = AdjDefaults<DT>::wide;
    env_key("DIFF3D_ACFG", k);
    const bool aligned = (uintptr_t)lout % 16 == 0 && (uintptr_t)lin % 16 == 0 && (uintptr_t)Ci % 16 == 0 &&
                         (uintptr_t)Tk % 16 == 0 && (uintptr_t)gCi % 16 == 0;
    if (k.V > 1 && (env_int("DIFF3D_NARROW", 0) || nx % k.V != 0 || !aligned)) k = kNarrow;
    const int zlen = env_int("DIFF3D_AZLEN", 0);
    const int zdef = AdjDefaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw) \
    if (k.V == v && k.R == r && k.NW == nw) return launch_adj_cfg<DT, v, r, nw>(a, st, zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_ADJ_CFGS_8(DIFF3D_TRY)
    } else {
        DIFF3D_ADJ_CFGS_4(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

// Two adjoint steps per pass.
#define DIFF3D_ADJ2_CFGS_8(X) X(1, 1, 8) X(1, 2, 8) X(1, 2, 4) X(2, 1, 8) X(1, 4, 4)
#define DIFF3D_ADJ2_CFGS_4(X) X(1, 1, 8) X(2, 1, 8) X(1, 4, 4) X(1, 2, 8) X(2, 2, 4) X(4, 1, 8)

template <int DT>
struct Adj2Defaults;
template <> struct Adj2Defaults<DIFF3D_F64> { static constexpr ZKey wide{1, 2, 8, 0}; static constexpr int zdef = 64; };
template <> struct Adj2Defaults<DIFF3D_F32> { static constexpr ZKey wide{1, 4, 4, 0}; static constexpr int zdef = 32; };
constexpr ZKey kNarrowAdj2{1, 2, 8, 0};

template <int DT, int V, int R, int NW>
int launch_adj2_cfg(const AdjArgs<DT>& a, hipStream_t st, int zlen_req, int zdef)
{
    // one workgroup of this register-heavy kernel per CU is enough: allow
    // chunks as long as zdef down to 256 workgroups
    const ZPlan p = plan_tiles(a.nx, a.ny, a.nz, 64 * V, R * NW, zlen_req, zdef, 256);
    adj_tb2<DT, V, R, NW><<<p.blocks, 64 * NW, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

template <int DT>
int launch_adj2(void* lout, const void* lin, const void* Ci, const void* Tk, const void* Tk1, void* gCi, int nx,
                int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    AdjArgs<DT> a = make_adj_args<DT>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz);
    a.Tk1 = static_cast<const S*>(Tk1);
    ZKey k = Adj2Defaults<DT>::wide;
    env_key("DIFF3D_BCFG", k);
    const bool aligned = (uintptr_t)lout % 16 == 0 && (uintptr_t)lin % 16 == 0 && (uintptr_t)Ci % 16 == 0 &&
                         (uintptr_t)Tk % 16 == 0 && (uintptr_t)Tk1 % 16 == 0 && (uintptr_t)gCi % 16 == 0;
    if (k.V > 1 && (env_int("DIFF3D_NARROW", 0) || nx % k.V != 0 || !aligned)) k = kNarrowAdj2;
    const int zlen = env_int("DIFF3D_BZLEN", 0);
    const int zdef = Adj2Defaults<DT>::zdef;
#define DIFF3D_TRY(v, r, nw) \
    if (k.V == v && k.R == r && k.NW == nw) return launch_adj2_cfg<DT, v, r, nw>(a, st, zlen, zdef);
    if constexpr (sizeof(S) == 8) {
        DIFF3D_ADJ2_CFGS_8(DIFF3D_TRY)
    } else {
        DIFF3D_ADJ2_CFGS_4(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

int adj2_dispatch(int dtype, void* lout, const void* lin, const void* Ci, const void* Tk, const void* Tk1, void* gCi,
                  int nx, int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_adj2<DIFF3D_F64>(lout, lin, Ci, Tk, Tk1, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    case DIFF3D_F32:
        return launch_adj2<DIFF3D_F32>(lout, lin, Ci, Tk, Tk1, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    default: return DIFF3D_EDTYPE;
    }
}

// Fused reverse passes (forward states recomputed on chip): W0 x H0 region,
// NTH threads, per number of steps S.
struct RKey {
    int W0, H0, NTH;
};

#define DIFF3D_REV_CFGS_8(X) X(2, 64, 16, 1024) X(3, 64, 16, 1024) X(3, 64, 16, 512)
#define DIFF3D_REV_CFGS_4(X) X(2, 64, 32, 1024) X(3, 64, 32, 1024) X(3, 64, 16, 1024)
constexpr int kMaxRevSteps = 3;

// Measured: FP64 three-step passes on 64 x 16 regions take the 256^3 reverse
// sweep (nt = 200, C = 14) from 40.3 ms (two-step kernels over recomputed
// states) to 33 ms; FP32 three-step passes take the 1024^3 one (nt = 500,
// C = 32) from 3.26 to 2.74 s.  With FP32 fields inside the last-level cache
// (256^3: 67 MB) re-reading recomputed states is cheap and the two-step
// kernels are as fast (21.5 vs 21.8 ms), so AUTO keeps them there.
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
template <int DT>
struct RevDefaults;
template <> struct RevDefaults<DIFF3D_F64> {
    static constexpr int S = 3;
    static constexpr RKey key[kMaxRevSteps + 1] = {{0, 0, 0}, {0, 0, 0}, {64, 16, 1024}, {64, 16, 1024}};
};
template <> struct RevDefaults<DIFF3D_F32> {
    static constexpr int S = 3;
    static constexpr RKey key[kMaxRevSteps + 1] = {{0, 0, 0}, {0, 0, 0}, {64, 32, 1024}, {64, 32, 1024}};
};

template <int DT, int S, int W0, int H0, int NTH>
int launch_rev_cfg(const RevArgs<DT>& a, hipStream_t st, int zlen_req)
{
    static int cdev = -1;
    static long cslots = 0;
    auto kernel = rev_tbs<DT, S, W0, H0, NTH>;
    const long slots = resident_slots(kernel, NTH, cdev, cslots);
    const ZPlan p = plan_rounds(edge_tiles(a.nx, W0, W0 - 2 * S), edge_tiles(a.ny, H0, H0 - 2 * S), a.nz, zlen_req,
                                3 * S - 3, slots);
    kernel<<<p.blocks, NTH, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

// S reverse steps lambda_{k+S} -> lambda_k from the state T_k (2 <= S <= kMaxRevSteps).
template <int DT>
int launch_rev(int nsteps, void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx, int ny,
               int nz, double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    using Sz = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    if (nsteps < 2 || nsteps > kMaxRevSteps) return DIFF3D_EINVAL;
    RevArgs<DT> a;
    a.lout = static_cast<Sz*>(lout);
    a.lin = static_cast<const Sz*>(lin);
    a.Ci = static_cast<const Sz*>(Ci);
    a.Tk = static_cast<const Sz*>(Tk);
    a.gCi = static_cast<Sz*>(gCi);
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.lam = (C)lam;
    a.dt = (C)dt;
    a.dtlam = (C)dt * (C)lam;
    a.cx = (C)(rdx * rdx);
    a.cy = (C)(rdy * rdy);
    a.cz = (C)(rdz * rdz);
    RKey k = RevDefaults<DT>::key[nsteps];
    {
        // tuning override "S,W0,H0,NTH" for passes of S steps
        const char* e = getenv("DIFF3D_RCFG");
        int es = 0;
        RKey r{0, 0, 0};
        if (e && *e && sscanf(e, "%d,%d,%d,%d", &es, &r.W0, &r.H0, &r.NTH) == 4 && es == nsteps) k = r;
    }
    const int zlen = env_int("DIFF3D_RZLEN", 0);
#define DIFF3D_TRY(s, w0, h0, nth) \
    if (nsteps == s && k.W0 == w0 && k.H0 == h0 && k.NTH == nth) return launch_rev_cfg<DT, s, w0, h0, nth>(a, st, zlen);
    if constexpr (sizeof(Sz) == 8) {
        DIFF3D_REV_CFGS_8(DIFF3D_TRY)
    } else {
        DIFF3D_REV_CFGS_4(DIFF3D_TRY)
    }
#undef DIFF3D_TRY
    return DIFF3D_EINVAL;
}

int rev_dispatch(int dtype, int nsteps, void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx,
                 int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_rev<DIFF3D_F64>(nsteps, lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    case DIFF3D_F32:
        return launch_rev<DIFF3D_F32>(nsteps, lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    default: return DIFF3D_EDTYPE;
    }
}

// Steps per fused reverse pass: the dtype's default, or the S-step pass
// length when set (capped at kMaxRevSteps).
int rev_pass_steps(int dtype)
{
    const int d = dtype == DIFF3D_F64 ? RevDefaults<DIFF3D_F64>::S : RevDefaults<DIFF3D_F32>::S;
    if (g_kernel == DIFF3D_KERNEL_TBS && g_pass_steps >= 2) return min(g_pass_steps, kMaxRevSteps);
    return d;
}

int adj_dispatch(int dtype, void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx, int ny,
                 int nz, double lam, double dt, double rdx, double rdy, double rdz, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_adj<DIFF3D_F64>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    case DIFF3D_F32: return launch_adj<DIFF3D_F32>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
    default: return DIFF3D_EDTYPE;
    }
}

inline int nck_of(int nt, int C) { return nt > 0 ? (nt + C - 1) / C : 0; }

// ------------------------------------------------------------------ reductions
template <int DT, int OP>
int reduce_launch(const void* x, const void* y, void* seed, size_t n, double* acc, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    size_t parts = (n + 255) / 256;
    if (parts > (size_t)kRedParts) parts = kRedParts;
    if (parts < 1) parts = 1;
    reduce_partial<DT, OP><<<(unsigned)parts, 256, 0, st>>>(static_cast<const S*>(x), static_cast<const S*>(y),
                                                            static_cast<S*>(seed), n, acc);
    reduce_final<OP><<<1, 1024, 0, st>>>(acc, (int)parts);
    return hip_status();
}

template <int OP>
int reduce_dispatch(int dtype, const void* x, const void* y, void* seed, size_t n, double* acc, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return reduce_launch<DIFF3D_F64, OP>(x, y, seed, n, acc, st);
    case DIFF3D_F32: return reduce_launch<DIFF3D_F32, OP>(x, y, seed, n, acc, st);
    case DIFF3D_BF16:
    case DIFF3D_BF16_RNE: return reduce_launch<DIFF3D_BF16_RNE, OP>(x, y, seed, n, acc, st);
    default: return DIFF3D_EDTYPE;
    }
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* diff3d_strerror(int status)
{
    switch (status) {
    case DIFF3D_OK: return "ok";
    case DIFF3D_EINVAL: return "invalid argument (pointer, size, count or aliasing)";
    case DIFF3D_EDTYPE: return "unsupported dtype";
    case DIFF3D_EWORKSPACE: return "workspace missing or too small";
    case DIFF3D_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

size_t diff3d_dtype_size(int dtype) { return elem_size(dtype); }

const char* diff3d_version(void) { return "diff3d 0.1 gfx950"; }

int diff3d_scalars(int nx, int ny, int nz, double lx, double ly, double lz, double lam, double cimax, double* out)
{
    if (!out || check_grid(nx, ny, nz)) return DIFF3D_EINVAL;
    if (!(lam > 0.0) || !(cimax > 0.0) || !(lx > 0.0) || !(ly > 0.0) || !(lz > 0.0)) return DIFF3D_EINVAL;
    const double dx = lx / (nx - 1), dy = ly / (ny - 1), dz = lz / (nz - 1);
    double m = dx * dx;
    if (dy * dy < m) m = dy * dy;
    if (dz * dz < m) m = dz * dz;
    out[0] = dx;
    out[1] = dy;
    out[2] = dz;
    out[3] = 1.0 / dx;
    out[4] = 1.0 / dy;
    out[5] = 1.0 / dz;
    out[6] = m / lam / cimax / 6.1;
    return DIFF3D_OK;
}

int diff3d_max(const void* x, size_t n, int dtype, double* acc, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!x || !acc || n == 0) return DIFF3D_EINVAL;
    return reduce_dispatch<RED_MAX>(dtype, x, nullptr, nullptr, n, acc, as_stream(stream));
}

int diff3d_loss(const void* T, const void* Tt, void* seed, size_t n, int dtype, double* acc, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T || !Tt || !acc || n == 0) return DIFF3D_EINVAL;
    return reduce_dispatch<RED_SUMSQ_DIFF>(dtype, T, Tt, seed, n, acc, as_stream(stream));
}

int diff3d_norm2(const void* x, size_t n, int dtype, double* acc, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!x || !acc || n == 0) return DIFF3D_EINVAL;
    return reduce_dispatch<RED_SUMSQ>(dtype, x, nullptr, nullptr, n, acc, as_stream(stream));
}

int diff3d_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (bytes == 0) return DIFF3D_OK;
    if (!dst || !src || overlap(dst, bytes, src, bytes)) return DIFF3D_EINVAL;
    if ((uintptr_t)dst % 16 || (uintptr_t)src % 16) return DIFF3D_EINVAL;
    return copy_bytes(dst, src, bytes, as_stream(stream));
}

int diff3d_step(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                double rdy, double rdz, int dtype, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T2 || !T || !Ci || check_grid(nx, ny, nz)) return DIFF3D_EINVAL;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb)) return DIFF3D_EINVAL;
    const int rc = step_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, g_sr_step, as_stream(stream));
    g_sr_step += 1;
    return rc;
}

int diff3d_step2(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, int dtype, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T2 || !T || !Ci || check_grid(nx, ny, nz)) return DIFF3D_EINVAL;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb)) return DIFF3D_EINVAL;
    const int rc = pair_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, g_sr_step, as_stream(stream));
    g_sr_step += 2;
    return rc;
}

int diff3d_stepn(void* T2, const void* T, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
                 double rdy, double rdz, int nsteps, int dtype, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T2 || !T || !Ci || check_grid(nx, ny, nz)) return DIFF3D_EINVAL;
    if (nsteps < 1 || nsteps > DIFF3D_MAX_PASS_STEPS) return DIFF3D_EINVAL;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb)) return DIFF3D_EINVAL;
    const int rc =
        pass_dispatch(dtype, T2, T, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nsteps, g_sr_step, as_stream(stream));
    g_sr_step += (uint64_t)nsteps;
    return rc;
}

int diff3d_run(void* T, void* T2, const void* Ci, int nx, int ny, int nz, double lam, double dt, double rdx,
               double rdy, double rdz, int nt, int dtype, void* stream, void* ckpt, int ckpt_every)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (!T || !T2 || !Ci || check_grid(nx, ny, nz) || nt < 0) return DIFF3D_EINVAL;
    if (ckpt && ckpt_every < 1) return DIFF3D_EINVAL;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    if (overlap(T2, fb, T, fb) || overlap(T2, fb, Ci, fb) || overlap(T, fb, Ci, fb)) return DIFF3D_EINVAL;
    const size_t stride = align256(fb);
    if (ckpt) {
        const int nck = nck_of(nt, ckpt_every);
        const size_t cb = nck > 1 ? (size_t)(nck - 1) * stride : 0;
        if (cb && (overlap(ckpt, cb, T, fb) || overlap(ckpt, cb, T2, fb) || overlap(ckpt, cb, Ci, fb)))
            return DIFF3D_EINVAL;
    }
    if (nt == 0) return DIFF3D_OK;
    return run_loop(dtype, T, T2, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, nt, as_stream(stream), ckpt, ckpt_every,
                    stride, nt - 1, true);
}

size_t diff3d_adjoint_workspace_bytes(int nx, int ny, int nz, int nt, int ckpt_every, int dtype)
{
    if (!known_dtype(dtype) || check_grid(nx, ny, nz) || nt < 0 || ckpt_every < 1) return 0;
    const size_t stride = align256(npoints(nx, ny, nz) * elem_size(dtype));
    const int nck = nck_of(nt, ckpt_every);
    const size_t fields = (size_t)(nck > 1 ? nck - 1 : 0) + (size_t)(ckpt_every - 1) + 1;
    return fields * stride;
}

int diff3d_adjoint_run(const void* T0, const void* Ci, const void* gTnt, void* gT0, void* gCi, void* workspace,
                       size_t ws_bytes, int ckpt_ready, int nx, int ny, int nz, double lam, double dt, double rdx,
                       double rdy, double rdz, int nt, int ckpt_every, int dtype, void* stream)
{
    if (!known_dtype(dtype)) return DIFF3D_EDTYPE;
    if (dtype != DIFF3D_F64 && dtype != DIFF3D_F32) return DIFF3D_EDTYPE;
    if (!T0 || !Ci || !gTnt || !gT0 || !gCi || check_grid(nx, ny, nz) || nt < 0 || ckpt_every < 1)
        return DIFF3D_EINVAL;
    const size_t need = diff3d_adjoint_workspace_bytes(nx, ny, nz, nt, ckpt_every, dtype);
    if (!workspace || ws_bytes < need) return DIFF3D_EWORKSPACE;
    const size_t fb = npoints(nx, ny, nz) * elem_size(dtype);
    const void* ins[3] = {T0, Ci, gTnt};
    void* outs[2] = {gT0, gCi};
    for (int o = 0; o < 2; ++o) {
        for (int i = 0; i < 3; ++i)
            if (overlap(outs[o], fb, ins[i], fb)) return DIFF3D_EINVAL;
        if (overlap(outs[o], fb, workspace, need)) return DIFF3D_EINVAL;
    }
    if (overlap(gT0, fb, gCi, fb)) return DIFF3D_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (overlap(workspace, need, ins[i], fb)) return DIFF3D_EINVAL;

    hipStream_t st = as_stream(stream);
    const int C = ckpt_every;
    const size_t stride = align256(fb);
    char* ws = static_cast<char*>(workspace);
    const int nck = nck_of(nt, C);
    auto slot = [&](int j) -> void* { return ws + (size_t)(j - 1) * stride; };   // T_{jC}, j >= 1
    char* seg0 = ws + (size_t)(nck > 1 ? nck - 1 : 0) * stride;                  // C-1 recompute fields
    auto seg = [&](int i) -> void* { return seg0 + (size_t)i * stride; };
    void* W = seg0 + (size_t)(C - 1) * stride;                                   // adjoint ping-pong

    int rc = zero_bytes(gCi, fb, st);
    if (rc) return rc;
    if (nt == 0) return copy_bytes(gT0, gTnt, fb, st);

    if (!ckpt_ready && nck > 1) {
        // forward from T0 on the two scratch fields W and gT0, filling the slots
        rc = copy_bytes(W, T0, fb, st);
        const int last = (nck - 1) * C;
        if (!rc) rc = run_loop(dtype, W, gT0, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, last, st, ws, C, stride, last,
                               false);
        if (rc) return rc;
    }
    // recompute fields need T0's boundary (steps write interior points only)
    const int segn = (C - 1 < nt - 1 ? C - 1 : nt - 1);
    for (int i = 0; i < segn; ++i) {
        rc = boundary_dispatch(dtype, seg(i), T0, nx, ny, nz, st);
        if (rc) return rc;
    }

    if (g_kernel == DIFF3D_KERNEL_TBS ||
        (g_kernel == DIFF3D_KERNEL_AUTO && (dtype == DIFF3D_F64 || fb > kLastLevelCacheBytes))) {
        // Fused reverse passes of P steps (the first pass of a segment takes
        // the remainder): only the states at pass starts are recomputed (by
        // forward passes of the same lengths), the pass recomputes the rest
        // on chip.  lambda alternates between gT0 and W so that the last
        // launch writes gT0.
        const int P = rev_pass_steps(dtype);
        auto npass = [&](int len) { return (len + P - 1) / P; };
        long nlaunch = 0;
        for (int j = nck - 1; j >= 0; --j) nlaunch += npass(((j * C + C < nt) ? j * C + C : nt) - j * C);
        long launch = 0;
        const void* lin = gTnt;
        for (int j = nck - 1; j >= 0; --j) {
            const int s = j * C;
            const int len = ((s + C < nt) ? s + C : nt) - s;
            const int m = npass(len);
            const int r = len - (m - 1) * P;      // first pass: 1 .. P steps
            const void* base = j == 0 ? T0 : slot(j);
            // states at the starts of passes 1 .. m-1 into seg(0) .. seg(m-2)
            const void* src = base;
            for (int i = 1; i < m; ++i) {
                rc = pass_dispatch(dtype, seg(i - 1), src, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, i == 1 ? r : P, 0,
                                   st);
                if (rc) return rc;
                src = seg(i - 1);
            }
            for (int i = m - 1; i >= 0; --i) {
                const int n = i == 0 ? r : P;
                const void* Tk = i == 0 ? base : seg(i - 1);
                void* out = ((nlaunch - 1 - launch) % 2 == 0) ? gT0 : W;
                rc = n >= 2 ? rev_dispatch(dtype, n, out, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st)
                            : adj_dispatch(dtype, out, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
                if (rc) return rc;
                lin = out;
                ++launch;
            }
        }
        return DIFF3D_OK;
    }

    // adjoint launches (two steps per launch inside a segment where enabled);
    // lambda alternates between gT0 and W so that the last launch writes gT0
    const bool apairs = g_kernel == DIFF3D_KERNEL_AUTO || g_kernel == DIFF3D_KERNEL_TB2;
    long nlaunch = 0;
    for (int j = nck - 1; j >= 0; --j) {
        const int len = ((j * C + C < nt) ? j * C + C : nt) - j * C;
        nlaunch += apairs ? (len + 1) / 2 : len;
    }
    long launch = 0;
    const void* lin = gTnt;
    for (int j = nck - 1; j >= 0; --j) {
        const int s = j * C;
        const int e = (s + C < nt) ? s + C : nt;
        const void* base = j == 0 ? T0 : slot(j);
        // states T_{s+1} .. T_{e-1} into seg(0) .. seg(e-s-2), two at a time
        // where possible (one pass writing both the intermediate and the
        // second state), the two-step kernel unless single steps are selected
        const void* src = base;
        const bool pairs = g_kernel == DIFF3D_KERNEL_AUTO || g_kernel == DIFF3D_KERNEL_TB2;
        for (int k = s; k < e - 1;) {
            if (pairs && k + 2 <= e - 1) {
                rc = pair_mid_dispatch(dtype, seg(k - s + 1), seg(k - s), src, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz,
                                       st);
                src = seg(k - s + 1);
                k += 2;
            } else {
                rc = step_dispatch(dtype, seg(k - s), src, Ci, nx, ny, nz, lam, dt, rdx, rdy, rdz, 0, st);
                src = seg(k - s);
                k += 1;
            }
            if (rc) return rc;
        }
        auto state = [&](int k) -> const void* { return k == s ? base : seg(k - s - 1); };
        for (int k = e - 1; k >= s;) {
            void* out = ((nlaunch - 1 - launch) % 2 == 0) ? gT0 : W;
            if (apairs && k - 1 >= s) {
                rc = adj2_dispatch(dtype, out, lin, Ci, state(k), state(k - 1), gCi, nx, ny, nz, lam, dt, rdx, rdy,
                                   rdz, st);
                k -= 2;
            } else {
                rc = adj_dispatch(dtype, out, lin, Ci, state(k), gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, st);
                k -= 1;
            }
            if (rc) return rc;
            lin = out;
            ++launch;
        }
    }
    return DIFF3D_OK;
}

int diff3d_set_kernel(int kernel)
{
    if (kernel < DIFF3D_KERNEL_AUTO || kernel > DIFF3D_KERNEL_TBS) return DIFF3D_EINVAL;
    g_kernel = kernel;
    return DIFF3D_OK;
}

int diff3d_get_kernel(void) { return g_kernel; }

int diff3d_set_pass_steps(int nsteps)
{
    if (nsteps < 0 || nsteps == 1 || nsteps > DIFF3D_MAX_PASS_STEPS) return DIFF3D_EINVAL;
    g_pass_steps = nsteps;
    return DIFF3D_OK;
}

void diff3d_set_sr_seed(uint64_t seed, uint64_t step0)
{
    g_sr_seed = seed;
    g_sr_step = step0;
}

void diff3d_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const u32x4 r = philox4x32_10(u32x4{ctr[0], ctr[1], ctr[2], ctr[3]}, key[0], key[1]);
    out[0] = r.x;
    out[1] = r.y;
    out[2] = r.z;
    out[3] = r.w;
}

}  // extern "C"
