// Reverse-step launches: single and two-step adjoint kernels and fused
// reverse passes, with their configuration tables and dispatch.
#pragma once

#include "forward_launch.hpp"
#include "adjoint_kernels.hpp"
#include "rev_kernels.hpp"

namespace diff3d {
namespace {

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
               double lam, double dt, double rdx, double rdy, double rdz, const diff3d_config& c, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    const AdjArgs<DT> a = make_adj_args<DT>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz);
    if (c.kernel == DIFF3D_KERNEL_NAIVE) {
        dim3 grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4), (unsigned)min(nz, 65535));
        adj_naive<DT><<<grid, 256, 0, st>>>(a);
        return hip_status();
    }
    ZKey k = zkey_of(c.adj, AdjDefaults<DT>::wide);
    const bool aligned = (uintptr_t)lout % 16 == 0 && (uintptr_t)lin % 16 == 0 && (uintptr_t)Ci % 16 == 0 &&
                         (uintptr_t)Tk % 16 == 0 && (uintptr_t)gCi % 16 == 0;
    if (k.V > 1 && (c.narrow || nx % k.V != 0 || !aligned)) k = kNarrow;
    const int zlen = c.adj.zlen;
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
                int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz, const diff3d_config& c,
                hipStream_t st)
{
    using S = typename Traits<DT>::S;
    AdjArgs<DT> a = make_adj_args<DT>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz);
    a.Tk1 = static_cast<const S*>(Tk1);
    ZKey k = zkey_of(c.adj2, Adj2Defaults<DT>::wide);
    const bool aligned = (uintptr_t)lout % 16 == 0 && (uintptr_t)lin % 16 == 0 && (uintptr_t)Ci % 16 == 0 &&
                         (uintptr_t)Tk % 16 == 0 && (uintptr_t)Tk1 % 16 == 0 && (uintptr_t)gCi % 16 == 0;
    if (k.V > 1 && (c.narrow || nx % k.V != 0 || !aligned)) k = kNarrowAdj2;
    const int zlen = c.adj2.zlen;
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
                  int nx, int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz,
                  const diff3d_config& c, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_adj2<DIFF3D_F64>(lout, lin, Ci, Tk, Tk1, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    case DIFF3D_F32:
        return launch_adj2<DIFF3D_F32>(lout, lin, Ci, Tk, Tk1, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
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

// Measured reverse sweeps: 256^3, nt = 200, C = 14: FP64 40.3 ms with
// two-step kernels over recomputed states, 22.1 ms with three-step passes on
// 64 x 16 regions (20.6-21.0 ms with the later kernel changes); FP32 21.5 ms
// and 13.7 ms (64 x 32 regions; 13.4 ms with paired rows).  1024^3 FP32,
// nt = 500, C = 32: 3.26 s and 1.81 s (1.77 s).
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
    static std::atomic<long long> cache{0};
    auto kernel = rev_tbs<DT, S, W0, H0, NTH>;
    const long slots = resident_slots(kernel, NTH, cache);
    const ZPlan p = plan_rounds(edge_tiles(a.nx, W0, W0 - 2 * S), edge_tiles(a.ny, H0, H0 - 2 * S), a.nz, zlen_req,
                                3 * S - 3, slots);
    kernel<<<p.blocks, NTH, 0, st>>>(a, p.ntx, p.nty, p.zlen);
    return hip_status();
}

// S reverse steps lambda_{k+S} -> lambda_k from the state T_k (2 <= S <= kMaxRevSteps).
template <int DT>
int launch_rev(int nsteps, void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx, int ny,
               int nz, double lam, double dt, double rdx, double rdy, double rdz, const diff3d_config& c,
               hipStream_t st)
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
    if (tile_set(c.rev) && c.rev.steps == nsteps) k = RKey{c.rev.p[0], c.rev.p[1], c.rev.p[2]};
    const int zlen = szlen_of(c.rev, nsteps);
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
                 int ny, int nz, double lam, double dt, double rdx, double rdy, double rdz, const diff3d_config& c,
                 hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_rev<DIFF3D_F64>(nsteps, lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    case DIFF3D_F32:
        return launch_rev<DIFF3D_F32>(nsteps, lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    default: return DIFF3D_EDTYPE;
    }
}

// Steps per fused reverse pass: the dtype's default, or the S-step pass
// length when set (capped at kMaxRevSteps).
int rev_pass_steps(int dtype, const diff3d_config& c)
{
    const int d = dtype == DIFF3D_F64 ? RevDefaults<DIFF3D_F64>::S : RevDefaults<DIFF3D_F32>::S;
    if (c.kernel == DIFF3D_KERNEL_TBS && c.pass_steps >= 2) return min(c.pass_steps, kMaxRevSteps);
    return d;
}

// The reverse sweep runs fused passes under AUTO and TBS, and recomputes
// every state of a segment otherwise.
inline bool rev_fused(const diff3d_config& c)
{
    return c.kernel == DIFF3D_KERNEL_TBS || c.kernel == DIFF3D_KERNEL_AUTO;
}

// Fields for the states recomputed inside one checkpoint segment of at most
// L = min(C, nt) steps: the starts of the fused passes after the first
// (ceil(L/P) - 1), or every state after the segment's first (L - 1).
inline int recompute_fields(int dtype, int nt, int C, const diff3d_config& c)
{
    const int L = min(C, nt);
    if (L <= 1) return 0;
    if (rev_fused(c)) {
        const int P = rev_pass_steps(dtype, c);
        return (L + P - 1) / P - 1;
    }
    return L - 1;
}

int adj_dispatch(int dtype, void* lout, const void* lin, const void* Ci, const void* Tk, void* gCi, int nx, int ny,
                 int nz, double lam, double dt, double rdx, double rdy, double rdz, const diff3d_config& c,
                 hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64:
        return launch_adj<DIFF3D_F64>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    case DIFF3D_F32:
        return launch_adj<DIFF3D_F32>(lout, lin, Ci, Tk, gCi, nx, ny, nz, lam, dt, rdx, rdy, rdz, c, st);
    default: return DIFF3D_EDTYPE;
    }
}

inline bool adj_has(int size, const ZKey& k)
{
#define DIFF3D_HAS(v, r, nw) || (k.V == v && k.R == r && k.NW == nw && k.NT == 0)
    switch (size) {
    case 8: return false DIFF3D_ADJ_CFGS_8(DIFF3D_HAS);
    case 4: return false DIFF3D_ADJ_CFGS_4(DIFF3D_HAS);
    default: return false;
    }
#undef DIFF3D_HAS
}

inline bool adj2_has(int size, const ZKey& k)
{
#define DIFF3D_HAS(v, r, nw) || (k.V == v && k.R == r && k.NW == nw && k.NT == 0)
    switch (size) {
    case 8: return false DIFF3D_ADJ2_CFGS_8(DIFF3D_HAS);
    case 4: return false DIFF3D_ADJ2_CFGS_4(DIFF3D_HAS);
    default: return false;
    }
#undef DIFF3D_HAS
}

inline bool rev_has(int size, int S, const RKey& k)
{
#define DIFF3D_HAS(s, w0, h0, nth) || (S == s && k.W0 == w0 && k.H0 == h0 && k.NTH == nth)
    switch (size) {
    case 8: return false DIFF3D_REV_CFGS_8(DIFF3D_HAS);
    case 4: return false DIFF3D_REV_CFGS_4(DIFF3D_HAS);
    default: return false;
    }
#undef DIFF3D_HAS
}

// Validation of the reverse sweep's configuration (the forward part is
// checked by check_forward_config).
int check_adjoint_config(const diff3d_config& c, int dtype)
{
    const int size = (int)elem_size(dtype);
    if (c.adj.steps != 0 || c.adj2.steps != 0 || c.adj.zlen < 0 || c.adj2.zlen < 0 || c.rev.zlen < 0)
        return DIFF3D_EINVAL;
    if (tile_set(c.adj) && !adj_has(size, zkey_of(c.adj, kNarrow))) return DIFF3D_EINVAL;
    if (tile_set(c.adj2) && !adj2_has(size, zkey_of(c.adj2, kNarrow))) return DIFF3D_EINVAL;
    if (c.rev.steps != 0 && (c.rev.steps < 2 || c.rev.steps > kMaxRevSteps)) return DIFF3D_EINVAL;
    if (tile_set(c.rev) &&
        (c.rev.steps == 0 || c.rev.p[3] != 0 || !rev_has(size, c.rev.steps, RKey{c.rev.p[0], c.rev.p[1], c.rev.p[2]})))
        return DIFF3D_EINVAL;
    return DIFF3D_OK;
}

}  // namespace
}  // namespace diff3d
