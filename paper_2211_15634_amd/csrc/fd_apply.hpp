// The finite-difference operators of fd_ops.hpp applied to a whole field
// (diff3d_apply): interior selection (@inn), the second difference along x,
// y or z (@d2_xi, @d2_yi, @d2_zi) and the weighted Laplacian of the step,
// each written densely over the interior in the arithmetic type.
//
// A utility pass, not a hot path: each workgroup of 256 threads takes runs of
// 256 consecutive interior x points of one (y, z) row (coalesced loads of the
// row and its neighbour rows through the caches, one coalesced store), and
// the grid strides over all such runs.
#pragma once

#include "common.hpp"
#include "fd_ops.hpp"
#include "host_common.hpp"

namespace diff3d {

template <int DT>
struct ApplyArgs {
    using S = typename Traits<DT>::S;
    using C = typename Traits<DT>::C;
    typename Traits<DT>::C* __restrict__ out;
    const S* __restrict__ in;
    int nx, ny, nz;    // nz == 1: a 2-D field
    C cx, cy, cz;
};

template <int DT, int OP>
__global__ __launch_bounds__(256) void fd_apply(ApplyArgs<DT> a, long runs, int xruns)
{
    using Tr = Traits<DT>;
    using C = typename Tr::C;
    const bool twod = a.nz == 1;
    const int ix_n = a.nx - 2, iy_n = a.ny - 2;
    const size_t sy = (size_t)a.nx, sz = (size_t)a.nx * a.ny;
    for (long r = blockIdx.x; r < runs; r += gridDim.x) {
        const long row = r / xruns;              // (iy - 1) + iy_n*(iz - 1)
        const int ox = (int)(r - row * xruns) * 256 + (int)threadIdx.x;
        if (ox >= ix_n) continue;
        const int iy = (int)(row % iy_n) + 1;
        const int iz = twod ? 0 : (int)(row / iy_n) + 1;
        const size_t i = (size_t)(ox + 1) + sy * iy + sz * iz;
        const C t = Tr::load(a.in[i]);
        C v;
        if constexpr (OP == DIFF3D_OP_INN) {
            v = t;
        } else if constexpr (OP == DIFF3D_OP_D2_XI) {
            v = fd::d2(Tr::load(a.in[i - 1]), t, Tr::load(a.in[i + 1]));
        } else if constexpr (OP == DIFF3D_OP_D2_YI) {
            v = fd::d2(Tr::load(a.in[i - sy]), t, Tr::load(a.in[i + sy]));
        } else if constexpr (OP == DIFF3D_OP_D2_ZI) {
            v = fd::d2(Tr::load(a.in[i - sz]), t, Tr::load(a.in[i + sz]));
        } else {
            const C xm = Tr::load(a.in[i - 1]), xp = Tr::load(a.in[i + 1]);
            const C ym = Tr::load(a.in[i - sy]), yp = Tr::load(a.in[i + sy]);
            if (twod) {
                v = fd::lap2(t, xm, xp, ym, yp, a.cx, a.cy);
            } else {
                const C zm = Tr::load(a.in[i - sz]), zp = Tr::load(a.in[i + sz]);
                v = fd::lap3(t, xm, xp, ym, yp, zm, zp, a.cx, a.cy, a.cz);
            }
        }
        a.out[(size_t)ox + (size_t)ix_n * (size_t)row] = v;
    }
}

namespace {

template <int DT>
int launch_apply(int op, void* out, const void* in, int nx, int ny, int nz, double rdx, double rdy, double rdz,
                 hipStream_t st)
{
    using C = typename Traits<DT>::C;
    ApplyArgs<DT> a;
    a.out = static_cast<C*>(out);
    a.in = static_cast<const typename Traits<DT>::S*>(in);
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.cx = (C)(rdx * rdx);
    a.cy = (C)(rdy * rdy);
    a.cz = (C)(rdz * rdz);
    const int xruns = (nx - 2 + 255) / 256;
    const long rows = (long)(ny - 2) * (nz == 1 ? 1 : nz - 2);
    const long runs = rows * xruns;
    const unsigned grid = (unsigned)(runs < (1L << 20) ? runs : (1L << 20));
    switch (op) {
    case DIFF3D_OP_INN: fd_apply<DT, DIFF3D_OP_INN><<<grid, 256, 0, st>>>(a, runs, xruns); break;
    case DIFF3D_OP_D2_XI: fd_apply<DT, DIFF3D_OP_D2_XI><<<grid, 256, 0, st>>>(a, runs, xruns); break;
    case DIFF3D_OP_D2_YI: fd_apply<DT, DIFF3D_OP_D2_YI><<<grid, 256, 0, st>>>(a, runs, xruns); break;
    case DIFF3D_OP_D2_ZI: fd_apply<DT, DIFF3D_OP_D2_ZI><<<grid, 256, 0, st>>>(a, runs, xruns); break;
    case DIFF3D_OP_LAP: fd_apply<DT, DIFF3D_OP_LAP><<<grid, 256, 0, st>>>(a, runs, xruns); break;
    default: return DIFF3D_EINVAL;
    }
    return hip_status();
}

// BF16 inputs with either rounding mode are widened the same way; nothing is
// rounded back to BF16.
int apply_dispatch(int dtype, int op, void* out, const void* in, int nx, int ny, int nz, double rdx, double rdy,
                   double rdz, hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return launch_apply<DIFF3D_F64>(op, out, in, nx, ny, nz, rdx, rdy, rdz, st);
    case DIFF3D_F32: return launch_apply<DIFF3D_F32>(op, out, in, nx, ny, nz, rdx, rdy, rdz, st);
    case DIFF3D_BF16:
    case DIFF3D_BF16_RNE: return launch_apply<DIFF3D_BF16_RNE>(op, out, in, nx, ny, nz, rdx, rdy, rdz, st);
    default: return DIFF3D_EDTYPE;
    }
}

}  // namespace
}  // namespace diff3d
