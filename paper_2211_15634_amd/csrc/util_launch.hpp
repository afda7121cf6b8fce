// Launches of the utility kernels: copies, fills, boundary copies and the
// deterministic reductions.
#pragma once

#include "launch_plan.hpp"
#include "util_kernels.hpp"

namespace diff3d {
namespace {

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

// dst = src on the edges of an nx*ny plane (the 2-D form's boundary).
int boundary2d_dispatch(int dtype, void* dst, const void* src, int nx, int ny, hipStream_t st)
{
    const size_t total = 2 * ((size_t)nx + (size_t)ny);
    size_t blocks = (total + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    switch (elem_size(dtype)) {
    case 8:
        boundary_copy2d<uint64_t><<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint64_t*>(dst),
                                                                     static_cast<const uint64_t*>(src), nx, ny);
        break;
    case 4:
        boundary_copy2d<uint32_t><<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint32_t*>(dst),
                                                                     static_cast<const uint32_t*>(src), nx, ny);
        break;
    case 2:
        boundary_copy2d<uint16_t><<<(unsigned)blocks, 256, 0, st>>>(static_cast<uint16_t*>(dst),
                                                                     static_cast<const uint16_t*>(src), nx, ny);
        break;
    default: return DIFF3D_EDTYPE;
    }
    return hip_status();
}

// ------------------------------------------------------------------ reductions
// partials: at least kRedParts doubles of device scratch; out: one double.
template <int DT, int OP>
int reduce_launch(const void* x, const void* y, void* seed, size_t n, double* partials, double* out, hipStream_t st)
{
    using S = typename Traits<DT>::S;
    size_t parts = (n + 255) / 256;
    if (parts > (size_t)kRedParts) parts = kRedParts;
    if (parts < 1) parts = 1;
    reduce_partial<DT, OP><<<(unsigned)parts, 256, 0, st>>>(static_cast<const S*>(x), static_cast<const S*>(y),
                                                            static_cast<S*>(seed), n, partials);
    reduce_final<OP><<<1, 1024, 0, st>>>(partials, (int)parts, out);
    return hip_status();
}

template <int OP>
int reduce_dispatch(int dtype, const void* x, const void* y, void* seed, size_t n, double* partials, double* out,
                    hipStream_t st)
{
    switch (dtype) {
    case DIFF3D_F64: return reduce_launch<DIFF3D_F64, OP>(x, y, seed, n, partials, out, st);
    case DIFF3D_F32: return reduce_launch<DIFF3D_F32, OP>(x, y, seed, n, partials, out, st);
    case DIFF3D_BF16:
    case DIFF3D_BF16_RNE: return reduce_launch<DIFF3D_BF16_RNE, OP>(x, y, seed, n, partials, out, st);
    default: return DIFF3D_EDTYPE;
    }
}

}  // namespace
}  // namespace diff3d
