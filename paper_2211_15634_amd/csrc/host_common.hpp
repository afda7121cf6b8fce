// Host side of the library: argument helpers and the per-call configuration.
// Everything here is internal to the library (one translation unit); the
// library keeps no state between calls.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "diff3d.h"

namespace diff3d {
namespace {

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

// The caller's configuration, or the defaults (a zero-filled struct).
inline diff3d_config config_of(const diff3d_config* cfg)
{
    diff3d_config c;
    memset(&c, 0, sizeof c);
    if (cfg) c = *cfg;
    return c;
}

inline bool tile_set(const diff3d_tile& t)
{
    return t.p[0] || t.p[1] || t.p[2] || t.p[3];
}

}  // namespace
}  // namespace diff3d
