// Support kernels: boundary copy (T2 = T on the boundary, as T2 = copy(T)
// in Fig. 1), zero fill, the bandwidth-reference copy and deterministic FP64
// reductions (max, loss, squared norm).
#pragma once

#include "common.hpp"

namespace diff3d {

// dst = src on the six faces of an nx*ny*nz grid (edges are written twice
// with the same value).
template <class S>
__global__ __launch_bounds__(256) void boundary_copy(S* __restrict__ dst, const S* __restrict__ src, int nx,
                                                     int ny, int nz)
{
    const size_t fz = (size_t)nx * ny, fy = (size_t)nx * nz, fx = (size_t)ny * nz;
    const size_t total = 2 * (fz + fy + fx);
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (size_t)gridDim.x * 256) {
        size_t i;
        size_t q = k;
        if (q < 2 * fz) {                      // z = 0 and z = nz-1
            const size_t side = q / fz, r = q % fz;
            i = r + sz * (side ? (size_t)(nz - 1) : 0);
        } else if ((q -= 2 * fz) < 2 * fy) {   // y = 0 and y = ny-1
            const size_t side = q / fy, r = q % fy;
            const size_t x = r % nx, z = r / nx;
            i = x + sy * (side ? (size_t)(ny - 1) : 0) + sz * z;
        } else {                               // x = 0 and x = nx-1
            q -= 2 * fy;
            const size_t side = q / fx, r = q % fx;
            const size_t y = r % ny, z = r / ny;
            i = (side ? (size_t)(nx - 1) : 0) + sy * y + sz * z;
        }
        dst[i] = src[i];
    }
}

// dst = src on the four edges of an nx*ny plane (corners written twice with
// the same value).
template <class S>
__global__ __launch_bounds__(256) void boundary_copy2d(S* __restrict__ dst, const S* __restrict__ src, int nx, int ny)
{
    const size_t rows = 2 * (size_t)nx, total = rows + 2 * (size_t)ny;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (size_t)gridDim.x * 256) {
        size_t i;
        if (k < rows) {                        // y = 0 and y = ny-1
            const size_t side = k / nx, x = k % nx;
            i = x + (size_t)nx * (side ? (size_t)(ny - 1) : 0);
        } else {                               // x = 0 and x = nx-1
            const size_t q = k - rows, side = q / ny, y = q % ny;
            i = (side ? (size_t)(nx - 1) : 0) + (size_t)nx * y;
        }
        dst[i] = src[i];
    }
}

__global__ __launch_bounds__(256) void fill_zero(uint4* __restrict__ p, size_t n16, unsigned char* __restrict__ tail,
                                                 size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// Streaming copy: each workgroup moves one contiguous chunk of 256*4
// 16-byte vectors (all four loads in flight before the stores), with
// non-temporal loads and stores.  One short-lived workgroup per 16 KiB keeps
// the whole chip busy without a grid-stride loop.
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(256) void copy16(u32v4* __restrict__ dst, const u32v4* __restrict__ src, size_t n16)
{
    const size_t base = (size_t)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x;
    u32v4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n16) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n16) __builtin_nontemporal_store(v[u], dst + i);
    }
}

__global__ __launch_bounds__(256) void copy_u16(uint16_t* __restrict__ dst, const uint16_t* __restrict__ src,
                                                size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

__global__ void copy_tail(unsigned char* __restrict__ dst, const unsigned char* __restrict__ src, size_t n)
{
    if (threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

// ------------------------------------------------------------------ reductions
// Pass 1: block b reduces a fixed grid-stride subset into partials[b]
// (fixed tree in LDS); pass 2: one block reduces partials[0 .. nparts-1]
// into out[0].  Same grid and same order on every call: deterministic.
// Every partial the second pass reads is written by the first, so the
// partials need no clearing.
enum { RED_MAX = 0, RED_SUMSQ_DIFF = 1, RED_SUMSQ = 2 };
constexpr int kRedParts = 1024;

template <int DT, int OP>
__global__ __launch_bounds__(256) void reduce_partial(const typename Traits<DT>::S* __restrict__ x,
                                                      const typename Traits<DT>::S* __restrict__ y,
                                                      typename Traits<DT>::S* __restrict__ seed, size_t n,
                                                      double* __restrict__ partials)
{
    using Tr = Traits<DT>;
    __shared__ double sh[256];
    double s = OP == RED_MAX ? -__builtin_huge_val() : 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double v = (double)Tr::load(x[i]);
        if (OP == RED_MAX) {
            s = v > s ? v : s;
        } else if (OP == RED_SUMSQ) {
            s += v * v;
        } else {
            const double r = v - (double)Tr::load(y[i]);
            if (seed) {
                // RNE for every storage form (the reverse sweep runs in FP64/FP32)
                if (sizeof(typename Tr::S) == 2)
                    seed[i] = (typename Tr::S)f32_to_bf16_rne((float)r);
                else
                    seed[i] = (typename Tr::S)r;
            }
            s += r * r;
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = sh[threadIdx.x + w];
            sh[threadIdx.x] = OP == RED_MAX ? (o > sh[threadIdx.x] ? o : sh[threadIdx.x]) : sh[threadIdx.x] + o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

template <int OP>
__global__ __launch_bounds__(1024) void reduce_final(const double* __restrict__ partials, int nparts,
                                                     double* __restrict__ out)
{
    __shared__ double sh[1024];
    const double id = OP == RED_MAX ? -__builtin_huge_val() : 0.0;
    sh[threadIdx.x] = (int)threadIdx.x < nparts ? partials[threadIdx.x] : id;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = sh[threadIdx.x + w];
            sh[threadIdx.x] = OP == RED_MAX ? (o > sh[threadIdx.x] ? o : sh[threadIdx.x]) : sh[threadIdx.x] + o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = OP == RED_SUMSQ_DIFF ? 0.5 * sh[0] : sh[0];
}

}  // namespace diff3d
