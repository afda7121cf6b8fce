// Finite-difference operators in the notation of the paper's kernel (Fig. 1
// writes the step as @inn(T2) = @inn(T) + dt*(lam*@inn(Ci)*(@d2_xi(T)*_dx^2
// + @d2_yi(T)*_dy^2 + @d2_zi(T)*_dz^2))).  Every stencil of the library --
// the forward step in 3-D and 2-D, the recomputation and the adjoint step --
// is composed of these, so they define its operation order:
//
//   inn(A)   the interior points of A (every index shifted by one);
//   d2(A) along an axis at an interior point c with neighbours m and p:
//            (A[p] - A[c]) - (A[c] - A[m]), the difference of the two
//            one-sided differences (the paper does not print @d2_xi; this is
//            the reading taken, exactly A[p] - 2A[c] + A[m] in exact
//            arithmetic, zero on constants);
//   lap(A)   the weighted sum of the three second differences,
//            (d2x*cx + d2y*cy) + d2z*cz, left to right;
//   update   t + dt*(lamci*lap), lamci = lam*Ci formed first.
//
// Host and device functions, built without contraction (-ffp-contract=off).
#pragma once

#include <hip/hip_runtime.h>

namespace diff3d {
namespace fd {

// @d2_xi / @d2_yi / @d2_zi at one point: centre c, neighbours m and p along the axis
template <class C>
__host__ __device__ __attribute__((always_inline)) inline C d2(C m, C c, C p)
{
    return (p - c) - (c - m);
}

// the weighted 7-point Laplacian of the 3-D step
template <class C>
__host__ __device__ __attribute__((always_inline)) inline C lap3(C t, C xm, C xp, C ym, C yp, C zm, C zp, C cx, C cy, C cz)
{
    const C dx = d2(xm, t, xp), dy = d2(ym, t, yp), dz = d2(zm, t, zp);
    return (dx * cx + dy * cy) + dz * cz;
}

// the weighted 5-point Laplacian of the 2-D step
template <class C>
__host__ __device__ __attribute__((always_inline)) inline C lap2(C t, C xm, C xp, C ym, C yp, C cx, C cy)
{
    const C dx = d2(xm, t, xp), dy = d2(ym, t, yp);
    return dx * cx + dy * cy;
}

// the explicit update of Fig. 1 from the Laplacian and lam*Ci
template <class C>
__host__ __device__ __attribute__((always_inline)) inline C update(C t, C dt, C lamci, C lap)
{
    return t + dt * (lamci * lap);
}

}  // namespace fd
}  // namespace diff3d
