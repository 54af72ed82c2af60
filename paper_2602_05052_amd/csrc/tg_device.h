// Device helpers shared by the assembly and adjoint kernels: addressing,
// XCD-aware block order, and the affine P1 simplex geometry.
#pragma once
#include "tg_internal.h"

namespace tg {
namespace {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on
// XCD i % 8).  Neighbouring row blocks share elements, so give each XCD one
// contiguous range of blocks and let its L2 serve the shared gathers.
__device__ __forceinline__ int xcd_swizzle(int i, int n) {
    const int q = n >> 3, rem = n & 7;
    const int x = i & 7, j = i >> 3;
    return x * q + min(x, rem) + j;
}

// Loads and stores through a uniform base pointer and a 32-bit unsigned byte
// offset, so that the compiler can use the scalar-base + vector-offset
// addressing of global memory instructions instead of 64-bit address
// arithmetic per lane.  Every array the kernels touch is below 4 GiB (checked
// on the host before the launch).
template <typename T>
__device__ __forceinline__ T ldg(const T *__restrict__ base, unsigned idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T *__restrict__ base, unsigned idx, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (unsigned)sizeof(T)) = v;
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Reference-simplex measure 1/d! (the weight of the 1-point centroid rule).
template <int D> struct RefSimplex;
template <> struct RefSimplex<2> { static constexpr double vol = 1.0 / 2.0; };
template <> struct RefSimplex<3> { static constexpr double vol = 1.0 / 6.0; };

// Cofactor form of the P1 gradients: grad(lambda_b) = C_b / det J, where
// C_1..C_d are the rows of adj(J) (the reciprocal basis times det J) and
// C_0 = -(C_1 + ... + C_d).  Then |T| grad(lambda_a).grad(lambda_b) =
// (C_a . C_b) / (d! |det J|), which needs one division per element and no
// scaling of the gradients.  Returns det J.
template <int D>
__device__ __forceinline__ double p1_cofactors(const double (&x)[D + 1][D], double (&C)[D + 1][D]) {
    if constexpr (D == 2) {
        const double e1x = x[1][0] - x[0][0], e1y = x[1][1] - x[0][1];
        const double e2x = x[2][0] - x[0][0], e2y = x[2][1] - x[0][1];
        C[1][0] = e2y;
        C[1][1] = -e2x;
        C[2][0] = -e1y;
        C[2][1] = e1x;
        C[0][0] = -(e2y - e1y);
        C[0][1] = -(e1x - e2x);
        return e1x * e2y - e1y * e2x;
    } else {
        double e[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 3; ++r) e[c][r] = x[c + 1][r] - x[0][r];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
            C[1][r] = e[1][r1] * e[2][r2] - e[1][r2] * e[2][r1];
            C[2][r] = e[2][r1] * e[0][r2] - e[2][r2] * e[0][r1];
            C[3][r] = e[0][r1] * e[1][r2] - e[0][r2] * e[1][r1];
            C[0][r] = -(C[1][r] + C[2][r] + C[3][r]);
        }
        return e[0][0] * C[1][0] + e[0][1] * C[1][1] + e[0][2] * C[1][2];
    }
}

// J is numerically singular when |det J| <= 16 eps |x_1 - x_0| ... |x_d - x_0|
// (a fraction of the Hadamard bound of J).  With fused multiply-adds, an
// element with two coincident vertices need not give det J == 0 exactly, so a
// scale-invariant threshold replaces the exact test; NaN and Inf fail it too.
template <int D>
__device__ __forceinline__ bool numerically_singular(const double (&x)[D + 1][D], double det) {
    double prod = 1.0;
#pragma unroll
    for (int c = 1; c <= D; ++c) {
        double n = 0.0;
#pragma unroll
        for (int r = 0; r < D; ++r) n += (x[c][r] - x[0][r]) * (x[c][r] - x[0][r]);
        prod *= n;
    }
    constexpr double tol = 16.0 * 2.220446049250313e-16;
    return (bool)((int)!(det * det > tol * tol * prod) | (int)!finite(det));
}

}  // namespace
}  // namespace tg
