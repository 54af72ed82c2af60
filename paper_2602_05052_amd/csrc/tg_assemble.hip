// Fused Batch-Map + Sparse-Reduce kernels for gfx950 (TensorGalerkin Sec. 2,
// Alg. 1 and Alg. 2).
//
// One workgroup owns a block of consecutive CSR node rows.  Work inside it:
//   Map    : one lane per (row node i, element e, local node a) pair of the
//            block.  It gathers e's vertices, forms J, |det J| and J^{-1} in
//            FP64 (Alg. 1 Geometry), pushes the reference gradients forward
//            (Push-forward), evaluates the per-element coefficients (Physics),
//            and integrates row a of K_e and entry a of F_e with the
//            quadrature rule (Integration, eq. kloc1).  The row goes to LDS.
//   Reduce : one lane per CSR value of the block sums the element slots that
//            the routing table maps to it (the S_mat projection of Alg. 2),
//            in ascending element order, and writes the value once; one lane
//            per row sums its load contributions (the S_vec projection).
// K_local therefore never leaves the chip, every output is written exactly
// once with coalesced stores, and no atomics touch values: the result is
// bitwise reproducible and independent of the launch geometry.
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

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Reference-simplex measure 1/d! (the weight of the 1-point centroid rule).
template <int D> struct RefSimplex;
template <> struct RefSimplex<2> { static constexpr double vol = 1.0 / 2.0; };
template <> struct RefSimplex<3> { static constexpr double vol = 1.0 / 6.0; };

// Degree-2 rules on the reference simplex, in barycentric form: point q has
// barycentric coordinate hi at vertex q and lo elsewhere; weights are equal.
//   triangle: 3 points (2/3, 1/6, 1/6)
//   tetrahedron: 4 points (alpha, beta, beta, beta), alpha = (5 + 3 sqrt 5)/20,
//                beta = (5 - sqrt 5)/20  (Keast's 4-point rule)
template <int D> struct Deg2Rule;
template <> struct Deg2Rule<2> {
    static constexpr int Q = 3;
    static constexpr double hi = 2.0 / 3.0, lo = 1.0 / 6.0, w = 1.0 / 6.0;
};
template <> struct Deg2Rule<3> {
    static constexpr int Q = 4;
    static constexpr double hi = 0.58541019662496845446, lo = 0.13819660112501051518, w = 1.0 / 24.0;
};

// Physical gradients of the barycentric (P1) basis, G[a] = J^{-T} grad(lambda_hat_a):
// rows of J^{-1} for a >= 1, and G[0] = -(G[1] + ... + G[D]).  J has columns
// x_c - x_0.  Returns det J.
template <int D>
__device__ __forceinline__ double p1_gradients(const double (&x)[D + 1][D], double (&G)[D + 1][D]) {
    if constexpr (D == 2) {
        const double e1x = x[1][0] - x[0][0], e1y = x[1][1] - x[0][1];
        const double e2x = x[2][0] - x[0][0], e2y = x[2][1] - x[0][1];
        const double det = e1x * e2y - e1y * e2x;
        const double id = 1.0 / det;
        G[1][0] = e2y * id;
        G[1][1] = -e2x * id;
        G[2][0] = -e1y * id;
        G[2][1] = e1x * id;
        G[0][0] = -(G[1][0] + G[2][0]);
        G[0][1] = -(G[1][1] + G[2][1]);
        return det;
    } else {
        double e[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 3; ++r) e[c][r] = x[c + 1][r] - x[0][r];
        // rows of J^{-1} are the reciprocal basis: (e2 x e3, e3 x e1, e1 x e2) / det
        double c23[3], c31[3], c12[3];
        c23[0] = e[1][1] * e[2][2] - e[1][2] * e[2][1];
        c23[1] = e[1][2] * e[2][0] - e[1][0] * e[2][2];
        c23[2] = e[1][0] * e[2][1] - e[1][1] * e[2][0];
        c31[0] = e[2][1] * e[0][2] - e[2][2] * e[0][1];
        c31[1] = e[2][2] * e[0][0] - e[2][0] * e[0][2];
        c31[2] = e[2][0] * e[0][1] - e[2][1] * e[0][0];
        c12[0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
        c12[1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
        c12[2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
        const double det = e[0][0] * c23[0] + e[0][1] * c23[1] + e[0][2] * c23[2];
        const double id = 1.0 / det;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            G[1][r] = c23[r] * id;
            G[2][r] = c31[r] * id;
            G[3][r] = c12[r] * id;
            G[0][r] = -(G[1][r] + G[2][r] + G[3][r]);
        }
        return det;
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
    return !(det * det > tol * tol * prod) || !finite(det);
}

template <int D>
__device__ __forceinline__ void load_vertices(const int32_t *__restrict__ conn, const double *__restrict__ coords,
                                              int e, double (&x)[D + 1][D]) {
    int v[D + 1];
    if constexpr (D == 3) {
        const int4 q = *reinterpret_cast<const int4 *>(conn + 4 * (size_t)e);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = conn[3 * (size_t)e + a];
    }
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) x[a][c] = coords[(size_t)v[a] * D + c];
}

// ---------------------------------------------------------------- P1 scalar forms

template <int D, typename T, bool MASS>
__global__ __launch_bounds__(kP1Threads) void p1_assemble_kernel(
    const int32_t *__restrict__ blk_row, const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ node_rp, const int32_t *__restrict__ seg_ptr, const uint16_t *__restrict__ slot,
    const int32_t *__restrict__ conn, const double *__restrict__ coords, const T *__restrict__ coef,
    const T *__restrict__ load, T *__restrict__ values, T *__restrict__ rhs, int32_t *__restrict__ status,
    int nblk) {
    constexpr int K = D + 1;
    __shared__ T sK[kP1BlockCap * K];
    __shared__ T sF[kP1BlockCap];

    const int blk = xcd_swizzle(blockIdx.x, nblk);
    const int r0 = blk_row[blk], r1 = blk_row[blk + 1];
    const int q0 = inc_ptr[r0], q1 = inc_ptr[r1];
    const int np = q1 - q0;

    // ---- Map: row a of K_e (and F_e[a]) for every pair of the block
    for (int t = threadIdx.x; t < np; t += kP1Threads) {
        const int code = inc[q0 + t];
        const int e = code / K, a = code - e * K;
        double x[K][D], G[K][D];
        load_vertices<D>(conn, coords, e, x);
        const double det = p1_gradients<D>(x, G);
        const double adet = fabs(det);
        bool bad = numerically_singular<D>(x, det);
        if constexpr (MASS) {
            // M_ab = sum_q w_q |det J| phi_a(x_q) phi_b(x_q), degree-2 rule
            using R = Deg2Rule<D>;
#pragma unroll
            for (int b = 0; b < K; ++b) {
                double m = 0.0;
#pragma unroll
                for (int q = 0; q < R::Q; ++q) {
                    const double pa = (a == q) ? R::hi : R::lo;
                    const double pb = (b == q) ? R::hi : R::lo;
                    m += R::w * pa * pb;
                }
                sK[t * K + b] = (T)(adet * m);
            }
        } else {
            // 1-point centroid rule: the integrand a_e G_a . G_b is constant
            const double ce = (double)coef[e];
            const double fe = load ? (double)load[e] : 0.0;
            bad = bad || !finite(ce) || !finite(fe);
            const double w = adet * RefSimplex<D>::vol;
            const T wc = (T)(w * ce);
            T ga[D];
#pragma unroll
            for (int c = 0; c < D; ++c) ga[c] = (T)(a == 0 ? G[0][c] : a == 1 ? G[1][c] : a == 2 ? G[2][c] : G[K - 1][c]);
#pragma unroll
            for (int b = 0; b < K; ++b) {
                T s = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) s += ga[c] * (T)G[b][c];
                sK[t * K + b] = wc * s;
            }
            sF[t] = (T)(w * fe * (1.0 / K));  // phi_a(centroid) = 1/(d+1)
        }
        if (bad && status) atomicMin(status, e);
    }
    __syncthreads();

    // ---- Reduce: CSR values of the block rows (S_mat projection)
    const int v0 = node_rp[r0], v1 = node_rp[r1];
    for (int p = v0 + threadIdx.x; p < v1; p += kP1Threads) {
        const int s0 = seg_ptr[p], s1 = seg_ptr[p + 1];
        T acc = 0;
        for (int s = s0; s < s1; ++s) acc += sK[slot[s]];
        values[p] = acc;
    }
    // ---- Reduce: right-hand side (S_vec projection)
    if (!MASS && rhs) {
        for (int r = r0 + threadIdx.x; r < r1; r += kP1Threads) {
            const int u0 = inc_ptr[r] - q0, u1 = inc_ptr[r + 1] - q0;
            T acc = 0;
            for (int u = u0; u < u1; ++u) acc += sF[u];
            rhs[r] = acc;
        }
    }
}

// ---------------------------------------------------------------- P2 elasticity

constexpr int kP2LanesPerPair = 4;

// grad(phi_n) at a Keast point for P2 node n (vertices 0..3, then edges
// (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)):  vertex p: (4 lambda_p - 1) grad(lambda_p);
// edge (p,r): 4 (lambda_r grad(lambda_p) + lambda_p grad(lambda_r)).
// lam_q(p) is the barycentric coordinate of vertex p at the point.
template <typename T>
__device__ __forceinline__ void p2_grad(int n, int q, const T (&g)[4][3], T hi, T lo, T (&out)[3]) {
    const int p = n < 4 ? n : (n < 7 ? 0 : (n < 9 ? 1 : 2));
    const int r = n < 4 ? n : (n == 4 ? 1 : n == 5 ? 2 : n == 6 ? 3 : n == 7 ? 2 : 3);
    const T lp = (p == q) ? hi : lo;
    const T lr = (r == q) ? hi : lo;
    T gp[3], gr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        gp[c] = p == 0 ? g[0][c] : p == 1 ? g[1][c] : p == 2 ? g[2][c] : g[3][c];
        gr[c] = r == 0 ? g[0][c] : r == 1 ? g[1][c] : r == 2 ? g[2][c] : g[3][c];
    }
    if (n < 4) {
        const T s = (T)4 * lp - (T)1;
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = s * gp[c];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = (T)4 * (lr * gp[c] + lp * gr[c]);
    }
}

// int over the reference tetrahedron of phi_n (degree-2 rule; exact).
__device__ __forceinline__ double p2_ref_integral(int n) {
    using R = Deg2Rule<3>;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (n < 4) {
            const double l = (n == q) ? R::hi : R::lo;
            s += R::w * l * (2.0 * l - 1.0);
        } else {
            const int p = n < 7 ? 0 : (n < 9 ? 1 : 2);
            const int r = n == 4 ? 1 : n == 5 ? 2 : n == 6 ? 3 : n == 7 ? 2 : 3;
            s += R::w * 4.0 * ((p == q) ? R::hi : R::lo) * ((r == q) ? R::hi : R::lo);
        }
    }
    return s;
}

template <typename T>
__global__ __launch_bounds__(kP2Threads) void p2_elasticity_kernel(
    const int32_t *__restrict__ blk_row, const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ node_rp, const int32_t *__restrict__ seg_ptr, const uint16_t *__restrict__ slot,
    const int32_t *__restrict__ conn, const double *__restrict__ coords, const T *__restrict__ coef,
    const T *__restrict__ load, T *__restrict__ values, T *__restrict__ rhs, int32_t *__restrict__ status, int nblk,
    int E) {
    constexpr int K = 10;
    __shared__ T sK[kP2BlockCap * K * 9];
    __shared__ T sF[kP2BlockCap * 3];
    __shared__ int sRp[kP2BlockCap + 1];

    const int blk = xcd_swizzle(blockIdx.x, nblk);
    const int r0 = blk_row[blk], r1 = blk_row[blk + 1];
    const int q0 = inc_ptr[r0], q1 = inc_ptr[r1];
    const int np = q1 - q0;
    const int nrows = r1 - r0;
    const int rp0 = node_rp[r0];
    for (int r = threadIdx.x; r <= nrows; r += kP2Threads) sRp[r] = node_rp[r0 + r] - rp0;

    // ---- Map: block row a of K_e (10 blocks of 3x3), split over 4 lanes by column node
    using R = Deg2Rule<3>;
    for (int u = threadIdx.x; u < np * kP2LanesPerPair; u += kP2Threads) {
        const int t = u / kP2LanesPerPair, sub = u - t * kP2LanesPerPair;
        const int code = inc[q0 + t];
        const int e = code / K, a = code - e * K;
        double x[4][3], Gd[4][3];
        load_vertices<3>(conn, coords, e, x);
        const double det = p1_gradients<3>(x, Gd);
        const double adet = fabs(det);
        const double lam_d = (double)coef[e], mu_d = (double)coef[(size_t)E + e];
        bool bad = numerically_singular<3>(x, det) || !finite(lam_d) || !finite(mu_d);
        T g[4][3];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int c = 0; c < 3; ++c) g[p][c] = (T)Gd[p][c];
        const T hi = (T)R::hi, lo = (T)R::lo;
        const T w = (T)(adet * R::w);
        const T lam = (T)lam_d, mu = (T)mu_d;
        T ga[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) p2_grad<T>(a, q, g, hi, lo, ga[q]);
        for (int b = sub; b < K; b += kP2LanesPerPair) {
            // D_ab = sum_q w_q |det J| grad(phi_a) grad(phi_b)^T
            T Dm[3][3] = {};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T gb[3];
                p2_grad<T>(b, q, g, hi, lo, gb);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) Dm[c][cc] += w * ga[q][c] * gb[cc];
            }
            // Hooke: block[c][c'] = lam D[c][c'] + mu (D[c'][c] + delta_cc' tr D)
            const T tr = Dm[0][0] + Dm[1][1] + Dm[2][2];
            T *dst = sK + (t * K + b) * 9;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) dst[c * 3 + cc] = lam * Dm[c][cc] + mu * (Dm[cc][c] + (c == cc ? tr : (T)0));
        }
        if (sub == 0) {
            if (load) {
                const double ia = adet * p2_ref_integral(a);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double bc = (double)load[(size_t)e * 3 + c];
                    bad = bad || !finite(bc);
                    sF[t * 3 + c] = (T)(bc * ia);
                }
            }
            if (bad && status) atomicMin(status, e);
        }
    }
    __syncthreads();

    // ---- Reduce: the block's scalar values are the contiguous range [9 rp0, 9 rp1)
    const int nval = 9 * sRp[nrows];
    T *out = values + 9 * (size_t)rp0;
    for (int v = threadIdx.x; v < nval; v += kP2Threads) {
        int lo_r = 0, hi_r = nrows - 1;  // last row with 9 * sRp[r] <= v
        while (lo_r < hi_r) {
            const int mid = (lo_r + hi_r + 1) >> 1;
            if (9 * sRp[mid] <= v) lo_r = mid;
            else hi_r = mid - 1;
        }
        const int r = lo_r;
        const int m = sRp[r + 1] - sRp[r];
        const int off = v - 9 * sRp[r];
        const int c = off / (3 * m);
        const int rem = off - c * 3 * m;
        const int jpos = rem / 3;
        const int cc = rem - 3 * jpos;
        const int pnode = rp0 + sRp[r] + jpos;
        const int s0 = seg_ptr[pnode], s1 = seg_ptr[pnode + 1];
        T acc = 0;
        for (int s = s0; s < s1; ++s) acc += sK[(int)slot[s] * 9 + c * 3 + cc];
        out[v] = acc;
    }
    if (rhs && load) {
        for (int u = threadIdx.x; u < 3 * nrows; u += kP2Threads) {
            const int r = u / 3, c = u - 3 * r;
            const int u0 = inc_ptr[r0 + r] - q0, u1 = inc_ptr[r0 + r + 1] - q0;
            T acc = 0;
            for (int s = u0; s < u1; ++s) acc += sF[s * 3 + c];
            rhs[3 * (size_t)(r0 + r) + c] = acc;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <int D, typename T, bool MASS>
static hipError_t launch_p1_t(const tg_pattern &p, const double *coords, const void *coef, const void *load,
                              void *values, void *rhs, int32_t *status, hipStream_t s) {
    const DevicePattern &d = p.dev;
    const int nblk = (int)p.host.n_blocks();
    hipLaunchKernelGGL((p1_assemble_kernel<D, T, MASS>), dim3(nblk), dim3(kP1Threads), 0, s, d.blk_row, d.inc_ptr,
                       d.inc, d.node_rp, d.seg_ptr, d.slot, d.conn, coords, (const T *)coef, (const T *)load,
                       (T *)values, (T *)rhs, status, nblk);
    return hipGetLastError();
}

hipError_t launch_assemble_p1(const tg_pattern &p, tg_form form, tg_dtype dtype, const double *coords,
                              const void *coef, const void *load, void *values, void *rhs, int32_t *status,
                              hipStream_t s) {
    const bool mass = form == TG_MASS;
    const int D = p.host.dim;
#define TG_P1_CASE(DD, TT)                                                                               \
    if (D == DD) {                                                                                       \
        if (mass) return launch_p1_t<DD, TT, true>(p, coords, coef, load, values, rhs, status, s);      \
        return launch_p1_t<DD, TT, false>(p, coords, coef, load, values, rhs, status, s);                \
    }
    if (dtype == TG_F64) {
        TG_P1_CASE(2, double)
        TG_P1_CASE(3, double)
    } else {
        TG_P1_CASE(2, float)
        TG_P1_CASE(3, float)
    }
#undef TG_P1_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_assemble_p2(const tg_pattern &p, tg_dtype dtype, const double *coords, const void *coef,
                              const void *load, void *values, void *rhs, int32_t *status, hipStream_t s) {
    const DevicePattern &d = p.dev;
    const int nblk = (int)p.host.n_blocks();
    const int E = (int)p.host.E;
    if (dtype == TG_F64)
        hipLaunchKernelGGL(p2_elasticity_kernel<double>, dim3(nblk), dim3(kP2Threads), 0, s, d.blk_row, d.inc_ptr,
                           d.inc, d.node_rp, d.seg_ptr, d.slot, d.conn, coords, (const double *)coef,
                           (const double *)load, (double *)values, (double *)rhs, status, nblk, E);
    else
        hipLaunchKernelGGL(p2_elasticity_kernel<float>, dim3(nblk), dim3(kP2Threads), 0, s, d.blk_row, d.inc_ptr,
                           d.inc, d.node_rp, d.seg_ptr, d.slot, d.conn, coords, (const float *)coef,
                           (const float *)load, (float *)values, (float *)rhs, status, nblk, E);
    return hipGetLastError();
}

}  // namespace tg
