// Adjoint of P1 assembly (TensorGalerkin Sec. 2, eq. adj) on gfx950.
//
// For a batch of vector triples (lam_m, u_m, w_m) the bilinear quantity
//   Phi = sum_m lam_m^T (A u_m - M w_m),   A = K(c), M, or M + K(c),
// is differentiated with respect to the per-element log-coefficients and the
// vertex coordinates.  This is what a gradient through an assembled system
// needs once the adjoint vectors are known: with A^T lam = dL/du the chain
// rule gives dL/dtheta = -dPhi/dtheta (eq. adj: dL/dK = -lam u^T restricted
// to the pattern).
//
// Per element, with G_a = grad(lambda_a) = C_a / det J (cofactor form) and the
// member sums S_ab = sum_m lam_a u_b (stiffness) and
// t = sum_m sum_ab lam_a (mu u_b - w_b) (1 + delta_ab) (mass; mu = 1 when A
// holds M):
//   dPhi/dlog c    = c |T| tr P,                P = sum_ab S_ab G_a G_b^T
//   dPhi/dx_v      = c |T| [G_v tr P - (P + P^T) G_v] + Phi_M G_v,
//   Phi_M          = |T| t / ((d+1)(d+2))      (the P1 mass matrix of SM A.1)
// from d|T|/dx_v = |T| G_v and d(G_a)/dx_v = -G_v G_a^T (affine map).
//
// Kernel 1 (one lane per element) writes dPhi/dlog c_e and the k vertex
// gradients of the element to a staging array [E][k][d].  Kernel 2 (one lane
// per vertex) is the S_vec-type Reduce of Alg. 2: it sums the staged entries
// of the vertex's incident (element, local vertex) pairs in ascending element
// order, so the result is bitwise reproducible and needs no atomics.
#include <mutex>

#include "tg_device.h"

namespace tg {
namespace {

constexpr int kAdjThreads = 256;

template <int D, typename T, int FORM>
__global__ __launch_bounds__(kAdjThreads) void p1_adjoint_element_kernel(
    const int32_t *__restrict__ conn, const double *__restrict__ coords, const T *__restrict__ coef,
    const T *__restrict__ lam, const T *__restrict__ u, const T *__restrict__ w, unsigned stride, int nbatch,
    unsigned n_elem, double scale, double *__restrict__ dlogc, double *__restrict__ stage,
    int32_t *__restrict__ status) {
    constexpr int K = D + 1;
    constexpr bool HAS_K = FORM != TG_MASS;           // A contains K(c)
    constexpr bool HAS_MU = FORM != TG_LAPLACE;       // A contains M
    const unsigned e = blockIdx.x * kAdjThreads + threadIdx.x;
    if (e >= n_elem) return;

    unsigned v[K];
#pragma unroll
    for (int a = 0; a < K; ++a) v[a] = (unsigned)ldg(conn, (unsigned)K * e + a);
    double x[K][D];
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int i = 0; i < D; ++i) x[a][i] = ldg(coords, v[a] * D + i);
    double C[K][D];
    const double det = p1_cofactors<D>(x, C);
    const double c = HAS_K ? (double)ldg(coef, e) : 0.0;
    const bool bad = numerically_singular<D>(x, det) || !finite(c);
    if (bad && status) atomicMin(status, (int)e);

    double S[K][K];
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b < K; ++b) S[a][b] = 0.0;
    double t = 0.0;
    for (int m = 0; m < nbatch; ++m) {
        const unsigned off = (unsigned)m * stride;
        double l[K], uu[K], dd[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            l[a] = (double)ldg(lam, off + v[a]);
            uu[a] = (double)ldg(u, off + v[a]);
            dd[a] = (HAS_MU ? uu[a] : 0.0) - (w ? (double)ldg(w, off + v[a]) : 0.0);
        }
        if constexpr (HAS_K) {
#pragma unroll
            for (int a = 0; a < K; ++a)
#pragma unroll
                for (int b = 0; b < K; ++b) S[a][b] += l[a] * uu[b];
        }
        double sl = 0.0, sd = 0.0, ld = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            sl += l[a];
            sd += dd[a];
            ld += l[a] * dd[a];
        }
        t += sl * sd + ld;
    }

    // P~ = sum_ab S_ab C_a C_b^T = det^2 P;  H_b = sum_a S_ab C_a.
    double Pc[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) Pc[i][j] = 0.0;
    if constexpr (HAS_K) {
#pragma unroll
        for (int b = 0; b < K; ++b) {
            double H[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                H[i] = 0.0;
#pragma unroll
                for (int a = 0; a < K; ++a) H[i] += S[a][b] * C[a][i];
            }
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) Pc[i][j] += H[i] * C[b][j];
        }
    }
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) tr += Pc[i][i];

    const double rd = 1.0 / det;
    const double adet = fabs(det);
    const double kfac = c * fabs(rd) * RefSimplex<D>::vol;                          // c |T| / det^2
    const double phim = adet * RefSimplex<D>::vol * t * (1.0 / ((D + 1) * (D + 2)));  // Phi_M
    if (dlogc) stg(dlogc, e, HAS_K ? scale * kfac * tr : 0.0);
    const double diag = kfac * tr + phim;
#pragma unroll
    for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double q = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) q += (Pc[i][j] + Pc[j][i]) * C[a][j];
            stg(stage, (e * K + a) * D + i, scale * rd * (diag * C[a][i] - kfac * q));
        }
    }
}

template <int D>
__global__ __launch_bounds__(kAdjThreads) void vertex_reduce_kernel(const int32_t *__restrict__ inc_ptr,
                                                                    const int32_t *__restrict__ inc,
                                                                    const double *__restrict__ stage, unsigned nv,
                                                                    double *__restrict__ out) {
    const unsigned v = blockIdx.x * kAdjThreads + threadIdx.x;
    if (v >= nv) return;
    const int p0 = ldg(inc_ptr, v), p1 = ldg(inc_ptr, v + 1);
    double acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = 0.0;
    for (int q = p0; q < p1; ++q) {
        const unsigned code = (unsigned)ldg(inc, (unsigned)q);
#pragma unroll
        for (int i = 0; i < D; ++i) acc[i] += ldg(stage, code * D + i);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) stg(out, v * D + i, acc[i]);
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void scaled_exp_kernel(unsigned n, double dt, const double *__restrict__ x,
                                                                 T *__restrict__ y) {
    const unsigned i = blockIdx.x * kAdjThreads + threadIdx.x;
    if (i < n) stg(y, i, (T)(dt * exp(ldg(x, i))));
}

template <int D, typename T, int FORM>
hipError_t launch_adjoint_t(const tg_pattern &p, int nbatch, const double *coords, const void *coef,
                            const void *lam, const void *u, const void *w, int64_t stride, double scale,
                            double *dlogc, double *dcoords, double *stage, int32_t *status, hipStream_t s) {
    const unsigned E = (unsigned)p.host.E, nv = (unsigned)p.host.nv;
    if (E > 0)
        hipLaunchKernelGGL((p1_adjoint_element_kernel<D, T, FORM>), dim3((E + kAdjThreads - 1) / kAdjThreads),
                           dim3(kAdjThreads), 0, s, p.dev.conn, coords, (const T *)coef, (const T *)lam,
                           (const T *)u, (const T *)w, (unsigned)stride, nbatch, E, scale, dlogc, stage, status);
    if (dcoords && nv > 0)
        hipLaunchKernelGGL(vertex_reduce_kernel<D>, dim3((nv + kAdjThreads - 1) / kAdjThreads), dim3(kAdjThreads), 0,
                           s, p.dev.inc_ptr, p.dev.inc, stage, nv, dcoords);
    return hipGetLastError();
}

template <int D, typename T>
hipError_t launch_adjoint_d(const tg_pattern &p, tg_form form, int nbatch, const double *coords, const void *coef,
                            const void *lam, const void *u, const void *w, int64_t stride, double scale,
                            double *dlogc, double *dcoords, double *stage, int32_t *status, hipStream_t s) {
    switch (form) {
        case TG_LAPLACE:
            return launch_adjoint_t<D, T, TG_LAPLACE>(p, nbatch, coords, coef, lam, u, w, stride, scale, dlogc,
                                                      dcoords, stage, status, s);
        case TG_MASS:
            return launch_adjoint_t<D, T, TG_MASS>(p, nbatch, coords, coef, lam, u, w, stride, scale, dlogc, dcoords,
                                                   stage, status, s);
        case TG_MASS_LAPLACE:
            return launch_adjoint_t<D, T, TG_MASS_LAPLACE>(p, nbatch, coords, coef, lam, u, w, stride, scale, dlogc,
                                                           dcoords, stage, status, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_adjoint_p1(const tg_pattern &p, tg_form form, tg_dtype dtype, int nbatch, const double *coords,
                             const void *coef, const void *lam, const void *u, const void *w, int64_t stride,
                             double scale, double *dlogc, double *dcoords, double *stage, int32_t *status,
                             hipStream_t s) {
    if (p.host.dim == 2) {
        if (dtype == TG_F64)
            return launch_adjoint_d<2, double>(p, form, nbatch, coords, coef, lam, u, w, stride, scale, dlogc,
                                               dcoords, stage, status, s);
        return launch_adjoint_d<2, float>(p, form, nbatch, coords, coef, lam, u, w, stride, scale, dlogc, dcoords,
                                          stage, status, s);
    }
    if (dtype == TG_F64)
        return launch_adjoint_d<3, double>(p, form, nbatch, coords, coef, lam, u, w, stride, scale, dlogc, dcoords,
                                           stage, status, s);
    return launch_adjoint_d<3, float>(p, form, nbatch, coords, coef, lam, u, w, stride, scale, dlogc, dcoords,
                                      stage, status, s);
}

// The staging array of the allocation-free adjoint entry point: a file-scope
// device array, so each GPU the library runs on holds its own copy from the
// library's load until the process ends, and no call allocates.  Host code
// never uses the array's name as an address (on the host it is only a stand-in
// symbol): each device's address comes from hipGetSymbolAddress, called once
// per device with that device current.
static __device__ __align__(256) double scratch[kNoAllocStageDoubles];

hipError_t noalloc_stage(double **out) {
    static std::mutex mu;
    static double *addr[kNoAllocMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_scaled_exp(tg_dtype dtype, int64_t n, double dt, const double *x, void *y, hipStream_t s) {
    const unsigned nn = (unsigned)n;
    if (n == 0) return hipSuccess;
    if (dtype == TG_F64)
        hipLaunchKernelGGL(scaled_exp_kernel<double>, dim3((nn + kAdjThreads - 1) / kAdjThreads), dim3(kAdjThreads),
                           0, s, nn, dt, x, (double *)y);
    else
        hipLaunchKernelGGL(scaled_exp_kernel<float>, dim3((nn + kAdjThreads - 1) / kAdjThreads), dim3(kAdjThreads),
                           0, s, nn, dt, x, (float *)y);
    return hipGetLastError();
}

}  // namespace tg
