// Dirichlet elimination, SpMV and Jacobi-preconditioned CG on the assembled
// CSR system (TensorGalerkin Sec. B.1.2: Jacobi-preconditioned Krylov solve of
// the condensed system, stopped on ||K u - f|| / ||f||).
//
// Reductions are deterministic: each block reduces its grid-stride share in a
// fixed order, writes one partial, and every consumer sums the partials in the
// same fixed order, so the solver is bitwise reproducible without atomics.
#include <algorithm>
#include <cmath>

#include "tg_internal.h"

namespace tg {
namespace {

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = kVecThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Sum of partials[0..n) (stride `stride`) in a fixed order; same value in every block.
__device__ __forceinline__ double sum_partials(const double *__restrict__ partials, int n, int stride, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kVecThreads) v += partials[(size_t)i * stride];
    return block_sum(v, sh);
}

template <typename T>
__global__ __launch_bounds__(256) void dirichlet_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col_idx,
                                                        const uint8_t *__restrict__ constrained, T *__restrict__ values,
                                                        T *__restrict__ rhs, const T *__restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
    if (constrained[i]) {
        for (int p = p0; p < p1; ++p) values[p] = (col_idx[p] == i) ? (T)1 : (T)0;
        if (rhs) rhs[i] = g ? g[i] : (T)0;
    } else {
        double acc = rhs ? (double)rhs[i] : 0.0;
        for (int p = p0; p < p1; ++p) {
            const int j = col_idx[p];
            if (constrained[j]) {
                if (g) acc -= (double)values[p] * (double)g[j];
                values[p] = (T)0;
            }
        }
        if (rhs && g) rhs[i] = (T)acc;
    }
}

// Row i of K x, accumulated in FP64 by a group of G lanes in a fixed pattern.
template <typename T, int G>
__device__ __forceinline__ double row_dot(int i, int lane, const int32_t *__restrict__ row_ptr,
                                          const int32_t *__restrict__ col_idx, const T *__restrict__ values,
                                          const T *__restrict__ x) {
    const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
    double acc = 0.0;
    for (int p = p0 + lane; p < p1; p += G) acc += (double)values[p] * (double)x[col_idx[p]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    return acc;
}

template <typename T, int G>
__global__ __launch_bounds__(256) void spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx, const T *__restrict__ values,
                                                   const T *__restrict__ x, T *__restrict__ y) {
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (256 / G);
    for (int i = blockIdx.x * (256 / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<T, G>(i, lane, row_ptr, col_idx, values, x);
        if (lane == 0) y[i] = (T)v;
    }
}

// ---------------------------------------------------------------- PCG kernels
// Workspace layout (T elements of n each): r, z, p, q, dinv.

template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_init_kernel(int n, const T *__restrict__ b, T *__restrict__ x,
                                                               T *__restrict__ r, T *__restrict__ z,
                                                               T *__restrict__ p, T *__restrict__ dinv,
                                                               const T *__restrict__ values,
                                                               const int32_t *__restrict__ diag_pos,
                                                               double *__restrict__ partials) {
    __shared__ double sh[kVecThreads];
    double rz = 0.0, bb = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        const T bi = b[i];
        const T di = (T)1 / values[diag_pos[i]];
        const T zi = di * bi;
        x[i] = (T)0;
        r[i] = bi;
        z[i] = zi;
        p[i] = zi;
        dinv[i] = di;
        rz += (double)bi * (double)zi;
        bb += (double)bi * (double)bi;
    }
    rz = block_sum(rz, sh);
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = rz;
        partials[kMaxPartials + blockIdx.x] = bb;
    }
}

__global__ __launch_bounds__(kVecThreads) void pcg_init_finish_kernel(int nparts, const double *__restrict__ partials,
                                                                      PcgState *__restrict__ st, double rtol2) {
    __shared__ double sh[kVecThreads];
    const double rz = sum_partials(partials, nparts, 1, sh);
    const double bb = sum_partials(partials + kMaxPartials, nparts, 1, sh);
    if (threadIdx.x == 0) {
        st->rz[0] = rz;
        st->rz[1] = 0.0;
        st->bb = bb;
        st->rr = bb;
        st->tol2 = rtol2 * bb;
        st->done = (bb == 0.0) ? 1 : 0;
        st->iters = 0;
    }
}

// q = K p and a partial of p.q per block.
template <typename T, int G>
__global__ __launch_bounds__(256) void pcg_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col_idx,
                                                       const T *__restrict__ values, const T *__restrict__ p,
                                                       T *__restrict__ q, double *__restrict__ partials,
                                                       const PcgState *__restrict__ st) {
    __shared__ double sh[kVecThreads];
    if (st->done) return;  // written only by earlier launches: the same value for every wave
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (256 / G);
    double pq = 0.0;
    for (int i = blockIdx.x * (256 / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<T, G>(i, lane, row_ptr, col_idx, values, p);
        if (lane == 0) {
            const T qi = (T)v;
            q[i] = qi;
            pq += (double)p[i] * (double)qi;
        }
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) partials[2 * kMaxPartials + blockIdx.x] = pq;
}

// alpha = rz / pq; x += alpha p; r -= alpha q; z = D^{-1} r; partials of r.z and r.r
template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_update_xr_kernel(int n, int n_pq, T *__restrict__ x,
                                                                    T *__restrict__ r, T *__restrict__ z,
                                                                    const T *__restrict__ p, const T *__restrict__ q,
                                                                    const T *__restrict__ dinv,
                                                                    double *__restrict__ partials,
                                                                    const PcgState *__restrict__ st, int it) {
    __shared__ double sh[kVecThreads];
    if (st->done) return;  // written only by earlier launches: the same value for every wave
    const double pq = sum_partials(partials + 2 * kMaxPartials, n_pq, 1, sh);
    const double alpha = st->rz[it & 1] / pq;
    const T a = (T)alpha;
    double rz = 0.0, rr = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        const T ri = r[i] - a * q[i];
        x[i] += a * p[i];
        const T zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = rz;
        partials[kMaxPartials + blockIdx.x] = rr;
    }
}

// beta = rz_new / rz; p = z + beta p; stop test on ||r||^2 <= rtol^2 ||b||^2.
// `done` is not read here by the grid: every block takes the stop decision
// from the same partials.  Only thread 0 of block 0 reads and writes `done`
// and `iters`, so no block races with a writer inside this launch.  Once
// converged, pcg_update_xr skips and leaves the partials of the converged
// iteration in place, so later launches take the same decision again.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_update_p_kernel(int n, int nparts, const T *__restrict__ z,
                                                                   T *__restrict__ p,
                                                                   const double *__restrict__ partials,
                                                                   PcgState *__restrict__ st, int it) {
    __shared__ double sh[kVecThreads];
    const double rz_new = sum_partials(partials, nparts, 1, sh);
    const double rr = sum_partials(partials + kMaxPartials, nparts, 1, sh);
    if (rr <= st->tol2) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && !st->done) {
            st->rr = rr;
            st->done = 1;
            st->iters = it + 1;
        }
        return;
    }
    const T beta = (T)(rz_new / st->rz[it & 1]);
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) p[i] = z[i] + beta * p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rz[(it + 1) & 1] = rz_new;
        st->rr = rr;
    }
}

// partials of ||b - K x||^2
template <typename T, int G>
__global__ __launch_bounds__(256) void residual_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col_idx,
                                                       const T *__restrict__ values, const T *__restrict__ x,
                                                       const T *__restrict__ b, double *__restrict__ partials) {
    __shared__ double sh[kVecThreads];
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (256 / G);
    double acc = 0.0;
    for (int i = blockIdx.x * (256 / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<T, G>(i, lane, row_ptr, col_idx, values, x);
        if (lane == 0) {
            const double ri = (double)b[i] - v;
            acc += ri * ri;
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kVecThreads) void residual_finish_kernel(int nparts, const double *__restrict__ partials,
                                                                      PcgState *__restrict__ st) {
    __shared__ double sh[kVecThreads];
    const double rr = sum_partials(partials, nparts, 1, sh);
    if (threadIdx.x == 0) st->rr = rr;  // true residual, read back by the host
}

int vec_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxPartials, (n + 255) / 256)); }

template <int G>
int spmv_blocks(int64_t n) {
    const int64_t rows_per_block = 256 / G;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxPartials, (n + rows_per_block - 1) / rows_per_block));
}

template <typename T>
hipError_t launch_dirichlet_t(const tg_pattern &pt, void *values, void *rhs, const void *g, hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    hipLaunchKernelGGL(dirichlet_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, pt.dev.row_ptr,
                       pt.dev.col_idx, pt.dev.constrained, (T *)values, (T *)rhs, (const T *)g);
    return hipGetLastError();
}

template <typename T, int G>
hipError_t launch_spmv_t(const tg_pattern &pt, const void *values, const void *x, void *y, hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    hipLaunchKernelGGL((spmv_kernel<T, G>), dim3(spmv_blocks<G>(n)), dim3(256), 0, s, n, pt.dev.row_ptr,
                       pt.dev.col_idx, (const T *)values, (const T *)x, (T *)y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv_g(const tg_pattern &pt, const void *values, const void *x, void *y, hipStream_t s) {
    switch (pt.dev.spmv_group) {
        case 4: return launch_spmv_t<T, 4>(pt, values, x, y, s);
        case 8: return launch_spmv_t<T, 8>(pt, values, x, y, s);
        case 16: return launch_spmv_t<T, 16>(pt, values, x, y, s);
        default: return launch_spmv_t<T, 32>(pt, values, x, y, s);
    }
}

template <typename T, int G>
tg_status run_pcg_t(const tg_pattern &pt, const T *values, const T *b, T *x, double rtol, int max_iter,
                    int check_every, int32_t *iters, double *relres, hipStream_t s, std::string &msg) {
    const DevicePattern &d = pt.dev;
    const int n = (int)pt.host.n_dofs;
    T *r = (T *)d.work;
    T *z = r + n;
    T *p = z + n;
    T *q = p + n;
    T *dinv = q + n;
    const int nb = vec_blocks(n);
    const int ns = spmv_blocks<G>(n);
    hipError_t err;
#define TG_CHECK(call)                               \
    do {                                             \
        err = (call);                                \
        if (err != hipSuccess) {                     \
            msg = hipGetErrorString(err);            \
            return TG_E_HIP;                         \
        }                                            \
    } while (0)
    hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(nb), dim3(kVecThreads), 0, s, n, b, x, r, z, p, dinv, values,
                       d.diag_pos, d.partials);
    hipLaunchKernelGGL(pcg_init_finish_kernel, dim3(1), dim3(kVecThreads), 0, s, nb, d.partials, d.state,
                       rtol * rtol);
    TG_CHECK(hipGetLastError());
    int it = 0;
    bool done = false;
    while (it < max_iter && !done) {
        hipLaunchKernelGGL((pcg_spmv_kernel<T, G>), dim3(ns), dim3(256), 0, s, n, d.row_ptr, d.col_idx, values, p,
                           q, d.partials, d.state);
        hipLaunchKernelGGL(pcg_update_xr_kernel<T>, dim3(nb), dim3(kVecThreads), 0, s, n, ns, x, r, z, p, q, dinv,
                           d.partials, d.state, it);
        hipLaunchKernelGGL(pcg_update_p_kernel<T>, dim3(nb), dim3(kVecThreads), 0, s, n, nb, z, p, d.partials,
                           d.state, it);
        TG_CHECK(hipGetLastError());
        ++it;
        if (it % check_every == 0 || it == max_iter) {
            TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            TG_CHECK(hipStreamSynchronize(s));
            done = d.host_state->done != 0;
        }
    }
    if (!done) {  // converged at initialisation (b = 0) is caught here too
        TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        TG_CHECK(hipStreamSynchronize(s));
        done = d.host_state->done != 0;
    }
    const int32_t its = done ? d.host_state->iters : max_iter;
    const double bb = d.host_state->bb;
    hipLaunchKernelGGL((residual_kernel<T, G>), dim3(ns), dim3(256), 0, s, n, d.row_ptr, d.col_idx, values, x, b,
                       d.partials);
    hipLaunchKernelGGL(residual_finish_kernel, dim3(1), dim3(kVecThreads), 0, s, ns, d.partials, d.state);
    TG_CHECK(hipGetLastError());
    TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    TG_CHECK(hipStreamSynchronize(s));
#undef TG_CHECK
    if (iters) *iters = its;
    if (relres) *relres = bb > 0.0 ? std::sqrt(d.host_state->rr / bb) : std::sqrt(d.host_state->rr);
    if (!done) {
        msg = "PCG did not reach rtol within max_iter iterations";
        return TG_E_NOCONV;
    }
    return TG_OK;
}

template <typename T>
tg_status run_pcg_g(const tg_pattern &pt, const void *values, const void *rhs, void *x, double rtol, int max_iter,
                    int check_every, int32_t *iters, double *relres, hipStream_t s, std::string &msg) {
    const T *v = (const T *)values;
    const T *b = (const T *)rhs;
    T *xx = (T *)x;
    switch (pt.dev.spmv_group) {
        case 4: return run_pcg_t<T, 4>(pt, v, b, xx, rtol, max_iter, check_every, iters, relres, s, msg);
        case 8: return run_pcg_t<T, 8>(pt, v, b, xx, rtol, max_iter, check_every, iters, relres, s, msg);
        case 16: return run_pcg_t<T, 16>(pt, v, b, xx, rtol, max_iter, check_every, iters, relres, s, msg);
        default: return run_pcg_t<T, 32>(pt, v, b, xx, rtol, max_iter, check_every, iters, relres, s, msg);
    }
}

}  // namespace

hipError_t launch_dirichlet(const tg_pattern &p, tg_dtype dtype, void *values, void *rhs, const void *g,
                            hipStream_t s) {
    return dtype == TG_F64 ? launch_dirichlet_t<double>(p, values, rhs, g, s)
                           : launch_dirichlet_t<float>(p, values, rhs, g, s);
}

hipError_t launch_spmv(const tg_pattern &p, tg_dtype dtype, const void *values, const void *x, void *y,
                       hipStream_t s) {
    return dtype == TG_F64 ? launch_spmv_g<double>(p, values, x, y, s) : launch_spmv_g<float>(p, values, x, y, s);
}

tg_status run_pcg(const tg_pattern &p, tg_dtype dtype, const void *values, const void *rhs, void *x, double rtol,
                  int32_t max_iter, int32_t check_every, int32_t *iters, double *relres, hipStream_t s,
                  std::string &msg) {
    return dtype == TG_F64
               ? run_pcg_g<double>(p, values, rhs, x, rtol, max_iter, check_every, iters, relres, s, msg)
               : run_pcg_g<float>(p, values, rhs, x, rtol, max_iter, check_every, iters, relres, s, msg);
}

}  // namespace tg
