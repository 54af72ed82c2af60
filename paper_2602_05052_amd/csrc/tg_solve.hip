// Dirichlet elimination, SpMV and Jacobi-preconditioned CG on the assembled
// CSR system (TensorGalerkin Sec. B.1.2: Jacobi-preconditioned Krylov solve of
// the condensed system, stopped on ||K u - f|| / ||f||).
//
// One CG iteration is two kernels of at most 512 blocks of 1024 threads:
//   pcg_spmv   : stop test on r.r, beta = r.z / r.z_prev, p = z + beta p
//                (formed on the fly into the other half of a double buffer),
//                q = K p and per-block partials of p.q;
//   pcg_update : alpha = r.z / p.q, x += alpha p, r -= alpha q, z = D^{-1} r,
//                per-block partials of r.z and r.r.
// Every scalar (alpha, beta, the stop decision) is recomputed by every block
// from the previous kernel's partials, summed in one fixed order, so all
// blocks agree bitwise and the solver is reproducible with no atomics, no
// fences and no extra launches.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tg_internal.h"

namespace tg {
namespace {

constexpr int kWaves = kVecThreads / 64;

// Sum over the block in a fixed order: butterfly within each wave (every lane
// ends with the same bits: a + b == b + a), then the wave sums in index order.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// Sum of partials[0 .. n), n <= kVecThreads, identical in every block.
__device__ __forceinline__ double sum_partials(const double *__restrict__ partials, int n, double *sh) {
    return block_sum((int)threadIdx.x < n ? partials[threadIdx.x] : 0.0, sh);
}

__device__ __forceinline__ double *part(double *base, int which) { return base + (size_t)which * kMaxGrid; }

template <typename T>
__global__ __launch_bounds__(256) void dirichlet_kernel(int nrows, const int32_t *__restrict__ rows,
                                                        const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col_idx,
                                                        const uint8_t *__restrict__ constrained, T *__restrict__ values,
                                                        T *__restrict__ rhs, const T *__restrict__ g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrows) return;
    const int i = rows[k];
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

// Row i of K y, accumulated in FP64 by a group of G lanes in a fixed pattern,
// where y_j = z_j + beta p_j if DIR, else y_j = x_j.
template <typename T, int G, bool DIR>
__device__ __forceinline__ double row_dot(int i, int lane, const int32_t *__restrict__ row_ptr,
                                          const int32_t *__restrict__ col_idx, const T *__restrict__ values,
                                          const T *__restrict__ x, const T *__restrict__ p, T beta) {
    const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
    double acc = 0.0;
    for (int q = p0 + lane; q < p1; q += G) {
        const int j = col_idx[q];
        const T y = DIR ? x[j] + beta * p[j] : x[j];
        acc += (double)values[q] * (double)y;
    }
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
        const double v = row_dot<T, G, false>(i, lane, row_ptr, col_idx, values, x, nullptr, (T)0);
        if (lane == 0) y[i] = (T)v;
    }
}

// ---------------------------------------------------------------- PCG kernels
// Workspace (T elements of n each): r, z, pA, pB, q, dinv.

template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_init_kernel(int n, const T *__restrict__ b, T *__restrict__ x,
                                                               T *__restrict__ r, T *__restrict__ z,
                                                               T *__restrict__ p, T *__restrict__ dinv,
                                                               const T *__restrict__ values,
                                                               const int32_t *__restrict__ diag_pos,
                                                               double *__restrict__ partials) {
    __shared__ double sh[kWaves];
    double rz = 0.0, bb = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        const T bi = b[i];
        const T di = (T)1 / values[diag_pos[i]];
        const T zi = di * bi;
        x[i] = (T)0;
        r[i] = bi;
        z[i] = zi;
        p[i] = (T)0;
        dinv[i] = di;
        rz += (double)bi * (double)zi;
        bb += (double)bi * (double)bi;
    }
    rz = block_sum(rz, sh);
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        part(partials, kRZ0)[blockIdx.x] = rz;
        part(partials, kBB)[blockIdx.x] = bb;
    }
}

// Stop test on the residual of the last update, then p_new = z + beta p_old,
// q = K p_new and partials of p.q.  CHECK_ONLY launches stop after the test.
// n_prev: number of partials written by the previous kernel (init or update).
template <typename T, int G, bool CHECK_ONLY>
__global__ __launch_bounds__(kVecThreads) void pcg_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col_idx,
                                                               const T *__restrict__ values, const T *__restrict__ z,
                                                               const T *__restrict__ p_old, T *__restrict__ p_new,
                                                               T *__restrict__ q, double *__restrict__ partials,
                                                               PcgState *__restrict__ st, int it, int n_prev,
                                                               double rtol2) {
    __shared__ double sh[kWaves];
    if (st->done) return;  // written only by earlier launches: the same value for every wave
    double tol2, rr;
    if (it == 0) {
        const double bb = sum_partials(part(partials, kBB), n_prev, sh);
        tol2 = rtol2 * bb;
        rr = bb;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->bb = bb;
            st->tol2 = tol2;
        }
    } else {
        tol2 = st->tol2;
        rr = sum_partials(part(partials, kRR), n_prev, sh);
    }
    if (rr <= tol2) {  // the same decision in every block
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->iters = it;
        }
        return;
    }
    if (CHECK_ONLY) return;
    T beta = (T)0;
    if (it > 0) {
        const double rz = sum_partials(part(partials, kRZ0 + (it & 1)), n_prev, sh);
        const double rz_prev = sum_partials(part(partials, kRZ0 + ((it + 1) & 1)), n_prev, sh);
        beta = (T)(rz / rz_prev);
    }
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kVecThreads / G);
    double pq = 0.0;
    for (int i = blockIdx.x * (kVecThreads / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<T, G, true>(i, lane, row_ptr, col_idx, values, z, p_old, beta);
        if (lane == 0) {
            const T pi = z[i] + beta * p_old[i];
            const T qi = (T)v;
            p_new[i] = pi;
            q[i] = qi;
            pq += (double)pi * (double)qi;
        }
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) part(partials, kPQ)[blockIdx.x] = pq;
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = D^{-1} r; partials of r.z (next buffer) and r.r
template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_update_kernel(int n, T *__restrict__ x, T *__restrict__ r,
                                                                 T *__restrict__ z, const T *__restrict__ p,
                                                                 const T *__restrict__ q, const T *__restrict__ dinv,
                                                                 double *__restrict__ partials,
                                                                 const PcgState *__restrict__ st, int it,
                                                                 int n_pq, int n_rz) {
    __shared__ double sh[kWaves];
    if (st->done) return;  // written only by earlier launches
    const double pq = sum_partials(part(partials, kPQ), n_pq, sh);
    const double rz = sum_partials(part(partials, kRZ0 + (it & 1)), n_rz, sh);
    const T a = (T)(rz / pq);
    double rzn = 0.0, rr = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        const T ri = r[i] - a * q[i];
        x[i] += a * p[i];
        const T zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        rzn += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    rzn = block_sum(rzn, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part(partials, kRZ0 + ((it + 1) & 1))[blockIdx.x] = rzn;
        part(partials, kRR)[blockIdx.x] = rr;
    }
}

// per-block partials of ||b - K x||^2 (summed on the host in index order)
template <typename T, int G>
__global__ __launch_bounds__(kVecThreads) void residual_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col_idx,
                                                               const T *__restrict__ values, const T *__restrict__ x,
                                                               const T *__restrict__ b, double *__restrict__ partials) {
    __shared__ double sh[kWaves];
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kVecThreads / G);
    double acc = 0.0;
    for (int i = blockIdx.x * (kVecThreads / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<T, G, false>(i, lane, row_ptr, col_idx, values, x, nullptr, (T)0);
        if (lane == 0) {
            const double ri = (double)b[i] - v;
            acc += ri * ri;
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part(partials, kRR)[blockIdx.x] = acc;
}

int vec_blocks(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxGrid, (n + kVecThreads - 1) / kVecThreads));
}

template <int G>
int spmv_blocks(int64_t n) {
    const int64_t rows_per_block = kVecThreads / G;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxGrid, (n + rows_per_block - 1) / rows_per_block));
}

template <int G>
int spmv_blocks_256(int64_t n) {
    const int64_t rows_per_block = 256 / G;
    return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + rows_per_block - 1) / rows_per_block));
}

template <typename T>
hipError_t launch_dirichlet_t(const tg_pattern &pt, void *values, void *rhs, const void *g, hipStream_t s) {
    const int nr = (int)pt.dev.n_dir_rows;
    if (nr == 0) return hipSuccess;
    hipLaunchKernelGGL(dirichlet_kernel<T>, dim3((nr + 255) / 256), dim3(256), 0, s, nr, pt.dev.dir_rows,
                       pt.dev.row_ptr, pt.dev.col_idx, pt.dev.constrained, (T *)values, (T *)rhs, (const T *)g);
    return hipGetLastError();
}

template <typename T, int G>
hipError_t launch_spmv_t(const tg_pattern &pt, const void *values, const void *x, void *y, hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    hipLaunchKernelGGL((spmv_kernel<T, G>), dim3(spmv_blocks_256<G>(n)), dim3(256), 0, s, n, pt.dev.row_ptr,
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
    T *pA = z + n;
    T *pB = pA + n;
    T *q = pB + n;
    T *dinv = q + n;
    const int nb = vec_blocks(n);
    const int ns = spmv_blocks<G>(n);
    const double rtol2 = rtol * rtol;
    hipError_t err;
#define TG_CHECK(call)                    \
    do {                                  \
        err = (call);                     \
        if (err != hipSuccess) {          \
            msg = hipGetErrorString(err); \
            return TG_E_HIP;              \
        }                                 \
    } while (0)
    // reset the host-visible state (done = 0) with a copy, not a memset: a caller may capture this stream
    d.host_state->done = 0;
    d.host_state->iters = 0;
    TG_CHECK(hipMemcpyAsync(d.state, d.host_state, sizeof(PcgState), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(nb), dim3(kVecThreads), 0, s, n, b, x, r, z, pA, dinv, values,
                       d.diag_pos, d.partials);
    TG_CHECK(hipGetLastError());
    int it = 0;
    bool done = false;
    while (it < max_iter && !done) {
        T *p_old = (it & 1) ? pB : pA;
        T *p_new = (it & 1) ? pA : pB;
        hipLaunchKernelGGL((pcg_spmv_kernel<T, G, false>), dim3(ns), dim3(kVecThreads), 0, s, n, d.row_ptr,
                           d.col_idx, values, z, p_old, p_new, q, d.partials, d.state, it, nb, rtol2);
        hipLaunchKernelGGL(pcg_update_kernel<T>, dim3(nb), dim3(kVecThreads), 0, s, n, x, r, z, p_new, q, dinv,
                           d.partials, d.state, it, ns, nb);
        TG_CHECK(hipGetLastError());
        ++it;
        if (it % check_every == 0) {
            TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            TG_CHECK(hipStreamSynchronize(s));
            done = d.host_state->done != 0;
        }
    }
    // stop test on the last update (sets done/iters if it converged)
    hipLaunchKernelGGL((pcg_spmv_kernel<T, G, true>), dim3(1), dim3(kVecThreads), 0, s, n, d.row_ptr, d.col_idx,
                       values, z, pA, pB, q, d.partials, d.state, it, nb, rtol2);
    hipLaunchKernelGGL((residual_kernel<T, G>), dim3(ns), dim3(kVecThreads), 0, s, n, d.row_ptr, d.col_idx, values,
                       x, b, d.partials);
    TG_CHECK(hipGetLastError());
    std::vector<double> host_parts(ns);
    TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    TG_CHECK(hipMemcpyAsync(host_parts.data(), d.partials + (size_t)kRR * kMaxGrid, sizeof(double) * ns,
                            hipMemcpyDeviceToHost, s));
    TG_CHECK(hipStreamSynchronize(s));
#undef TG_CHECK
    done = d.host_state->done != 0;
    double rr = 0.0;
    for (double v : host_parts) rr += v;
    const double bb = d.host_state->bb;
    if (iters) *iters = done ? d.host_state->iters : it;
    if (relres) *relres = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
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
