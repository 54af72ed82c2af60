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
        if (values)
            for (int p = p0; p < p1; ++p) values[p] = (col_idx[p] == i) ? (T)1 : (T)0;
        if (rhs) rhs[i] = g ? g[i] : (T)0;
    } else if (values) {
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
// Each launch serves the slots slots[list[blockIdx.y]] (one CG system each, all
// on the same pattern); blockIdx.x strides over the rows.  A slot's iteration
// is step - start, so systems that joined at different steps share launches.
// Slot workspace (T elements of n each): r, z, pA, pB, q, dinv.

template <typename T>
struct SlotVecs {
    T *r, *z, *pA, *pB, *q, *dinv;
    __device__ __forceinline__ SlotVecs(const PcgSlot &S, int n) {
        r = (T *)S.work;
        z = r + n;
        pA = z + n;
        pB = pA + n;
        q = pB + n;
        dinv = q + n;
    }
};

template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_init_kernel(int n, const PcgSlot *__restrict__ slots,
                                                               const int32_t *__restrict__ list,
                                                               const int32_t *__restrict__ diag_pos) {
    __shared__ double sh[kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    const SlotVecs<T> v(S, n);
    const T *__restrict__ b = (const T *)S.b;
    const T *__restrict__ values = (const T *)S.values;
    T *__restrict__ x = (T *)S.x;
    double rz = 0.0, bb = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        const T bi = b[i];
        const T di = (T)1 / values[diag_pos[i]];
        const T zi = di * bi;
        x[i] = (T)0;
        v.r[i] = bi;
        v.z[i] = zi;
        v.pA[i] = (T)0;
        v.dinv[i] = di;
        rz += (double)bi * (double)zi;
        bb += (double)bi * (double)bi;
    }
    rz = block_sum(rz, sh);
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        part(S.partials, kRZ0)[blockIdx.x] = rz;
        part(S.partials, kBB)[blockIdx.x] = bb;
    }
}

// Stop test on the residual of the last update, then p_new = z + beta p_old,
// q = K p_new and partials of p.q.  CHECK_ONLY launches stop after the test,
// and so does iteration max_iter.  n_prev: number of partials written by the
// previous kernel (init or update).
template <typename T, int G, bool CHECK_ONLY>
__global__ __launch_bounds__(kVecThreads) void pcg_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col_idx,
                                                               const PcgSlot *__restrict__ slots,
                                                               const int32_t *__restrict__ list, int step,
                                                               int n_prev) {
    __shared__ double sh[kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    PcgState *__restrict__ st = S.state;
    const int it = step - S.start;
    if (st->done) return;  // written only by earlier launches: the same value for every wave
    double tol2, rr;
    if (it == 0) {
        const double bb = sum_partials(part(S.partials, kBB), n_prev, sh);
        tol2 = S.rtol2 * bb;
        rr = bb;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->bb = bb;
            st->tol2 = tol2;
        }
    } else {
        tol2 = st->tol2;
        rr = sum_partials(part(S.partials, kRR), n_prev, sh);
    }
    if (rr <= tol2) {  // the same decision in every block
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->iters = it;
        }
        return;
    }
    if (CHECK_ONLY || it >= S.max_iter) return;
    const SlotVecs<T> v(S, n);
    const T *__restrict__ values = (const T *)S.values;
    const T *__restrict__ p_old = (it & 1) ? v.pB : v.pA;
    T *__restrict__ p_new = (it & 1) ? v.pA : v.pB;
    T beta = (T)0;
    if (it > 0) {
        const double rz = sum_partials(part(S.partials, kRZ0 + (it & 1)), n_prev, sh);
        const double rz_prev = sum_partials(part(S.partials, kRZ0 + ((it + 1) & 1)), n_prev, sh);
        beta = (T)(rz / rz_prev);
    }
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kVecThreads / G);
    double pq = 0.0;
    for (int i = blockIdx.x * (kVecThreads / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double acc = row_dot<T, G, true>(i, lane, row_ptr, col_idx, values, v.z, p_old, beta);
        if (lane == 0) {
            const T pi = v.z[i] + beta * p_old[i];
            const T qi = (T)acc;
            p_new[i] = pi;
            v.q[i] = qi;
            pq += (double)pi * (double)qi;
        }
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) part(S.partials, kPQ)[blockIdx.x] = pq;
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = D^{-1} r; partials of r.z (next buffer) and r.r
template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_update_kernel(int n, const PcgSlot *__restrict__ slots,
                                                                 const int32_t *__restrict__ list, int step,
                                                                 int n_pq, int n_rz) {
    __shared__ double sh[kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    const int it = step - S.start;
    if (S.state->done || it >= S.max_iter) return;  // done: written only by earlier launches
    const SlotVecs<T> v(S, n);
    const T *__restrict__ p = (it & 1) ? v.pA : v.pB;  // the p_new of this iteration's spmv
    T *__restrict__ x = (T *)S.x;
    const double pq = sum_partials(part(S.partials, kPQ), n_pq, sh);
    const double rz = sum_partials(part(S.partials, kRZ0 + (it & 1)), n_rz, sh);
    const T a = (T)(rz / pq);
    double rzn = 0.0, rr = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        const T ri = v.r[i] - a * v.q[i];
        x[i] += a * p[i];
        const T zi = v.dinv[i] * ri;
        v.r[i] = ri;
        v.z[i] = zi;
        rzn += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    rzn = block_sum(rzn, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part(S.partials, kRZ0 + ((it + 1) & 1))[blockIdx.x] = rzn;
        part(S.partials, kRR)[blockIdx.x] = rr;
    }
}

// per-block partials of ||b - K x||^2 (summed on the host in index order)
template <typename T, int G>
__global__ __launch_bounds__(kVecThreads) void residual_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col_idx,
                                                               const PcgSlot *__restrict__ slots,
                                                               const int32_t *__restrict__ list) {
    __shared__ double sh[kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    const T *__restrict__ values = (const T *)S.values;
    const T *__restrict__ x = (const T *)S.x;
    const T *__restrict__ b = (const T *)S.b;
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
    if (threadIdx.x == 0) part(S.partials, kRR)[blockIdx.x] = acc;
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
void launch_init_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(vec_blocks(n), count), dim3(kVecThreads), 0, s, n, slots, list,
                       pt.dev.diag_pos);
}

template <typename T, int G>
void launch_step_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, int step,
                   hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    const int nb = vec_blocks(n), ns = spmv_blocks<G>(n);
    hipLaunchKernelGGL((pcg_spmv_kernel<T, G, false>), dim3(ns, count), dim3(kVecThreads), 0, s, n,
                       pt.dev.row_ptr, pt.dev.col_idx, slots, list, step, nb);
    hipLaunchKernelGGL(pcg_update_kernel<T>, dim3(nb, count), dim3(kVecThreads), 0, s, n, slots, list, step, ns,
                       nb);
}

template <typename T, int G>
void launch_check_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, int step,
                    hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    hipLaunchKernelGGL((pcg_spmv_kernel<T, G, true>), dim3(1, count), dim3(kVecThreads), 0, s, n, pt.dev.row_ptr,
                       pt.dev.col_idx, slots, list, step, vec_blocks(n));
}

template <typename T, int G>
int launch_residual_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    const int ns = spmv_blocks<G>(n);
    hipLaunchKernelGGL((residual_kernel<T, G>), dim3(ns, count), dim3(kVecThreads), 0, s, n, pt.dev.row_ptr,
                       pt.dev.col_idx, slots, list);
    return ns;
}

// Dispatch on (dtype, lanes per row): F is called as F.template operator()<T, G>().
template <typename F>
auto dispatch(const tg_pattern &pt, tg_dtype dtype, F &&f) {
    const int g = pt.dev.spmv_group;
    if (dtype == TG_F64) {
        if (g == 4) return f.template operator()<double, 4>();
        if (g == 8) return f.template operator()<double, 8>();
        if (g == 16) return f.template operator()<double, 16>();
        return f.template operator()<double, 32>();
    }
    if (g == 4) return f.template operator()<float, 4>();
    if (g == 8) return f.template operator()<float, 8>();
    if (g == 16) return f.template operator()<float, 16>();
    return f.template operator()<float, 32>();
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

hipError_t launch_pcg_init(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list, int count,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    dispatch(p, dtype, [&]<typename T, int G>() { launch_init_t<T, G>(p, slots, list, count, s); });
    return hipGetLastError();
}

hipError_t launch_pcg_step(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list, int count,
                           int step, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    dispatch(p, dtype, [&]<typename T, int G>() { launch_step_t<T, G>(p, slots, list, count, step, s); });
    return hipGetLastError();
}

hipError_t launch_pcg_residual(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list,
                               int count, int *n_partials, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int ns = dispatch(p, dtype, [&]<typename T, int G>() {
        return launch_residual_t<T, G>(p, slots, list, count, s);
    });
    if (n_partials) *n_partials = ns;
    return hipGetLastError();
}

tg_status run_pcg(const tg_pattern &pt, tg_dtype dtype, const void *values, const void *rhs, void *x, double rtol,
                  int32_t max_iter, int32_t check_every, int32_t *iters, double *relres, hipStream_t s,
                  std::string &msg) {
    const DevicePattern &d = pt.dev;
    hipError_t err;
#define TG_CHECK(call)                    \
    do {                                  \
        err = (call);                     \
        if (err != hipSuccess) {          \
            msg = hipGetErrorString(err); \
            return TG_E_HIP;              \
        }                                 \
    } while (0)
    // The previous call ended with a stream synchronisation, so the pinned
    // staging copies are free to reuse.  Reset with copies, not memsets: a
    // caller may capture this stream.
    d.host_state->done = 0;
    d.host_state->iters = 0;
    *d.host_pcg_slot = PcgSlot{values, rhs, x, d.work, d.partials, d.state, rtol * rtol, 0, max_iter};
    TG_CHECK(hipMemcpyAsync(d.state, d.host_state, sizeof(PcgState), hipMemcpyHostToDevice, s));
    TG_CHECK(hipMemcpyAsync(d.pcg_slot, d.host_pcg_slot, sizeof(PcgSlot), hipMemcpyHostToDevice, s));
    TG_CHECK(launch_pcg_init(pt, dtype, d.pcg_slot, d.pcg_list, 1, s));
    int it = 0;
    bool done = false;
    while (it < max_iter && !done) {
        TG_CHECK(launch_pcg_step(pt, dtype, d.pcg_slot, d.pcg_list, 1, it, s));
        ++it;
        if (it % check_every == 0) {
            TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            TG_CHECK(hipStreamSynchronize(s));
            done = d.host_state->done != 0;
        }
    }
    // stop test on the last update (sets done/iters if it converged)
    dispatch(pt, dtype, [&]<typename T, int G>() { launch_check_t<T, G>(pt, d.pcg_slot, d.pcg_list, 1, it, s); });
    int ns = 0;
    TG_CHECK(launch_pcg_residual(pt, dtype, d.pcg_slot, d.pcg_list, 1, &ns, s));
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

}  // namespace tg
