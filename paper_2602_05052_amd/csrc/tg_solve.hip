// Dirichlet elimination, SpMV and Jacobi-preconditioned CG on the assembled
// CSR system (TensorGalerkin Sec. B.1.2: Jacobi-preconditioned Krylov solve of
// the condensed system, stopped on ||K u - f|| / ||f||).
//
// One CG iteration is one kernel of 512-thread blocks, one wave per slice of 64
// rows of a sliced-ELL copy of the matrix (the single-reduction form described
// with the PCG kernels below).  Every scalar
// (alpha, beta, the stop decision) is recomputed by every block from the
// previous launch's per-block partials, summed in one fixed order, so all
// blocks agree bitwise and the solver is reproducible with no atomics, no
// fences and no extra launches.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "tg_device.h"

namespace tg {
namespace {

constexpr int kWaves = kVecThreads / 64;

// One DPP move of a double (both 32-bit halves); lanes whose source is outside
// the row, and lanes of rows outside ROW_MASK, receive +0.0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROW_MASK, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave in a fixed order with DPP moves (VALU only,
// no LDS round trips): an inclusive scan within each row of 16 lanes (shifts
// by 1, 2, 4, 8), then lane 15 of rows 0 and 2 added into rows 1 and 3, then
// lane 31 into rows 2 and 3.  Lane 63 ends with the total.
__device__ __forceinline__ double wave_sum_last(double v) {
    v += dpp_move<0x111>(v);       // row_shr:1
    v += dpp_move<0x112>(v);       // row_shr:2
    v += dpp_move<0x114>(v);       // row_shr:4
    v += dpp_move<0x118>(v);       // row_shr:8
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15
    v += dpp_move<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// Sum over the lanes of a row group of G lanes, in a fixed order, every lane of
// the group ending with the same bits (a + b == b + a): DPP moves within a row
// of 16 lanes for G <= 16 (swap neighbours, swap pairs, mirror 8, mirror 16),
// lane shuffles for G = 32.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 32, "row groups of 4 to 32 lanes");
    if constexpr (G <= 16) {
        v += dpp_move<0xB1>(v);  // quad_perm [1, 0, 3, 2]
        v += dpp_move<0x4E>(v);  // quad_perm [2, 3, 0, 1]
        if constexpr (G >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
        if constexpr (G >= 16) v += dpp_move<0x140>(v);  // row_mirror
    } else {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    }
    return v;
}

// Sum over the block in a fixed order: wave_sum_last, then the wave totals in
// index order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum_last(v);
    if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// Block sums of three values, in a fixed order (wave_sum_last, then the wave
// totals in index order), delivered to thread 0 only (the writer of the
// block's partials).  W: waves of the block; sh: 3 W doubles.
template <int W = kWaves>
__device__ __forceinline__ void block_sum3_first(double &a, double &b, double &c, double *sh) {
    a = wave_sum_last(a);
    b = wave_sum_last(b);
    c = wave_sum_last(c);
    if ((threadIdx.x & 63) == 63) {
        const int w = threadIdx.x >> 6;
        sh[w] = a;
        sh[W + w] = b;
        sh[2 * W + w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ra = 0.0, rb = 0.0, rc = 0.0;
#pragma unroll 2
        for (int w = 0; w < W; ++w) {
            ra += sh[w];
            rb += sh[W + w];
            rc += sh[2 * W + w];
        }
        a = ra;
        b = rb;
        c = rc;
    }
}

// Sums of three partial values per thread, identical in every block (the fixed
// order of block_sum3_first), delivered to every thread with one barrier.
// sh: 3 W doubles, not written again by the caller's block in this launch (no
// barrier protects its later reuse).
template <int W = kWaves>
__device__ __forceinline__ void reduce_partials3(double *sh, double &a, double &b, double &c) {
    a = wave_sum_last(a);
    b = wave_sum_last(b);
    c = wave_sum_last(c);
    if ((threadIdx.x & 63) == 63) {
        const int w = threadIdx.x >> 6;
        sh[w] = a;
        sh[W + w] = b;
        sh[2 * W + w] = c;
    }
    __syncthreads();
    double ra = 0.0, rb = 0.0, rc = 0.0;
#pragma unroll 2
    for (int w = 0; w < W; ++w) {
        ra += sh[w];
        rb += sh[W + w];
        rc += sh[2 * W + w];
    }
    a = ra;
    b = rb;
    c = rc;
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

// Row i of K x, accumulated in FP64 by a group of G lanes in a fixed pattern
// (VP, XP: pointers to T in any address space).
template <int G, typename VP, typename XP>
__device__ __forceinline__ double row_dot(int i, int lane, const int32_t *__restrict__ row_ptr,
                                          const int32_t *__restrict__ col_idx, VP values, XP x) {
    const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
    double acc = 0.0;
    for (int q = p0 + lane; q < p1; q += G) acc += (double)values[q] * (double)x[col_idx[q]];
    acc = group_sum<G>(acc);
    return acc;
}

template <typename T, int G>
__global__ __launch_bounds__(256) void spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx, const T *__restrict__ values,
                                                   const T *__restrict__ x, T *__restrict__ y) {
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (256 / G);
    for (int i = blockIdx.x * (256 / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<G>(i, lane, row_ptr, col_idx, values, x);
        if (lane == 0) y[i] = (T)v;
    }
}

// ---------------------------------------------------------------- PCG kernels
// Preconditioned CG in the single-reduction form of Chronopoulos and Gear:
// besides r, u = D^{-1} r, p and x it carries w = K u and s = K p, updated by
// recurrences, so that the two inner products of an iteration, r.u and w.u,
// come out of the same pass as the SpMV:
//   beta_i  = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
//   p = u + beta p;  s = w + beta s;  x += alpha p;  r -= alpha s;  u = D^{-1} r;  w = K u
//   gamma_{i+1} = r.u,  delta_{i+1} = w.u  (and r.r for the stop test)
// with gamma_i = r_i.u_i, delta_i = w_i.u_i, beta_0 = 0, alpha_0 = gamma_0 / delta_0.
// In exact arithmetic it produces the iterates of standard PCG.
//
// Each launch serves the slots slots[list[blockIdx.y]] (one CG system each, all
// on the same pattern); blockIdx.x strides over the rows.  A slot's iteration
// is step - start, so systems that joined at different steps share launches.
// One iteration is one launch: the SpMV needs the new u at neighbouring rows,
// which every block recomputes from the previous iteration's record of that
// row with the same expressions its owner uses, so the values agree bitwise
// and no grid-wide barrier is needed.  The record holds the row's r, w and s
// scaled by D^{-1} (u = D^{-1} r, D^{-1} w, D^{-1} s): the recurrences are
// linear, so they run unchanged on the scaled values, the new u is
// u - alpha (D^{-1} w + beta D^{-1} s), and w's update needs D^{-1} K u, one
// product by the row's own D^{-1}; the inner products use the diagonal K_ii
// (r = K_ii u).  Three values per gathered record instead of four.  Records
// are double buffered by iteration parity (the owner writes the new record
// while neighbours still read the old one).

// A slot's arrays are reached through pointers read from memory, which the
// compiler cannot place in an address space; casting them to the global one
// gives global (not flat) memory instructions.
#define TG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ TG_GLOBAL T *gl(T *p) {
    return (TG_GLOBAL T *)p;
}

template <typename T>
struct Rec {  // the per-row record gathered by the SpMV (24 / 12 bytes): u = D^{-1} r, D^{-1} w, D^{-1} s
    T u, w, s;
};

// A slot's workspace (kPcgWorkVectors vectors of n values): the records of even
// and odd iterates (3 n each), p (n) and the Jacobi factors D^{-1} = 1 / K_ii
// (n; K_ii itself is recovered as 1 / D^{-1} where the inner products need it).
template <typename T>
struct SlotVecs {
    TG_GLOBAL Rec<T> *rec0, *rec1;
    TG_GLOBAL T *p;
    TG_GLOBAL T *dinv;
    __device__ __forceinline__ SlotVecs(const PcgSlot &S, int n) {
        rec0 = gl((Rec<T> *)S.work);
        rec1 = rec0 + n;
        p = (TG_GLOBAL T *)(rec1 + n);
        dinv = p + n;
    }
    __device__ __forceinline__ TG_GLOBAL Rec<T> *rec(int parity) const { return parity ? rec1 : rec0; }
};

template <typename T>
__device__ __forceinline__ Rec<T> load_rec(const TG_GLOBAL Rec<T> *__restrict__ a, int i) {
    return Rec<T>{a[i].u, a[i].w, a[i].s};
}

template <typename T>
__device__ __forceinline__ void store_rec(TG_GLOBAL Rec<T> *__restrict__ a, int i, T u, T w, T s) {
    a[i].u = u;
    a[i].w = w;
    a[i].s = s;
}

// The recurrences of a row's scaled s and u: the owner's update, and (FP32
// iterations) every neighbour's view of the row's new u as an SpMV column.
template <typename T>
__device__ __forceinline__ T next_s(const Rec<T> &o, T beta) { return o.w + beta * o.s; }
template <typename T>
__device__ __forceinline__ T next_u_s(const Rec<T> &o, T s_new, T alpha) { return o.u - alpha * s_new; }
template <typename T>
__device__ __forceinline__ T next_u(const Rec<T> &o, T beta, T alpha) {
    return next_u_s(o, next_s(o, beta), alpha);
}

// x = 0, p = 0, u = D^{-1} b, s = 0, the Jacobi factors (record of parity 0; w follows).
template <typename T>
__global__ __launch_bounds__(kVecThreads) void pcg_init_kernel(int n, const PcgSlot *__restrict__ slots,
                                                               const int32_t *__restrict__ list,
                                                               const int32_t *__restrict__ diag_pos) {
    const PcgSlot S = slots[list[blockIdx.y]];
    const SlotVecs<T> v(S, n);
    const TG_GLOBAL T *__restrict__ b = gl((const T *)S.b);
    const TG_GLOBAL T *__restrict__ values = gl((const T *)S.values);
    TG_GLOBAL T *__restrict__ x = gl((T *)S.x);
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        x[i] = (T)0;
        v.p[i] = (T)0;
        const T kii = values[diag_pos[i]], d = (T)1 / kii;
        v.dinv[i] = d;
        store_rec(v.rec0, i, d * b[i], (T)0, (T)0);
    }
}

// Warm start: u = D^{-1} (b - K x) for the given x, p = 0, s = 0, the Jacobi
// factors (record of parity 0; w follows), and per-block partials of b.b at kResid.
template <typename T, int G>
__global__ __launch_bounds__(kVecThreads, 8) void pcg_warm_init_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                                    const int32_t *__restrict__ col_idx,
                                                                    const PcgSlot *__restrict__ slots,
                                                                    const int32_t *__restrict__ list,
                                                                    const int32_t *__restrict__ diag_pos) {
    __shared__ double sh[kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    const SlotVecs<T> v(S, n);
    const TG_GLOBAL T *__restrict__ b = gl((const T *)S.b);
    const TG_GLOBAL T *__restrict__ values = gl((const T *)S.values);
    const TG_GLOBAL T *__restrict__ x = gl((const T *)S.x);
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kVecThreads / G);
    double bb = 0.0;
    for (int i = blockIdx.x * (kVecThreads / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double kx = row_dot<G>(i, lane, row_ptr, col_idx, values, x);
        if (lane == 0) {
            const T bi = b[i];
            v.p[i] = (T)0;
            const T kii = values[diag_pos[i]], d = (T)1 / kii;
            v.dinv[i] = d;
            store_rec(v.rec0, i, d * (T)((double)bi - kx), (T)0, (T)0);
            bb += (double)bi * (double)bi;
        }
    }
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) part(S.partials, kResid)[blockIdx.x] = bb;
}

// Warm start: b.b from the n_prev partials -> state bb and tol2 = rtol^2 b.b.
__global__ __launch_bounds__(kVecThreads) void pcg_warm_tol_kernel(const PcgSlot *__restrict__ slots,
                                                                   const int32_t *__restrict__ list, int n_prev) {
    __shared__ double sh[kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    double bb = (int)threadIdx.x < n_prev ? part(S.partials, kResid)[threadIdx.x] : 0.0;
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        S.state->bb = bb;
        S.state->tol2 = S.rtol2 * bb;
    }
}

// w_0 = K u_0 (stored scaled by D^{-1}), and partials of r.u, w.u, r.r with
// r = K_ii u (parity 0).  Reads the u field of neighbouring records and writes
// only the w field of its own rows.
template <typename T, int G>
__global__ __launch_bounds__(kVecThreads, 8) void pcg_init_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                                    const int32_t *__restrict__ col_idx,
                                                                    const PcgSlot *__restrict__ slots,
                                                                    const int32_t *__restrict__ list) {
    __shared__ double sh[3 * kWaves];
    const PcgSlot S = slots[list[blockIdx.y]];
    const SlotVecs<T> v(S, n);
    TG_GLOBAL Rec<T> *__restrict__ rec = v.rec0;
    const TG_GLOBAL T *__restrict__ values = gl((const T *)S.values);
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kVecThreads / G);
    double gam = 0.0, del = 0.0, rr = 0.0;
    for (int i = blockIdx.x * (kVecThreads / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
        double acc = 0.0;
#pragma unroll 2
        for (int q = p0 + lane; q < p1; q += G) {
            const int j = col_idx[q];
            acc += (double)values[q] * (double)rec[j].u;
        }
        acc = group_sum<G>(acc);
        if (lane == 0) {
            const T d = v.dinv[i];
            const double ui = (double)rec[i].u, ri = (double)((T)1 / d) * ui;
            rec[i].w = (T)((double)d * acc);
            gam += ri * ui;
            del += acc * ui;
            rr += ri * ri;
        }
    }
    block_sum3_first(gam, del, rr, sh);
    if (threadIdx.x == 0) {
        part(S.partials, kGam)[blockIdx.x] = gam;
        part(S.partials, kDel)[blockIdx.x] = del;
        part(S.partials, kRr)[blockIdx.x] = rr;
    }
}

// The slot of a launch's system: by value for a solo system (no dependent load
// before its state), else through the batch's table.
template <bool SOLO>
__device__ __forceinline__ PcgSlot pick_slot(const PcgSlot *__restrict__ slots, const int32_t *__restrict__ list,
                                             const PcgSlot &solo) {
    if constexpr (SOLO)
        return solo;
    else
        return slots[list[blockIdx.y]];
}

// Column of sliced-ELL entry q of a row whose clamped index is rb: the 32-bit
// column itself, or rb plus a 16-bit offset when the pattern's columns all lie
// within 32767 of their rows (half the index bytes of every iteration).
template <typename CI> struct SellCols;
template <> struct SellCols<int32_t> {
    const int32_t *__restrict__ c;
    __device__ __forceinline__ int operator()(int q, int) const { return c[q]; }
};
template <> struct SellCols<int16_t> {
    const int16_t *__restrict__ c;
    __device__ __forceinline__ int operator()(int q, int rb) const { return rb + (int)c[q]; }
};

// Entries of a row per round of the iteration kernel's SpMV (FP64 products,
// FP32 new-u terms).
constexpr int kIterRound = 3;
constexpr int kIterRound32 = 4;

// The three products of row i that give (K u_new)_i once alpha and beta are
// known: with the scaled record (u, D^{-1} w, D^{-1} s) and
// u_new = u - alpha (D^{-1} w + beta D^{-1} s),
//   K u_new = K u - alpha (K D^{-1} w + beta K D^{-1} s),
// and the three products need only the previous iterate's records.  Entries
// [0, len) of the row start at q = e and stride 64 (sliced-ELL); each product
// sums the row's terms in entry order.  The loop is software-pipelined: the
// next round's columns and values are requested before this round's records
// are consumed.
template <typename T, typename CI>
__device__ __forceinline__ void row_products(const TG_GLOBAL T *__restrict__ sv, const SellCols<CI> &cols, int rb,
                                             const TG_GLOBAL Rec<T> *__restrict__ ra, int e, int len, double &A,
                                             double &B, double &C) {
    constexpr int R = kIterRound;
    int c[R];
    T val[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int q = e + 64 * min(u, len - 1);  // clamped: entries past the row re-read its last one, unused
        c[u] = cols(q, rb);
        val[u] = sv[q];
    }
    for (int k = 0; k < len; k += R) {
        Rec<T> rc[R];
#pragma unroll
        for (int u = 0; u < R; ++u) rc[u] = load_rec(ra, c[u]);
        int cn[R];
        T vn[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int q = e + 64 * min(k + R + u, len - 1);
            cn[u] = cols(q, rb);
            vn[u] = sv[q];
        }
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (k + u < len) {
                const double vd = (double)val[u];
                A += vd * (double)rc[u].u;
                B += vd * (double)rc[u].w;
                C += vd * (double)rc[u].s;
            }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            c[u] = cn[u];
            val[u] = vn[u];
        }
    }
}

// Entries [k0, len) of row i's (K u_new)_i with u_new of every column from its
// previous record (next_u), in entry order and rounds of kIterRound32 (the FP32
// iterations: u_new in FP32, products and sum in FP64).
template <typename T, typename CI>
__device__ __forceinline__ double row_tail_new_u(const TG_GLOBAL T *__restrict__ sv, const SellCols<CI> &cols, int rb,
                                                 const TG_GLOBAL Rec<T> *__restrict__ ra, int e, int k0, int len,
                                                 T alpha, T beta, double acc) {
    constexpr int R = kIterRound32;
    for (int k = k0; k < len; k += R) {
        T val[R];
        Rec<T> rc[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int q = e + 64 * min(k + u, len - 1);
            val[u] = sv[q];
            rc[u] = load_rec(ra, cols(q, rb));
        }
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (k + u < len) acc += (double)val[u] * (double)next_u(rc[u], beta, alpha);
    }
    return acc;
}

// Iteration `it` of the system: stop test on r.r of the current iterate, then
// the updates of every owned row and w = K u for them, with the partials of
// the next iterate.  CHECK_ONLY launches stop after the test, and so does
// iteration max_iter.  n_prev: number of partials written by the previous
// launch (n_prev_init for iteration 0, whose partials come from
// pcg_init_spmv_kernel); both are at most kMaxGrid.
//
// The SpMV runs on the sliced-ELL copy of the values: each wave owns slices of
// 64 consecutive rows, one row per lane, and step k of the wave reads entry k of
// its 64 rows from 64 consecutive places (coalesced values and columns; on a
// structured mesh the gathered records are consecutive too).  In FP64 its
// three products (row_products) do not depend on alpha and beta, so they run
// before the reduction of the previous partials, whose loads are issued first
// and whose latency the SpMV hides.  In FP32 (where three FP64 products per
// entry cost more than they hide) the first kIterRound32 entries and their
// records are fetched before the reduction and the new u of each column is
// formed after it.  Waves own slices in XCD-contiguous ranges (neighbouring
// rows' records stay in one L2).
template <typename T, bool CHECK_ONLY, bool SOLO, typename CI>
__global__ __launch_bounds__(iter_threads<T>()) __attribute__((amdgpu_waves_per_eu(6)))
void pcg_iter_kernel(int n, int nsl, int ulen, const int32_t *__restrict__ sell_ptr, const CI *__restrict__ sell_col,
                     const PcgSlot *__restrict__ slots, const int32_t *__restrict__ list, PcgSlot solo, int step,
                     int n_prev_init, int n_prev) {
    constexpr int kThreads = iter_threads<T>(), W = kThreads / 64;
    __shared__ double sh[3 * W];   // the previous partials' reduction
    __shared__ double sh2[3 * W];  // this launch's block sums
    __shared__ double sst[4];
    const PcgSlot S = pick_slot<SOLO>(slots, list, solo);
    PcgState *__restrict__ st = S.state;
    const int it = step - S.start;
    const int cur = 3 * (it & 1), nxt = 3 * ((it + 1) & 1);
    const SlotVecs<T> v(S, n);
    const TG_GLOBAL Rec<T> *__restrict__ ra = v.rec(it & 1);
    TG_GLOBAL Rec<T> *__restrict__ rb = v.rec((it + 1) & 1);
    const TG_GLOBAL T *__restrict__ sv = gl((const T *)S.sell);
    TG_GLOBAL T *__restrict__ x = gl((T *)S.x);
    const int lane = threadIdx.x & 63;
    const SellCols<CI> cols{sell_col};
    const int waves = gridDim.x * W;
    const int sl0 = xcd_swizzle(blockIdx.x, gridDim.x) * W + (int)(threadIdx.x >> 6);  // this wave's first slice

    // the previous launch's partials (strided over the threads) and, by the block's last
    // thread, the stop flag and scalars of earlier launches; the reduction's
    // barrier publishes them through LDS
    const int np = it == 0 ? n_prev_init : n_prev;
    const TG_GLOBAL double *p_rr = gl(part(S.partials, kRr + cur)), *p_gam = gl(part(S.partials, kGam + cur)),
                           *p_del = gl(part(S.partials, kDel + cur));
    double rr_cur = 0.0, gam = 0.0, del = 0.0;
    for (int t = threadIdx.x; t < np; t += kThreads) {
        rr_cur += p_rr[t];
        gam += p_gam[t];
        del += p_del[t];
    }
    if (threadIdx.x == kThreads - 1) {
        sst[0] = (double)st->done;
        sst[1] = st->tol2;
        sst[2] = st->gamma[(it + 1) & 1];
        sst[3] = st->alpha[(it + 1) & 1];
    }
    // the first slice's SpMV products, then the row's own record, p and x (their
    // latency overlaps the reduction).  A wave that finds the system already
    // converged skips the products (launches after convergence cost little); a
    // stale flag only costs the work, and the decision below is taken on the
    // published flag and partials.
    constexpr bool kSplit = sizeof(T) == 8;
    constexpr int R32 = kIterRound32;
    const int s0 = min(sl0, nsl - 1);
    const int i0 = min(s0 * 64 + lane, n - 1);
    Rec<T> f_o{};
    T f_d = 0;
    T f_pold = 0, f_xold = 0;
    double A = 0.0, B = 0.0, C = 0.0;
    int e0 = 0, len0 = 0;
    T f_val[kSplit ? 1 : R32];
    Rec<T> f_rec[kSplit ? 1 : R32];
    if constexpr (!CHECK_ONLY) {
        e0 = ulen ? s0 * 64 * ulen + lane : sell_ptr[s0] + lane;
        len0 = ulen ? ulen : (sell_ptr[s0 + 1] - sell_ptr[s0]) >> 6;
        if constexpr (kSplit) {
            if (sl0 < nsl && st->done == 0) row_products(sv, cols, i0, ra, e0, len0, A, B, C);
        } else {
#pragma unroll
            for (int u = 0; u < R32; ++u) {  // clamped: entries past the row re-read its last one, unused
                const int q = e0 + 64 * min(u, len0 - 1);
                f_val[u] = sv[q];
                f_rec[u] = load_rec(ra, cols(q, i0));
            }
        }
        f_o = load_rec(ra, i0);
        f_d = v.dinv[i0];
        f_pold = v.p[i0];
        f_xold = x[i0];
    }
    reduce_partials3<W>(sh, rr_cur, gam, del);
    if (sst[0] != 0.0) return;
    const double tol2_prev = sst[1], gam_prev = sst[2], alpha_prev = sst[3];
    double tol2;
    if (it == 0 && !S.warm) {
        tol2 = S.rtol2 * rr_cur;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->bb = rr_cur;
            st->tol2 = tol2;
        }
    } else {
        tol2 = tol2_prev;
    }
    if (rr_cur <= tol2) {  // the same decision in every block
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->iters = it;
        }
        return;
    }
    if (CHECK_ONLY || it >= S.max_iter) return;
    double alpha_d, beta_d;
    if (it == 0) {
        beta_d = 0.0;
        alpha_d = gam / del;
    } else {
        beta_d = gam / gam_prev;
        alpha_d = gam / (del - beta_d * gam / alpha_prev);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // read by the next launch only
        st->alpha[it & 1] = alpha_d;
        st->gamma[it & 1] = gam;
    }
    const T alpha = (T)alpha_d, beta = (T)beta_d;
    double gn = 0.0, dn = 0.0, rn = 0.0;
    // row i's update from its own record, Jacobi factor d, p, x and w = (K u_new)_i;
    // the inner products with r = K_ii u
    auto update_row = [&](int i, double w, const Rec<T> &o, T d, T p_old, T x_old) {
        const T pi = o.u + beta * p_old;  // u_i + beta p
        const T si = next_s(o, beta);
        const T ui = next_u_s(o, si, alpha);
        const T wi = (T)w;
        x[i] = x_old + alpha * pi;
        v.p[i] = pi;
        store_rec(rb, i, ui, (T)((double)d * w), si);
        const double ud = (double)ui, rd = (double)((T)1 / d) * ud;
        gn += rd * ud;
        dn += (double)wi * ud;
        rn += rd * rd;
    };
    if (sl0 < nsl) {
        double w;
        if constexpr (kSplit) {
            w = A - alpha_d * (B + beta_d * C);
        } else {
            w = 0.0;
#pragma unroll
            for (int u = 0; u < R32; ++u)
                if (u < len0) w += (double)f_val[u] * (double)next_u(f_rec[u], beta, alpha);
            w = row_tail_new_u(sv, cols, i0, ra, e0, R32, len0, alpha, beta, w);
        }
        if (s0 * 64 + lane < n) update_row(s0 * 64 + lane, w, f_o, f_d, f_pold, f_xold);
    }
    for (int sl = sl0 + waves; sl < nsl; sl += waves) {  // systems with more slices than waves
        const int i = sl * 64 + lane;
        const int ic = min(i, n - 1);
        const Rec<T> o = load_rec(ra, ic);
        const T dd = v.dinv[ic];
        const T p_old = v.p[ic], x_old = x[ic];
        const int e = ulen ? sl * 64 * ulen + lane : sell_ptr[sl] + lane;
        const int len = ulen ? ulen : (sell_ptr[sl + 1] - sell_ptr[sl]) >> 6;
        double w;
        if constexpr (kSplit) {
            double a = 0.0, b = 0.0, c = 0.0;
            row_products(sv, cols, ic, ra, e, len, a, b, c);
            w = a - alpha_d * (b + beta_d * c);
        } else {
            w = row_tail_new_u(sv, cols, ic, ra, e, 0, len, alpha, beta, 0.0);
        }
        if (i < n) update_row(i, w, o, dd, p_old, x_old);
    }
    block_sum3_first<W>(gn, dn, rn, sh2);
    if (threadIdx.x == 0) {
        part(S.partials, kGam + nxt)[blockIdx.x] = gn;
        part(S.partials, kDel + nxt)[blockIdx.x] = dn;
        part(S.partials, kRr + nxt)[blockIdx.x] = rn;
    }
}

// The sliced-ELL copy of CSR values: one wave per slice, lane l on row 64 s + l;
// padding entries get 0.
template <typename T>
__global__ __launch_bounds__(kFillThreads) void sell_fill_kernel(int n, int nsl, const int32_t *__restrict__ sell_ptr,
                                                                 const int32_t *__restrict__ row_ptr,
                                                                 const T *__restrict__ values, T *__restrict__ sell) {
    const int lane = threadIdx.x & 63;
    for (int sl = blockIdx.x * (kFillThreads / 64) + (int)(threadIdx.x >> 6); sl < nsl;
         sl += gridDim.x * (kFillThreads / 64)) {
        const int e = sell_ptr[sl] + lane, len = (sell_ptr[sl + 1] - sell_ptr[sl]) >> 6;
        const int i = sl * 64 + lane;
        const int p0 = i < n ? row_ptr[i] : 0, m = i < n ? row_ptr[i + 1] - p0 : 0;
        for (int k = 0; k < len; ++k) sell[e + 64 * k] = k < m ? values[p0 + k] : (T)0;
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
    const TG_GLOBAL T *__restrict__ values = gl((const T *)S.values);
    const TG_GLOBAL T *__restrict__ x = gl((const T *)S.x);
    const TG_GLOBAL T *__restrict__ b = gl((const T *)S.b);
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kVecThreads / G);
    double acc = 0.0;
    for (int i = blockIdx.x * (kVecThreads / G) + threadIdx.x / G; i < n; i += rows_per_grid) {
        const double v = row_dot<G>(i, lane, row_ptr, col_idx, values, x);
        if (lane == 0) {
            const double ri = (double)b[i] - v;
            acc += ri * ri;
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part(S.partials, kResid)[blockIdx.x] = acc;
}

int vec_blocks(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kSetupMaxGrid, (n + kVecThreads - 1) / kVecThreads));
}

template <int G>
int spmv_blocks(int64_t n) {
    const int64_t rows_per_block = kVecThreads / G;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kSetupMaxGrid, (n + rows_per_block - 1) / rows_per_block));
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
    hipLaunchKernelGGL((pcg_init_spmv_kernel<T, G>), dim3(spmv_blocks<G>(n), count), dim3(kVecThreads), 0, s, n,
                       pt.dev.row_ptr, pt.dev.col_idx, slots, list);
}

template <typename T, int G>
void launch_warm_init_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    const int ns = spmv_blocks<G>(n);
    hipLaunchKernelGGL((pcg_warm_init_kernel<T, G>), dim3(ns, count), dim3(kVecThreads), 0, s, n, pt.dev.row_ptr,
                       pt.dev.col_idx, slots, list, pt.dev.diag_pos);
    hipLaunchKernelGGL(pcg_warm_tol_kernel, dim3(1, count), dim3(kVecThreads), 0, s, slots, list, ns);
    hipLaunchKernelGGL((pcg_init_spmv_kernel<T, G>), dim3(ns, count), dim3(kVecThreads), 0, s, n, pt.dev.row_ptr,
                       pt.dev.col_idx, slots, list);
}

// Blocks of the iteration kernel: one slice per wave, at most kMaxGrid blocks
// (grid-stride over slices beyond).
template <typename T>
int iter_blocks(const tg_pattern &pt) {
    const int64_t per = iter_threads<T>() / 64;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxGrid, (pt.dev.n_slices + per - 1) / per));
}

template <typename T, int G>
void launch_step_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, int step,
                   hipStream_t s, const PcgSlot *solo) {
    const int n = (int)pt.host.n_dofs, nsl = (int)pt.dev.n_slices;
    const int ns0 = spmv_blocks<G>(n), ns = iter_blocks<T>(pt);
    auto go = [&](auto *cols) {
        using CI = std::remove_const_t<std::remove_pointer_t<decltype(cols)>>;
        if (solo)
            hipLaunchKernelGGL((pcg_iter_kernel<T, false, true, CI>), dim3(ns, 1), dim3(iter_threads<T>()), 0, s, n,
                               nsl, pt.dev.sell_len, pt.dev.sell_ptr, cols, slots, list, *solo, step, ns0, ns);
        else
            hipLaunchKernelGGL((pcg_iter_kernel<T, false, false, CI>), dim3(ns, count), dim3(iter_threads<T>()), 0, s,
                               n, nsl, pt.dev.sell_len, pt.dev.sell_ptr, cols, slots, list, PcgSlot{}, step, ns0, ns);
    };
    if (pt.dev.sell16)
        go((const int16_t *)pt.dev.sell_off);
    else
        go((const int32_t *)pt.dev.sell_col);
}

template <typename T, int G>
void launch_check_t(const tg_pattern &pt, const PcgSlot *slots, const int32_t *list, int count, int step,
                    hipStream_t s) {
    const int n = (int)pt.host.n_dofs;
    hipLaunchKernelGGL((pcg_iter_kernel<T, true, false, int32_t>), dim3(1, count), dim3(iter_threads<T>()), 0, s, n,
                       (int)pt.dev.n_slices, 0, pt.dev.sell_ptr, pt.dev.sell_col, slots, list, PcgSlot{}, step,
                       spmv_blocks<G>(n), iter_blocks<T>(pt));
}

template <typename T>
hipError_t launch_sell_fill_t(const tg_pattern &pt, const void *values, void *sell, hipStream_t s) {
    const int64_t per = kFillThreads / 64;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (pt.dev.n_slices + per - 1) / per));
    hipLaunchKernelGGL(sell_fill_kernel<T>, dim3(nb), dim3(kFillThreads), 0, s, (int)pt.host.n_dofs,
                       (int)pt.dev.n_slices, pt.dev.sell_ptr, pt.dev.row_ptr, (const T *)values, (T *)sell);
    return hipGetLastError();
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

bool state_finite(const PcgState &st) {
    return std::isfinite(st.bb) && std::isfinite(st.alpha[0]) && std::isfinite(st.alpha[1]) &&
           std::isfinite(st.gamma[0]) && std::isfinite(st.gamma[1]);
}

RunEnd run_end(bool done, double relres, double prev_relres, double rtol, bool nonfinite, int run, int total,
               int max_iter) {
    if (nonfinite || !std::isfinite(relres)) return RunEnd::kNonFinite;
    if (!done) return RunEnd::kNoConv;
    if (relres <= rtol) return RunEnd::kOk;
    const bool progress = run == 0 || relres <= 0.5 * prev_relres;
    if (!progress) return RunEnd::kAccuracy;
    if (run < kPcgRestarts && total < max_iter) return RunEnd::kRestart;
    return total < max_iter ? RunEnd::kAccuracy : RunEnd::kNoConv;
}

hipError_t launch_dirichlet(const tg_pattern &p, tg_dtype dtype, void *values, void *rhs, const void *g,
                            hipStream_t s) {
    return dtype == TG_F64 ? launch_dirichlet_t<double>(p, values, rhs, g, s)
                           : launch_dirichlet_t<float>(p, values, rhs, g, s);
}

hipError_t launch_spmv(const tg_pattern &p, tg_dtype dtype, const void *values, const void *x, void *y,
                       hipStream_t s) {
    return dtype == TG_F64 ? launch_spmv_g<double>(p, values, x, y, s) : launch_spmv_g<float>(p, values, x, y, s);
}

hipError_t launch_sell_fill(const tg_pattern &p, tg_dtype dtype, const void *values, void *sell, hipStream_t s) {
    return dtype == TG_F64 ? launch_sell_fill_t<double>(p, values, sell, s)
                           : launch_sell_fill_t<float>(p, values, sell, s);
}

hipError_t launch_pcg_init(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list, int count,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    dispatch(p, dtype, [&]<typename T, int G>() { launch_init_t<T, G>(p, slots, list, count, s); });
    return hipGetLastError();
}

hipError_t launch_pcg_warm_init(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list,
                                int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    dispatch(p, dtype, [&]<typename T, int G>() { launch_warm_init_t<T, G>(p, slots, list, count, s); });
    return hipGetLastError();
}

hipError_t launch_pcg_step(const tg_pattern &p, tg_dtype dtype, const PcgSlot *slots, const int32_t *list, int count,
                           int step, hipStream_t s, const PcgSlot *solo) {
    if (count <= 0) return hipSuccess;
    dispatch(p, dtype, [&]<typename T, int G>() { launch_step_t<T, G>(p, slots, list, count, step, s, solo); });
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
                  std::string &msg, bool warm, bool strict) {
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
    if (pt.host.n_dofs == 0) {  // nothing to solve
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return TG_OK;
    }
    TG_CHECK(launch_sell_fill(pt, dtype, values, d.sell_vals, s));
    int total = 0;              // iterations of all runs
    double prev_rel = INFINITY;  // the previous run's true residual
    for (int run = 0;; ++run) {
        // The previous run (or call) ended with a stream synchronisation, so the
        // pinned staging copies are free to reuse.  Reset with copies, not
        // memsets: a caller may capture this stream.
        const int32_t budget = max_iter - total;
        const bool warm_run = warm || run > 0;
        d.host_state->done = 0;
        d.host_state->iters = 0;
        const PcgSlot slot{values, d.sell_vals, rhs, x, d.work, d.partials, d.state, rtol * rtol, 0, budget,
                           warm_run ? 1 : 0};
        *d.host_pcg_slot = slot;
        TG_CHECK(hipMemcpyAsync(d.state, d.host_state, sizeof(PcgState), hipMemcpyHostToDevice, s));
        TG_CHECK(hipMemcpyAsync(d.pcg_slot, d.host_pcg_slot, sizeof(PcgSlot), hipMemcpyHostToDevice, s));
        if (warm_run) {
            TG_CHECK(launch_pcg_warm_init(pt, dtype, d.pcg_slot, d.pcg_list, 1, s));
        } else {
            TG_CHECK(launch_pcg_init(pt, dtype, d.pcg_slot, d.pcg_list, 1, s));
        }
        // Iterations go out in chunks of check_every, each followed by a copy of the
        // state into one of two pinned mirrors and an event.  The host polls a chunk's
        // state while the next chunk already runs, so the GPU never idles on the
        // round trip; launches after convergence return at once (the stop test is
        // taken on the device), so the result is the same as stopping exactly.  A
        // non-finite step length or inner product ends the run.
        int it = 0;
        bool nonfinite = false;
        auto chunk = [&](int buf) -> hipError_t {
            for (int k = 0; k < check_every && it < budget; ++k, ++it) {
                const hipError_t e = launch_pcg_step(pt, dtype, d.pcg_slot, d.pcg_list, 1, it, s, &slot);
                if (e != hipSuccess) return e;
            }
            const hipError_t e =
                hipMemcpyAsync(d.host_state + buf, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s);
            return e != hipSuccess ? e : hipEventRecord(d.poll_ev[buf], s);
        };
        TG_CHECK(chunk(0));
        for (int cur = 0;; cur ^= 1) {
            const bool more = it < budget;
            if (more) TG_CHECK(chunk(cur ^ 1));
            TG_CHECK(hipEventSynchronize(d.poll_ev[cur]));
            nonfinite = !state_finite(d.host_state[cur]);
            if (d.host_state[cur].done || !more || nonfinite) break;
        }
        // stop test on the last update (sets done/iters if it converged)
        dispatch(pt, dtype,
                 [&]<typename T, int G>() { launch_check_t<T, G>(pt, d.pcg_slot, d.pcg_list, 1, it, s); });
        int ns = 0;
        TG_CHECK(launch_pcg_residual(pt, dtype, d.pcg_slot, d.pcg_list, 1, &ns, s));
        std::vector<double> host_parts(ns);
        TG_CHECK(hipMemcpyAsync(d.host_state, d.state, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        TG_CHECK(hipMemcpyAsync(host_parts.data(), d.partials + (size_t)kResid * kMaxGrid, sizeof(double) * ns,
                                hipMemcpyDeviceToHost, s));
        TG_CHECK(hipStreamSynchronize(s));
        const bool done = d.host_state->done != 0;
        double rr = 0.0;
        for (double v : host_parts) rr += v;
        const double bb = d.host_state->bb;
        const double rel = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        total += done ? d.host_state->iters : std::min(it, budget);
        if (iters) *iters = total;
        if (relres) *relres = rel;
        const bool bad = nonfinite || !state_finite(*d.host_state);
        RunEnd end = run_end(done, rel, prev_rel, rtol, bad, run, total, max_iter);
        if (!strict && (end == RunEnd::kRestart || end == RunEnd::kAccuracy)) end = RunEnd::kOk;
        prev_rel = rel;
        if (end == RunEnd::kRestart) continue;
        if (end == RunEnd::kAccuracy) {
            msg = "the recursive residual met rtol but the true residual stays above it (restarts from x no "
                  "longer reduce it): rtol is below the attainable accuracy of this dtype";
            return TG_E_ACCURACY;
        }
        if (end == RunEnd::kNonFinite) {
            msg = "PCG met a non-finite value (check the matrix and right-hand side)";
            return TG_E_NONFINITE;
        }
        if (end == RunEnd::kNoConv) {
            msg = "PCG did not reach rtol within max_iter iterations";
            return TG_E_NOCONV;
        }
        return TG_OK;
    }
#undef TG_CHECK
}

}  // namespace tg
