// Fused Batch-Map + Sparse-Reduce kernels for gfx950 (TensorGalerkin Sec. 2,
// Alg. 1 and Alg. 2).
//
// One workgroup owns a block of consecutive CSR node rows.  Work inside it:
//   Stage  : the distinct vertices of the block's elements (a list built with
//            the pattern) are copied into LDS once.
//   Map    : one lane per (row node i, element e, local node a) pair of the
//            block (P2: in each of three waves, for a third of the column
//            nodes).  It reads e's vertices from LDS, forms J, |det J| and the
//            cofactors of J in FP64 (Alg. 1 Geometry), pushes the reference
//            gradients forward (Push-forward), evaluates the per-element
//            coefficients (Physics), and integrates row a of K_e and entry a
//            of F_e (Integration, eq. kloc1: the quadrature rule, or for the
//            P2 stiffness the exact integrals that rule gives).  The row goes
//            to LDS.
//   Reduce : one lane per CSR value (P1) or per 3x3 node block (P2) sums the
//            element slots that the routing table maps to it (the S_mat
//            projection of Alg. 2), in ascending element order, and writes it
//            once; one lane per row sums its load contributions (the S_vec
//            projection) and the row's diagonal entry (block), whose terms
//            are exactly the row's pairs in order, so it needs no slots.
// K_local therefore never leaves the chip, every output is written exactly
// once, and no atomics touch values: the result is bitwise reproducible and
// independent of the launch geometry.
#include <type_traits>

#include "tg_device.h"

namespace tg {
namespace {

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


// ---------------------------------------------------------------- P1 scalar forms

// Sum of src[slot[u]] for u in [u0, u1), added strictly left to right.  The
// slot indices and values are read four at a time so that the dependent LDS
// round trips overlap; the order of the additions is unchanged.
template <typename T, int STRIDE = 1, typename S>
__device__ __forceinline__ T segment_sum(const T *__restrict__ src, const S *__restrict__ slot, int u0, int u1,
                                         int off = 0) {
    T acc = 0;
    int u = u0;
    for (; u + 4 <= u1; u += 4) {
        const int a0 = slot[u], a1 = slot[u + 1], a2 = slot[u + 2], a3 = slot[u + 3];
        const T k0 = src[a0 * STRIDE + off], k1 = src[a1 * STRIDE + off];
        const T k2 = src[a2 * STRIDE + off], k3 = src[a3 * STRIDE + off];
        acc += k0;
        acc += k1;
        acc += k2;
        acc += k3;
    }
    for (; u < u1; ++u) acc += src[slot[u] * STRIDE + off];
    return acc;
}

// Dynamic LDS of one P2 row block: local matrices, loads, and the block's
// share of the routing (segment pointers and slot list, copied in with
// coalesced loads, so the Reduce touches only LDS).
template <typename T>
struct BlockLds {
    T *K;            // [mp * kk]  local matrix entries (kk = 9 k: 3x3 blocks)
    T *F;            // [mp * nc]  local load entries
    int32_t *seg;    // [me + 1]   segment starts, relative to the block's first slot
    uint16_t *slot;  // [mp * k]   slots of the block, in CSR entry order
    __device__ BlockLds(unsigned char *base, int mp, int me, int kk, int nc) {
        K = reinterpret_cast<T *>(base);
        F = K + (size_t)mp * kk;
        seg = reinterpret_cast<int32_t *>(F + (size_t)mp * nc);
        slot = reinterpret_cast<uint16_t *>(seg + ((me + 2) & ~1));
    }
    __host__ __device__ static size_t bytes(int mp, int me, int kk, int nc, int k) {
        return sizeof(T) * (size_t)mp * (kk + nc) + sizeof(int32_t) * (size_t)((me + 2) & ~1) +
               sizeof(uint16_t) * (size_t)mp * k;
    }
};

// Row a (run time) of a [D+1][D] table as sum_k [a == k] C_k: exact (a product
// by 1 and sums with zeros), branch-free, and with no run-time index into the
// table (a select of two table entries can be folded into a load through a
// selected address, which sends the table to scratch memory).
template <int D, typename T>
__device__ __forceinline__ void select_row(const T (&C)[D + 1][D], int a, T (&out)[D]) {
#pragma unroll
    for (int c = 0; c < D; ++c) out[c] = (T)0;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        const T m = (a == k) ? (T)1 : (T)0;
#pragma unroll
        for (int c = 0; c < D; ++c) out[c] += m * C[k][c];
    }
}

// P1 scalar forms handled by one kernel.
enum P1Form { kLaplace = 0, kMass = 1, kMassLaplace = 2 };

// Geometry of the pair's element, computed once and reused for every
// coefficient set of a batched call.
template <int D>
struct P1Geom {
    double C[D + 1][D];  // cofactor rows (det J grad(lambda_b))
    double adet;         // |det J|
    bool bad;            // numerically singular
};

template <int D>
__device__ __forceinline__ void p1_geometry(const double (&x)[D + 1][D], P1Geom<D> &g) {
    const double det = p1_cofactors<D>(x, g.C);
    g.adet = fabs(det);
    g.bad = numerically_singular<D>(x, det);
}

// Row a of the local matrix and entry a of the local load of one pair for
// coefficient c and source f:
//   Laplace:      K_ab = c (C_a . C_b) / (d! |det J|)       (1-point rule, exact)
//   Mass:         M_ab = sum_q w_q |det J| phi_a(x_q) phi_b(x_q)  (degree-2 rule)
//   MassLaplace:  M_ab + K_ab
// F_a = f |det J| / (d! (d+1)) (centroid rule, exact for constant f).
template <int D, typename T, int FORM>
__device__ __forceinline__ void p1_row(const P1Geom<D> &g, int a, double c, double f, T (&row)[D + 1], T &fa) {
    constexpr int K = D + 1;
    T kr[K];
#pragma unroll
    for (int b = 0; b < K; ++b) kr[b] = (T)0;
    if constexpr (FORM != kMass) {
        const T sc = (T)(c / (g.adet * (1.0 / RefSimplex<D>::vol)));
        // the cofactors rounded to T first (selecting a row is exact, so this
        // equals rounding the selected row)
        T Ct[K][D];
#pragma unroll
        for (int b = 0; b < K; ++b)
#pragma unroll
            for (int k = 0; k < D; ++k) Ct[b][k] = (T)g.C[b][k];
        T ca[D];
        select_row<D, T>(Ct, a, ca);
#pragma unroll
        for (int b = 0; b < K; ++b) {
            T sum = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) sum += ca[k] * Ct[b][k];
            kr[b] = sc * sum;
        }
    }
#pragma unroll
    for (int b = 0; b < K; ++b) {
        if constexpr (FORM == kLaplace) {
            row[b] = kr[b];
        } else {
            using R = Deg2Rule<D>;
            double m = 0.0;
#pragma unroll
            for (int q = 0; q < R::Q; ++q) {
                const double pa = (a == q) ? R::hi : R::lo;
                const double pb = (b == q) ? R::hi : R::lo;
                m += R::w * pa * pb;
            }
            const T mv = (T)(g.adet * m);
            row[b] = (FORM == kMass) ? mv : mv + kr[b];
        }
    }
    fa = (T)(f * g.adet * (RefSimplex<D>::vol / K));  // phi_a(centroid) = 1/(d+1)
}

// Per-block LDS copy of the vertex coordinates: VS doubles per vertex (16-byte
// records), placed after the other per-block arrays.
template <int D>
struct VertLds {
    static constexpr int VS = D == 3 ? 4 : 2;
    __host__ __device__ static size_t offset(size_t block_lds_bytes) { return (block_lds_bytes + 15) & ~(size_t)15; }
    __host__ __device__ static size_t bytes(int nverts) { return sizeof(double) * VS * (size_t)nverts; }
};

// Vertex l of the block's list -> LDS (coordinates are AoS [Nv][D] FP64).
template <int D>
__device__ __forceinline__ void stage_vertex(const double *__restrict__ coords, unsigned v, double *lx) {
    if constexpr (D == 3) {
        const double x0 = ldg(coords, 3u * v), x1 = ldg(coords, 3u * v + 1u), x2 = ldg(coords, 3u * v + 2u);
        *reinterpret_cast<double2 *>(lx) = make_double2(x0, x1);
        lx[2] = x2;
    } else {
        *reinterpret_cast<double2 *>(lx) = ldg(reinterpret_cast<const double2 *>(coords), v);
    }
}

// The element's vertices from the block's LDS copy; lv holds one 8-bit local id per vertex.
template <int D>
__device__ __forceinline__ void lds_vertices(const double *lx, uint32_t lv, double (&x)[D + 1][D]) {
    constexpr int VS = VertLds<D>::VS;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        const double *r = lx + ((lv >> (8 * a)) & 255u) * VS;
        const double2 xy = *reinterpret_cast<const double2 *>(r);
        x[a][0] = xy.x;
        x[a][1] = xy.y;
        if constexpr (D == 3) x[a][2] = r[2];
    }
}

template <typename T> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

// Dynamic LDS of one P1 row block (mp pairs, me node entries, mr rows at most):
//   K    [mp * k]  row a of every pair's local matrix: column-major (b * np + t)
//                  for the wide routing, row-major (t * k + b) for the compact one
//   DF   [mp]      every pair's diagonal entry K_e[a][a] and load entry F_e[a]
//   seg  [me + 1]  wide: segment starts relative to sb (int32); compact: the
//                  entries' ent16 codes (uint16) and a sentinel
//   slot [mp (k-1) + 8]  the block's routing slots (uint16 wide, uint8 compact)
//                  from the 4-aligned base sb
//   ip   [mr + 1]  first pair of every row of the block
template <typename T, bool COMPACT>
struct P1Lds {
    using T2 = typename Pair2<T>::type;
    using Seg = typename std::conditional<COMPACT, uint16_t, int32_t>::type;
    using Slot = typename std::conditional<COMPACT, uint8_t, uint16_t>::type;
    T *K;
    T2 *DF;
    Seg *seg;
    Slot *slot;
    int32_t *ip;
    __host__ __device__ static size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }
    __host__ __device__ static size_t off_df(int mp, int k) { return a16(sizeof(T) * (size_t)mp * k); }
    __host__ __device__ static size_t off_seg(int mp, int k) { return a16(off_df(mp, k) + sizeof(T2) * (size_t)mp); }
    __host__ __device__ static size_t off_slot(int mp, int me, int k) {
        return a16(off_seg(mp, k) + sizeof(Seg) * (size_t)(me + 1));
    }
    __host__ __device__ static size_t off_ip(int mp, int me, int k) {
        return a16(off_slot(mp, me, k) + sizeof(Slot) * ((size_t)mp * (k - 1) + 8));
    }
    __host__ __device__ static size_t bytes(int mp, int me, int mr, int k) {
        return a16(off_ip(mp, me, k) + sizeof(int32_t) * (size_t)(mr + 1));
    }
    __device__ P1Lds(unsigned char *base, int mp, int me, int k) {
        K = reinterpret_cast<T *>(base);
        DF = reinterpret_cast<T2 *>(base + off_df(mp, k));
        seg = reinterpret_cast<Seg *>(base + off_seg(mp, k));
        slot = reinterpret_cast<Slot *>(base + off_slot(mp, me, k));
        ip = reinterpret_cast<int32_t *>(base + off_ip(mp, me, k));
    }
};

// Descriptor prefetch distance, in blocks (see p1_assemble_kernel).
constexpr int kP1DescAhead = 256;
constexpr int kP2DescAhead = 128;  // about one round of P2 workgroups on an XCD
constexpr int kP2PhaseCols = 6;     // column nodes of a P2 pair held in LDS at once (the edges)
constexpr int kP2ClsLen = (kP2BlockCap + 1 + 3) & ~3;  // class prefixes of a P2 block, padded to int4s

// Minimum waves per SIMD the register allocation must allow: 8 for the
// single-set Laplace kernels (they fit in 64 VGPRs without spilling), 7 for the
// mass forms, 5 (Laplace) or 4 (mass forms) for the batched kernels (they keep
// the pair's geometry live across the member loop).
template <typename T, int FORM, bool BATCHED>
constexpr int p1_waves_per_eu() {
    return BATCHED ? (FORM == 0 ? 5 : 4) : (FORM == 0 ? 8 : 7);
}

// Fused Map + Reduce over a batch of coefficient sets (nbatch >= 1; a plain
// call is nbatch = 1).  Member m reads coef[m E + e] and load[m E + e] and
// writes values[m nnz + p] and rhs[m N + i]; the geometry and the routing are
// read once for the whole batch.  Every member runs exactly the arithmetic
// of a single call, so it is bitwise equal to assembling it alone.  COMPACT
// selects the one-byte routing (ent16 / slot8) over the wide one (seg_ptr /
// slot); both name the same slots in the same order.
template <int D, typename T, int FORM, bool LOAD, bool BATCHED, bool COMPACT>
__global__ __launch_bounds__(kP1Threads) __attribute__((amdgpu_waves_per_eu(p1_waves_per_eu<T, FORM, BATCHED>())))
void p1_assemble_kernel(
    const int32_t *__restrict__ blk_desc, const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc,
    const void *__restrict__ seg_v, const void *__restrict__ slot_v, const int32_t *__restrict__ blk_vert,
    const uint32_t *__restrict__ pair_lv, const int32_t *__restrict__ diag_pos, const double *__restrict__ coords,
    const T *__restrict__ coef, const T *__restrict__ load, T *__restrict__ values, T *__restrict__ rhs,
    int32_t *__restrict__ status, int nblk, int mp, int me, int nbatch, unsigned n_elem, unsigned nnz,
    unsigned n_rows, unsigned lds_verts) {
    constexpr int K = D + 1;
    constexpr int VS = VertLds<D>::VS;
    constexpr bool COEF = FORM != kMass;
    using LdsT = P1Lds<T, COMPACT>;
    using T2 = typename LdsT::T2;
    using Seg = typename LdsT::Seg;
    static_assert(kP1BlockVerts <= kP1Threads, "one staged vertex per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    LdsT L(smem, mp, me, K);
    double *Lx = reinterpret_cast<double *>(smem + lds_verts);
    const Seg *__restrict__ seg_g = static_cast<const Seg *>(seg_v);  // seg_ptr (wide) or ent16 (compact)
    // the slot list as 8-byte units (4 wide slots) or 4-byte units (4 compact slots)
    using Unit = typename std::conditional<COMPACT, uint32_t, uint2>::type;
    const Unit *__restrict__ slot_u = static_cast<const Unit *>(slot_v);

    const int blk = xcd_swizzle(blockIdx.x, nblk);
    const int4 dsc = ldg(reinterpret_cast<const int4 *>(blk_desc), 3u * blk);
    const int4 dsv = ldg(reinterpret_cast<const int4 *>(blk_desc), 3u * blk + 1u);
    const int r0 = dsc.x, r1 = dsc.y, q0 = dsc.z, q1 = dsc.w, v0 = dsv.x, v1 = dsv.y, w0 = dsv.z, w1 = dsv.w;
    const int np = q1 - q0, nent = v1 - v0, nvb = w1 - w0, nr = r1 - r0;
    // the block's slots: wide slot[s0 .. s1) from the descriptor; compact slot8[q0 (k-1) .. q1 (k-1));
    // copied in 4-slot units from sb = s0 rounded down to 4
    int s0, s1;
    if constexpr (COMPACT) {
        s0 = q0 * (K - 1);
        s1 = q1 * (K - 1);
    } else {
        const int2 dss = ldg(reinterpret_cast<const int2 *>(blk_desc), 6u * blk + 4u);
        s0 = dss.x;
        s1 = dss.y;
    }
    const int sb = s0 & ~3;
    const int nu = (s1 - sb + 3) >> 2;
    const int tid = threadIdx.x;
    const int rr = kP1Threads - 1 - tid;  // the row this thread sums (the Reduce's last threads)
    const int nmem = BATCHED ? nbatch : 1;

    if (np == 0) {  // rows of nodes that belong to no element: no values, zero loads
        if (LOAD)
            for (int m = 0; m < nmem; ++m)
                for (int r = r0 + tid; r < r1; r += kP1Threads) stg(rhs, (unsigned)m * n_rows + (unsigned)r, (T)0);
        return;
    }

    // ---- Every load that needs only the block descriptor, issued back to back
    // with clamped (always valid) indices and no branches, so that their
    // latencies overlap: the vertex this thread stages, its pair's code and
    // local vertex ids, a 4-slot unit of the routing, one entry's segment
    // pointer (or code), one row offset and one row's diagonal position.  Then
    // the loads that need one of them: the staged vertex's coordinates and the
    // pair's coefficients.  Two memory latencies in all.
    const int tp = min(tid, np - 1);
    const unsigned vid = (unsigned)ldg(blk_vert, (unsigned)(w0 + min(tid, nvb - 1)));
    const unsigned code = (unsigned)ldg(inc, (unsigned)(q0 + tp));
    const uint32_t lv = ldg(pair_lv, (unsigned)(q0 + tp));
    const int te = COMPACT ? min(tid, nent - 1) : min(tid, nent);  // compact: the sentinel is written below
    const Seg seg_reg = ldg(seg_g, (unsigned)(v0 + te));
    const int ip_reg = ldg(inc_ptr, (unsigned)(r0 + min(tid, nr)));
    const int dp_reg = ldg(diag_pos, (unsigned)(r0 + min(rr, nr - 1)));
    const Unit slot_w = ldg(slot_u, (unsigned)(sb >> 2) + (unsigned)min(tid, nu - 1));
    double vxyz[D];
    if constexpr (D == 3) {
        vxyz[0] = ldg(coords, 3u * vid);
        vxyz[1] = ldg(coords, 3u * vid + 1u);
        vxyz[2] = ldg(coords, 3u * vid + 2u);
    } else {
        const double2 xy = ldg(reinterpret_cast<const double2 *>(coords), vid);
        vxyz[0] = xy.x;
        vxyz[1] = xy.y;
    }
    const unsigned e = code / K;
    const int a = (int)(code - e * K);
    T c_next = COEF ? ldg(coef, e) : (T)1;  // member 0's coefficients (then each next member's)
    T f_next = LOAD ? ldg(load, e) : (T)0;
    // Bring into L2 the descriptor of the block that starts on this XCD about one
    // round of workgroups later (32 CUs x 8 resident blocks), so that its first,
    // dependent load hits: a vector load issued after this block's own loads and
    // consumed only at the end.
    const int pf_desc = ldg(blk_desc, (unsigned)(min(blk + kP1DescAhead, nblk - 1) * kBlkDesc + (tid & 7)));

    // ---- staged vertex and routing -> LDS, also without branches: a thread past
    // the end of a list writes the last element's value to the last element's
    // place, the same value its owner writes there.  (A branch here lets the
    // compiler sink the loads into it, behind a wait for every earlier load.)
    const bool own = tid < np;
    {
        double *lx = Lx + min(tid, nvb - 1) * VS;
        *reinterpret_cast<double2 *>(lx) = make_double2(vxyz[0], vxyz[1]);
        if constexpr (D == 3) lx[2] = vxyz[2];
    }
    reinterpret_cast<Unit *>(L.slot)[min(tid, nu - 1)] = slot_w;
    if constexpr (COMPACT) {
        L.seg[te] = seg_reg;
        if (tid == 0) L.seg[nent] = (uint16_t)(nr << 8);  // sentinel: row nr, offset 0 = the block's end
    } else {
        L.seg[te] = seg_reg - sb;
    }
    L.ip[min(tid, nr)] = ip_reg - q0;
    // remainders of large blocks (a single row with more pairs, entries or rows than threads)
    for (int u = tid + kP1Threads; u < nu; u += kP1Threads)
        reinterpret_cast<Unit *>(L.slot)[u] = ldg(slot_u, (unsigned)((sb >> 2) + u));
    for (int u = tid + kP1Threads; u < nent + (COMPACT ? 0 : 1); u += kP1Threads)
        L.seg[u] = COMPACT ? ldg(seg_g, (unsigned)(v0 + u)) : (Seg)(ldg(seg_g, (unsigned)(v0 + u)) - sb);
    for (int u = tid + kP1Threads; u <= nr; u += kP1Threads) L.ip[u] = ldg(inc_ptr, (unsigned)(r0 + u)) - q0;
    __syncthreads();  // vertices and routing are in LDS

    // ---- Map geometry of this thread's pair (kept for the whole batch)
    P1Geom<D> g;
    g.adet = 1.0;
    g.bad = false;
    if (own) {
        double x[K][D];
        lds_vertices<D>(Lx, lv, x);
        p1_geometry<D>(x, g);
    }

    for (int m = 0; m < nmem; ++m) {
        const unsigned eo = (unsigned)m * n_elem;
        const double c = (double)c_next, f = (double)f_next;
        if (BATCHED && m + 1 < nmem) {  // the next member's coefficients, fetched ahead
            if (COEF) c_next = ldg(coef, eo + n_elem + e);
            if (LOAD) f_next = ldg(load, eo + n_elem + e);
        }
        // ---- Map: row a of the local matrix (and F_e[a]) for member m
        if (own) {
            T row[K], fa;
            p1_row<D, T, FORM>(g, a, c, f, row, fa);
            T kd = row[0];
#pragma unroll
            for (int b = 1; b < K; ++b) kd = (a == b) ? row[b] : kd;
#pragma unroll
            for (int b = 0; b < K; ++b) L.K[COMPACT ? tid * K + b : b * np + tid] = row[b];
            L.DF[tid] = T2{kd, fa};
            const bool bad = (bool)((int)g.bad | (int)!finite(c) | (int)!finite(f));
            if (bad && status) atomicMin(status, (int)e);
        }
        for (int t = tid + kP1Threads; t < np; t += kP1Threads) {  // a single row with more pairs than threads
            const unsigned code_t = (unsigned)ldg(inc, (unsigned)(q0 + t));
            const unsigned ee = code_t / K;
            const int at = (int)(code_t - ee * K);
            double x[K][D];
            lds_vertices<D>(Lx, ldg(pair_lv, (unsigned)(q0 + t)), x);
            P1Geom<D> gg;
            p1_geometry<D>(x, gg);
            const double ct = COEF ? (double)ldg(coef, eo + ee) : 1.0;
            const double ft = LOAD ? (double)ldg(load, eo + ee) : 0.0;
            T row[K], fa;
            p1_row<D, T, FORM>(gg, at, ct, ft, row, fa);
            T kd = row[0];
#pragma unroll
            for (int b = 1; b < K; ++b) kd = (at == b) ? row[b] : kd;
#pragma unroll
            for (int b = 0; b < K; ++b) L.K[COMPACT ? t * K + b : b * np + t] = row[b];
            L.DF[t] = T2{kd, fa};
            if (((int)gg.bad | (int)!finite(ct) | (int)!finite(ft)) && status) atomicMin(status, (int)ee);
        }
        __syncthreads();

        // ---- Reduce: off-diagonal CSR values of the block rows (S_mat
        // projection), LDS only; a row's diagonal entry has no slots.
        const unsigned vo = (unsigned)m * nnz;
        for (int p = tid; p < nent; p += kP1Threads) {
            if constexpr (COMPACT) {
                const unsigned e0 = L.seg[p], e1 = L.seg[p + 1];
                const int u0 = L.ip[e0 >> 8];
                const int sa = s0 - sb + u0 * (K - 1) + (int)(e0 & 255u);
                const int se = s0 - sb + L.ip[e1 >> 8] * (K - 1) + (int)(e1 & 255u);
                if (sa != se) stg(values, vo + (unsigned)(v0 + p), segment_sum<T>(L.K + u0 * K, L.slot, sa, se));
            } else {
                const int sa = L.seg[p], se = L.seg[p + 1];
                if (sa != se) stg(values, vo + (unsigned)(v0 + p), segment_sum<T>(L.K, L.slot, sa, se));
            }
        }
        // ---- Reduce per row, on the threads from the last one down: the diagonal
        // entry (every pair of the row contributes K_e[a][a]) and the right-hand
        // side (S_vec projection), both in the row's pair order.
        const unsigned ro = (unsigned)m * n_rows;
        for (int r = rr; r < nr; r += kP1Threads) {
            const int u0 = L.ip[r], u1 = L.ip[r + 1];
            T accd = 0, accf = 0;
            int u = u0;
            for (; u + 4 <= u1; u += 4) {
                const T2 d0 = L.DF[u], d1 = L.DF[u + 1], d2 = L.DF[u + 2], d3 = L.DF[u + 3];
                accd += d0.x;
                accf += d0.y;
                accd += d1.x;
                accf += d1.y;
                accd += d2.x;
                accf += d2.y;
                accd += d3.x;
                accf += d3.y;
            }
            for (; u < u1; ++u) {
                const T2 d0 = L.DF[u];
                accd += d0.x;
                accf += d0.y;
            }
            const int dp = r == rr ? dp_reg : ldg(diag_pos, (unsigned)(r0 + r));
            stg(values, vo + (unsigned)dp, accd);
            if (LOAD) stg(rhs, ro + (unsigned)(r0 + r), accf);
        }
        if (m + 1 < nmem) __syncthreads();  // LDS is rewritten by the next member
    }
    asm volatile("" ::"v"(pf_desc));  // keeps the prefetch (its value is not needed)
}

// ---------------------------------------------------------------- P2 elasticity

// The 3x3 block of Hooke's law (Sec. B.1.1), lam D + mu (D^T + tr(D) I), for a
// rank-one D = u w^T, given L = lam u and M = mu u: L w^T + w M^T + (M . w) I.
template <typename T>
__device__ __forceinline__ void hooke_rank1(const T (&L)[3], const T (&M)[3], const T (&w)[3], T *o) {
    const T tr = M[0] * w[0] + M[1] * w[1] + M[2] * w[2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) o[c * 3 + cc] = L[c] * w[cc] + w[c] * M[cc] + (c == cc ? tr : (T)0);
}

// The same for D = u p^T + v q^T, given L = lam u, M = mu u, Lv = lam v, Mv = mu v.
template <typename T>
__device__ __forceinline__ void hooke_rank2(const T (&L)[3], const T (&M)[3], const T (&p)[3], const T (&Lv)[3],
                                            const T (&Mv)[3], const T (&q)[3], T *o) {
    const T tr = M[0] * p[0] + M[1] * p[1] + M[2] * p[2] + Mv[0] * q[0] + Mv[1] * q[1] + Mv[2] * q[2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            o[c * 3 + cc] = L[c] * p[cc] + Lv[c] * q[cc] + p[c] * M[cc] + q[c] * Mv[cc] + (c == cc ? tr : (T)0);
}

// The element row of one P2 pair, in the pair's frame: the routing and the
// staged vertex ids order the element's vertices so that the pair's node is
// vertex 0 (a vertex node) or edge (0, 1) (an edge node), the column nodes
// numbered in the same frame (vertices 0..3, then edges (0,1),(0,2),(0,3),
// (1,2),(1,3),(2,3)).  With V the element volume, g_v = grad(lambda_v) and the
// exact integrals int lambda_p = V/4, int lambda_p lambda_q = V (1 + [p = q])/20
// of the quadratic basis (vertex: lambda (2 lambda - 1); edge (i, j):
// 4 lambda_i lambda_j), D = int grad(phi_a) grad(phi_b)^T is
//   vertex node:  D = V g_0 w^T,  w = 3/5 g_0 (b = 0), -1/5 g_b (b = 1..3),
//                 3/5 g_j - 1/5 g_0 (edge (0, j)), -1/5 (g_i + g_j) (edge (i, j), 0 < i);
//   edge node:    vertex b: D = w g_b^T,  w = V (3/5 g_1 - 1/5 g_0) (b = 0),
//                 V (3/5 g_0 - 1/5 g_1) (b = 1), -V/5 (g_0 + g_1) (b = 2, 3);
//                 edge (k, l): D = 4/5 V (g_1 p^T + g_0 q^T) with
//                 p = (1 + [k = 0]) g_l + (1 + [l = 0]) g_k, q = (1 + [k = 1]) g_l + (1 + [l = 1]) g_k,
// then Hooke's law.  (The same integrals as the degree-2 rule of the
// quadrature, which is exact for them.)
template <typename T>
struct P2Pair {
    T g[4][3];  // grad(lambda_v) in the frame
    // vertex node: L0 = lam V g_0, M0 = mu V g_0 (L1, M1 unused);
    // edge node: L0, L1, M0, M1 = 4/5 V (lam g_0, lam g_1, mu g_0, mu g_1)
    T L0[3], L1[3], M0[3], M1[3];

    __device__ __forceinline__ void init(bool edge, T V, T lam, T mu) {
        const T s = edge ? (T)0.8 * V : V, ls = lam * s, ms = mu * s;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            L0[c] = ls * g[0][c];
            M0[c] = ms * g[0][c];
            L1[c] = ls * g[1][c];
            M1[c] = ms * g[1][c];
        }
    }

    // block (a, B) of a vertex node, written to o[0 .. 9) (row-major 3x3)
    template <int B>
    __device__ __forceinline__ void vertex_block(T *o) const {
        T w[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (B == 0) {
                w[c] = (T)0.6 * g[0][c];
            } else if constexpr (B < 4) {
                w[c] = (T)-0.2 * g[B][c];
            } else if constexpr (B < 7) {
                w[c] = (T)0.6 * g[B - 3][c] - (T)0.2 * g[0][c];
            } else {
                constexpr int i = B < 9 ? 1 : 2, j = B == 7 ? 2 : 3;
                w[c] = (T)-0.2 * (g[i][c] + g[j][c]);
            }
        }
        hooke_rank1<T>(L0, M0, w, o);
    }

    // block (a, B) of an edge node
    template <int B>
    __device__ __forceinline__ void edge_block(T *o) const {
        if constexpr (B < 4) {  // lam w and mu w from the stored 4/5 V lam g_0, ...
            T Lw[3], Mw[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (B == 0) {
                    Lw[c] = (T)0.75 * L1[c] - (T)0.25 * L0[c];
                    Mw[c] = (T)0.75 * M1[c] - (T)0.25 * M0[c];
                } else if constexpr (B == 1) {
                    Lw[c] = (T)0.75 * L0[c] - (T)0.25 * L1[c];
                    Mw[c] = (T)0.75 * M0[c] - (T)0.25 * M1[c];
                } else {
                    Lw[c] = (T)-0.25 * (L0[c] + L1[c]);
                    Mw[c] = (T)-0.25 * (M0[c] + M1[c]);
                }
            }
            hooke_rank1<T>(Lw, Mw, g[B], o);
        } else if constexpr (B == 9) {  // edge (2, 3): p = q = g_2 + g_3
            T p[3], Ls[3], Ms[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                p[c] = g[2][c] + g[3][c];
                Ls[c] = L0[c] + L1[c];
                Ms[c] = M0[c] + M1[c];
            }
            hooke_rank1<T>(Ls, Ms, p, o);
        } else {
            constexpr int k = B < 7 ? 0 : 1, l = B == 4 ? 1 : ((B == 5 || B == 7) ? 2 : 3);
            constexpr T pk = (T)(1 + (l == 0)), pl = (T)(1 + (k == 0));  // p = pl g_l + pk g_k
            constexpr T qk = (T)(1 + (l == 1)), ql = (T)(1 + (k == 1));  // q = ql g_l + qk g_k
            T p[3], q[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                p[c] = pl * g[l][c] + pk * g[k][c];
                q[c] = ql * g[l][c] + qk * g[k][c];
            }
            hooke_rank2<T>(L1, M1, p, L0, M0, q, o);
        }
    }

    template <int B>
    __device__ __forceinline__ void block(bool edge, T *o) const {
        if (edge)
            edge_block<B>(o);
        else
            vertex_block<B>(o);
    }
};

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

// Reduce of one column class of a P2 block: one lane per node-level entry
// whose column is an edge node (edge) or a vertex node (!edge) sums its routed
// 3x3 blocks (ascending element order, components in parallel) and writes the
// 9 scalars.  A row's vertex-node columns precede its edge-node columns
// (vertices are numbered first), so the class's entries of block row r are a
// run of the row: cls[r] of them come before it in the block (cls = sVp or
// sEp, block-relative prefixes), and lane t takes the class's t-th entry.
// The class's blocks sit in LDS at (slot - first slot of the class) * 9, slot
// = b np + pair.  Entry pe of row r, column position jpos, lands at 9 sRp[r]
// + c (3 m) + 3 jpos + cc of the block's value range (the 3 DoF rows of a
// node share its columns).  Diagonal entries (empty segments) are skipped.
// cls holds kP2ClsLen values, INT_MAX past the block's last row, so the row
// is found four prefix values (one 16-byte LDS read) at a time; slots are
// taken two at a time (their indices, then their blocks, in one LDS round
// trip each), the sum still in slot order.
template <typename T>
__device__ __forceinline__ void p2_reduce(const BlockLds<T> &L, const int *sRp, const int *sVp, const int *cls,
                                          int ncls, int np, bool edge, T *__restrict__ out) {
    const int first = edge ? 4 * np : 0;
    for (int t = threadIdx.x; t < ncls; t += kP2Threads) {
        int j = 0, cnt;
        do {  // rows r with cls[r] <= t (cls[0] = 0, non-decreasing): r = their count - 1
            const int4 c = reinterpret_cast<const int4 *>(cls)[j++];
            cnt = (c.x <= t) + (c.y <= t) + (c.z <= t) + (c.w <= t);
        } while (cnt == 4);
        const int r = 4 * (j - 1) + cnt - 1;
        const int m = sRp[r + 1] - sRp[r];
        const int jpos = (edge ? sVp[r + 1] - sVp[r] : 0) + (t - cls[r]);
        const int pe = sRp[r] + jpos;
        const int u0 = L.seg[pe], u1 = L.seg[pe + 1];
        if (u0 == u1) continue;
        T acc[9];
#pragma unroll
        for (int z = 0; z < 9; ++z) acc[z] = 0;
        int u = u0;
        for (; u + 2 <= u1; u += 2) {  // two slots per round trip of slot reads, then of block reads
            const T *s0 = L.K + ((int)L.slot[u] - first) * 9;
            const T *s1 = L.K + ((int)L.slot[u + 1] - first) * 9;
            T b0[9], b1[9];
#pragma unroll
            for (int z = 0; z < 9; ++z) {
                b0[z] = s0[z];
                b1[z] = s1[z];
            }
#pragma unroll
            for (int z = 0; z < 9; ++z) acc[z] = (acc[z] + b0[z]) + b1[z];
        }
        if (u < u1) {
            const T *s0 = L.K + ((int)L.slot[u] - first) * 9;
#pragma unroll
            for (int z = 0; z < 9; ++z) acc[z] += s0[z];
        }
        // 32-bit offsets from the block's (uniform) output base
        const unsigned ob = (unsigned)(9 * sRp[r] + 3 * jpos);
        const unsigned base_odd = (unsigned)(reinterpret_cast<uintptr_t>(out) >> 3) & 1u;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const unsigned oc = ob + (unsigned)(c * 3 * m);
            if constexpr (sizeof(T) == 8) {
                // the three values as a 16-byte store at a 16-byte boundary and one 8-byte store
                const bool odd = ((oc + base_odd) & 1u) != 0;
                double2 v2;
                v2.x = odd ? acc[c * 3 + 1] : acc[c * 3];
                v2.y = odd ? acc[c * 3 + 2] : acc[c * 3 + 1];
                *reinterpret_cast<double2 *>(reinterpret_cast<char *>(out) + (oc + (odd ? 1u : 0u)) * 8u) = v2;
                stg(out, oc + (odd ? 0u : 2u), odd ? acc[c * 3] : acc[c * 3 + 2]);
            } else {  // one 12-byte store
                T *o = out + oc;
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) o[cc] = acc[c * 3 + cc];
            }
        }
    }
}

// v[s t] summed left to right over t0 <= t < t1, four LDS reads per round trip.
template <typename T>
__device__ __forceinline__ T seq_sum(const T *v, int s, int t0, int t1) {
    T acc = 0;
    int t = t0;
    for (; t + 4 <= t1; t += 4) {
        const T a0 = v[s * t], a1 = v[s * (t + 1)], a2 = v[s * (t + 2)], a3 = v[s * (t + 3)];
        acc += a0;
        acc += a1;
        acc += a2;
        acc += a3;
    }
    for (; t < t1; ++t) acc += v[s * t];
    return acc;
}

// Diagonal blocks of the rows whose node is in this phase's class (vertex or
// edge node: the class of its local index in every element): component z of
// row r is the sum, over the row's pairs t in S_vec (ascending element) order,
// of component z of the pair's block (a_t, a_t) (column 0 or 4 of the pair's
// frame: the first block of the phase); nine lanes per row.  The routing
// lists no slots for these entries.  Written at the scalar CSR
// positions diag_pos[3 i] + c (3 m) + c' (m: node entries of the row; sDp[r]
// = diag_pos[3 i] for the block's row r of node i).
template <typename T>
__device__ __forceinline__ void p2_reduce_diagonal(const BlockLds<T> &L, const int *sIp, const uint8_t *sA,
                                                   const int *sDp, const int *sRp, int nrows, bool edge,
                                                   T *__restrict__ values) {
    for (int u = threadIdx.x; u < 9 * nrows; u += kP2Threads) {
        const int r = u / 9, z = u - 9 * r;
        const int t0 = sIp[r], t1 = sIp[r + 1];
        if (t0 == t1 || ((int)sA[t0] >= 4) != edge) continue;
        const T acc = seq_sum<T>(L.K + z, 9, t0, t1);
        const int c = z / 3;
        values[sDp[r] + c * 3 * (sRp[r + 1] - sRp[r]) + (z - 3 * c)] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(kP2Threads) void p2_elasticity_kernel(
    const int32_t *__restrict__ blk_desc, const int32_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ node_rp, const int32_t *__restrict__ node_vp, const int32_t *__restrict__ seg_ptr,
    const uint16_t *__restrict__ slot, const int32_t *__restrict__ blk_vert, const uint32_t *__restrict__ pair_lv,
    const int32_t *__restrict__ diag_pos, const double *__restrict__ coords, const T *__restrict__ coef,
    const T *__restrict__ load, T *__restrict__ values, T *__restrict__ rhs, int32_t *__restrict__ status, int nblk,
    int E, int mp, int me) {
    constexpr int K = 10;
    constexpr int VS = VertLds<3>::VS;
    extern __shared__ __align__(16) unsigned char smem[];
    BlockLds<T> L(smem, mp, me, 9 * kP2PhaseCols, 3);
    double *Lx =
        reinterpret_cast<double *>(smem + VertLds<3>::offset(BlockLds<T>::bytes(mp, me, 9 * kP2PhaseCols, 3, K)));
    __shared__ int sRp[kP2BlockCap + 1];  // row starts in the block's node-level entries
    __shared__ __align__(16) int sVp[kP2ClsLen];  // ... of the vertex-column entries only (then INT_MAX)
    __shared__ __align__(16) int sEp[kP2ClsLen];  // ... of the edge-column entries only (then INT_MAX)
    __shared__ int sIp[kP2BlockCap + 1];  // row starts in the block's pairs
    __shared__ int sDp[kP2BlockCap];      // diagonal position of each row's first DoF row
    __shared__ uint8_t sA[kP2BlockCap];   // local node of every pair

    static_assert(kP2Threads == 3 * 64, "one wave per set of column nodes");
    static_assert(kP2BlockCap <= 64, "one lane per pair in each wave");
    const int blk = xcd_swizzle(blockIdx.x, nblk);
    const int4 dsc = ldg(reinterpret_cast<const int4 *>(blk_desc), 3u * blk);
    const int4 dsv = ldg(reinterpret_cast<const int4 *>(blk_desc), 3u * blk + 1u);
    const int4 dsw = ldg(reinterpret_cast<const int4 *>(blk_desc), 3u * blk + 2u);
    const int r0 = dsc.x, r1 = dsc.y, q0 = dsc.z, q1 = dsc.w, rp0 = dsv.x, rp1 = dsv.y, w0 = dsv.z, w1 = dsv.w;
    const int vp0 = dsw.z, vp1 = dsw.w;
    const int np = q1 - q0, nent = rp1 - rp0, nvb = w1 - w0, nvent = vp1 - vp0;
    const int nrows = r1 - r0;
    // the block's slots: K - 1 per pair (a diagonal block has none), from s0,
    // copied in 4-byte units of two from the even sb
    const int s0 = q0 * (K - 1), sb = s0 & ~1;
    const int tid = threadIdx.x, lane = tid & 63;

    if (np == 0) {  // rows of nodes that belong to no element: no values, zero loads
        if (rhs && load)
            for (int u = tid; u < 3 * nrows; u += kP2Threads) rhs[3 * (size_t)r0 + u] = (T)0;
        return;
    }

    // ---- Every load that needs only the block descriptor, issued back to back
    // with clamped (always valid) indices and no branches, so that their
    // latencies overlap: the pair of this lane (code, local vertex ids), a row's
    // two offsets (entries, pairs), two segment starts, two 2-slot units of the routing and the vertex
    // this thread stages; then the loads that need one of them (coordinates,
    // coefficients, body force).  Two memory latencies in all for blocks of at
    // most 2 kP2Threads - 1 entries and kP2Threads vertices.
    const int nsu = (q1 * (K - 1) - sb + 1) >> 1;
    const uint32_t *__restrict__ slot_u = reinterpret_cast<const uint32_t *>(slot + sb);
    const int tp = min(lane, np - 1);
    const int code = ldg(inc, (unsigned)(q0 + tp));
    const uint32_t lv = ldg(pair_lv, (unsigned)(q0 + tp));
    const int rp_reg = ldg(node_rp, (unsigned)(r0 + min(tid, nrows)));
    const int vp_reg = ldg(node_vp, (unsigned)(r0 + min(tid, nrows)));
    const int ip_reg = ldg(inc_ptr, (unsigned)(r0 + min(tid, nrows)));
    const int sg_a = ldg(seg_ptr, (unsigned)(rp0 + min(tid, nent)));
    const int sg_b = ldg(seg_ptr, (unsigned)(rp0 + min(tid + kP2Threads, nent)));
    const uint32_t su_a = ldg(slot_u, (unsigned)min(tid, nsu - 1));
    const uint32_t su_b = ldg(slot_u, (unsigned)min(tid + kP2Threads, nsu - 1));
    const unsigned vid = (unsigned)ldg(blk_vert, (unsigned)(w0 + min(tid, nvb - 1)));
    const int dp_reg = ldg(diag_pos, 3u * (unsigned)(r0 + min(tid, nrows - 1)));
    const int e = code / K, a = code - e * K;
    const T lam_t = ldg(coef, (unsigned)e), mu_t = ldg(coef, (unsigned)(E + e));
    // the body force of the pair's element (or, with no load, a valid dummy read)
    const T *__restrict__ bsrc = load ? load : coef;
    const unsigned bidx = load ? 3u * (unsigned)e : (unsigned)e, bstep = load ? 1u : 0u;
    T bf[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) bf[c] = ldg(bsrc, bidx + (unsigned)c * bstep);
    double vx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) vx[c] = ldg(coords, 3u * vid + (unsigned)c);
    // Bring into L2 the descriptor of a block that starts on this XCD a round or
    // two of workgroups later, so that its first, dependent load hits (a vector
    // load consumed only at the end).
    const int pf_desc = ldg(blk_desc, (unsigned)(min(blk + kP2DescAhead, nblk - 1) * kBlkDesc + (tid & 7)));

    // ---- LDS staging, also without branches: a thread past the end of a list
    // writes the last element's value to the last element's place, the same
    // value its owner writes there.
    sRp[min(tid, nrows)] = rp_reg - rp0;
    if (tid < kP2ClsLen) {
        sVp[tid] = tid <= nrows ? vp_reg - vp0 : INT_MAX;
        sEp[tid] = tid <= nrows ? (rp_reg - rp0) - (vp_reg - vp0) : INT_MAX;
    }
    sIp[min(tid, nrows)] = ip_reg - q0;
    L.seg[min(tid, nent)] = sg_a - sb;
    L.seg[min(tid + kP2Threads, nent)] = sg_b - sb;
    sDp[min(tid, nrows - 1)] = dp_reg;
    reinterpret_cast<uint32_t *>(L.slot)[min(tid, nsu - 1)] = su_a;
    reinterpret_cast<uint32_t *>(L.slot)[min(tid + kP2Threads, nsu - 1)] = su_b;
#pragma unroll
    for (int c = 0; c < 3; ++c) Lx[min(tid, nvb - 1) * VS + c] = vx[c];
    // remainders of large blocks (more entries or vertices than the above covers)
    for (int u = tid + 2 * kP2Threads; u <= nent; u += kP2Threads) L.seg[u] = ldg(seg_ptr, (unsigned)(rp0 + u)) - sb;
    for (int l = tid + kP2Threads; l < nvb; l += kP2Threads) {
        const unsigned v = (unsigned)ldg(blk_vert, (unsigned)(w0 + l));
#pragma unroll
        for (int c = 0; c < 3; ++c) Lx[l * VS + c] = ldg(coords, 3u * v + (unsigned)c);
    }
    __syncthreads();

    // ---- Map and Reduce in two phases, one per class of column node: every
    // entry's column is a vertex node (local b = 0..3 in each of its elements)
    // or an edge node (b = 4..9), so the vertex-column blocks can be summed
    // and written before the edge-column blocks take their place in LDS (LDS
    // for 6 blocks per pair instead of 10: more resident blocks per CU).
    // One lane per pair; in each phase wave w forms a fixed set of column nodes
    // of the pair's frame (compile-time constants), and each wave forms the
    // pair's geometry once, kept in registers for both phases.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool own = lane < np;
    const int cs = np * 9;  // LDS stride between column nodes
    T *dst = L.K + lane * 9;
    const bool edge_node = a >= 4;  // the pair's node: an edge node (frame edge (0, 1)) or a vertex node
    P2Pair<T> pr;
    if (own) {
        double x[4][3], Gd[4][3];
        lds_vertices<3>(Lx, lv, x);  // the element's vertices in the pair's frame
        const double det = p1_gradients<3>(x, Gd);
        const double adet = fabs(det);
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int c = 0; c < 3; ++c) pr.g[p][c] = (T)Gd[p][c];
        pr.init(edge_node, (T)(adet * (1.0 / 6.0)), lam_t, mu_t);
        if (wave == 0) {
            sA[lane] = (uint8_t)a;
            pr.template block<0>(edge_node, dst);
            pr.template block<1>(edge_node, dst + cs);
        } else if (wave == 1) {
            pr.template block<2>(edge_node, dst + 2 * cs);
            pr.template block<3>(edge_node, dst + 3 * cs);
        } else {  // the local load and the checks
            const double lam_d = (double)lam_t, mu_d = (double)mu_t;
            bool bad = numerically_singular<3>(x, det) || !finite(lam_d) || !finite(mu_d);
            if (load) {
                const double ia = adet * (edge_node ? p2_ref_integral(4) : p2_ref_integral(0));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double bc = (double)bf[c];
                    bad = bad || !finite(bc);
                    L.F[lane * 3 + c] = (T)(bc * ia);
                }
            }
            if (bad && status) atomicMin(status, e);
        }
    }
    __syncthreads();
    p2_reduce<T>(L, sRp, sVp, sVp, nvent, np, false, values + 9 * (size_t)rp0);
    p2_reduce_diagonal<T>(L, sIp, sA, sDp, sRp, nrows, false, values);
    __syncthreads();  // the edge-column blocks reuse the LDS of the vertex-column ones
    if (own) {
        if (wave == 0) {
            pr.template block<4>(edge_node, dst);
            pr.template block<5>(edge_node, dst + cs);
        } else if (wave == 1) {
            pr.template block<6>(edge_node, dst + 2 * cs);
            pr.template block<7>(edge_node, dst + 3 * cs);
        } else {
            pr.template block<8>(edge_node, dst + 4 * cs);
            pr.template block<9>(edge_node, dst + 5 * cs);
        }
    }
    __syncthreads();
    p2_reduce<T>(L, sRp, sVp, sEp, nent - nvent, np, true, values + 9 * (size_t)rp0);
    p2_reduce_diagonal<T>(L, sIp, sA, sDp, sRp, nrows, true, values);
    if (rhs && load) {
        for (int u = threadIdx.x; u < 3 * nrows; u += kP2Threads) {
            const int r = u / 3, c = u - 3 * r;
            rhs[3 * (size_t)(r0 + r) + c] = seq_sum<T>(L.F + c, 3, sIp[r], sIp[r + 1]);
        }
    }
    asm volatile("" ::"v"(pf_desc));  // keeps the prefetch (its value is not needed)
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <int D, typename T, int FORM, bool LOAD>
static hipError_t launch_p1_t(const tg_pattern &p, int nbatch, const double *coords, const void *coef,
                              const void *load, void *values, void *rhs, int32_t *status, hipStream_t s) {
    const DevicePattern &d = p.dev;
    const HostPattern &h = p.host;
    const int nblk = (int)h.n_blocks();
    const int mp = h.max_block_pairs, me = h.max_block_entries, mr = h.max_block_rows;
    auto go = [&](auto batched, auto compact) {
        constexpr bool B = decltype(batched)::value, C = decltype(compact)::value;
        const size_t lds_verts = VertLds<D>::offset(P1Lds<T, C>::bytes(mp, me, mr, D + 1));
        const size_t lds = lds_verts + VertLds<D>::bytes(h.max_block_verts);
        const void *seg = C ? (const void *)d.ent16 : (const void *)d.seg_ptr;
        const void *slot = C ? (const void *)d.slot8 : (const void *)d.slot;
        hipLaunchKernelGGL((p1_assemble_kernel<D, T, FORM, LOAD, B, C>), dim3(nblk), dim3(kP1Threads), lds, s,
                           d.blk_desc, d.inc_ptr, d.inc, seg, slot, d.blk_vert, d.pair_lv, d.diag_pos, coords,
                           (const T *)coef, (const T *)load, (T *)values, (T *)rhs, status, nblk, mp, me, nbatch,
                           (unsigned)h.E, (unsigned)h.nnz, (unsigned)h.n_dofs, (unsigned)lds_verts);
    };
    using F_ = std::false_type;
    using T_ = std::true_type;
    if (nbatch == 1)
        h.compact ? go(F_{}, T_{}) : go(F_{}, F_{});
    else
        h.compact ? go(T_{}, T_{}) : go(T_{}, F_{});
    return hipGetLastError();
}

template <int D, typename T>
static hipError_t launch_p1_d(const tg_pattern &p, tg_form form, int nbatch, const double *coords, const void *coef,
                              const void *load, void *values, void *rhs, int32_t *status, hipStream_t s) {
    const bool with_load = form != TG_MASS && load && rhs;
    switch (form) {
        case TG_MASS: return launch_p1_t<D, T, kMass, false>(p, nbatch, coords, coef, load, values, rhs, status, s);
        case TG_LAPLACE:
            return with_load ? launch_p1_t<D, T, kLaplace, true>(p, nbatch, coords, coef, load, values, rhs, status, s)
                             : launch_p1_t<D, T, kLaplace, false>(p, nbatch, coords, coef, load, values, rhs, status, s);
        case TG_MASS_LAPLACE:
            return with_load
                       ? launch_p1_t<D, T, kMassLaplace, true>(p, nbatch, coords, coef, load, values, rhs, status, s)
                       : launch_p1_t<D, T, kMassLaplace, false>(p, nbatch, coords, coef, load, values, rhs, status, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_assemble_p1(const tg_pattern &p, tg_form form, tg_dtype dtype, int nbatch, const double *coords,
                              const void *coef, const void *load, void *values, void *rhs, int32_t *status,
                              hipStream_t s) {
    const int D = p.host.dim;
    if (dtype == TG_F64) {
        if (D == 2) return launch_p1_d<2, double>(p, form, nbatch, coords, coef, load, values, rhs, status, s);
        return launch_p1_d<3, double>(p, form, nbatch, coords, coef, load, values, rhs, status, s);
    }
    if (D == 2) return launch_p1_d<2, float>(p, form, nbatch, coords, coef, load, values, rhs, status, s);
    return launch_p1_d<3, float>(p, form, nbatch, coords, coef, load, values, rhs, status, s);
}

hipError_t launch_assemble_p2(const tg_pattern &p, tg_dtype dtype, const double *coords, const void *coef,
                              const void *load, void *values, void *rhs, int32_t *status, hipStream_t s) {
    const DevicePattern &d = p.dev;
    const int nblk = (int)p.host.n_blocks();
    const int E = (int)p.host.E;
    const int mp = p.host.max_block_pairs, me = p.host.max_block_entries;
    const size_t verts = VertLds<3>::bytes(p.host.max_block_verts);
    if (dtype == TG_F64)
        hipLaunchKernelGGL(p2_elasticity_kernel<double>, dim3(nblk), dim3(kP2Threads),
                           VertLds<3>::offset(BlockLds<double>::bytes(mp, me, 9 * kP2PhaseCols, 3, 10)) + verts, s, d.blk_desc,
                           d.inc_ptr, d.inc, d.node_rp, d.node_vp, d.seg_ptr, d.slot, d.blk_vert, d.pair_lv, d.diag_pos, coords,
                           (const double *)coef, (const double *)load, (double *)values, (double *)rhs, status, nblk,
                           E, mp, me);
    else
        hipLaunchKernelGGL(p2_elasticity_kernel<float>, dim3(nblk), dim3(kP2Threads),
                           VertLds<3>::offset(BlockLds<float>::bytes(mp, me, 9 * kP2PhaseCols, 3, 10)) + verts, s, d.blk_desc,
                           d.inc_ptr, d.inc, d.node_rp, d.node_vp, d.seg_ptr, d.slot, d.blk_vert, d.pair_lv, d.diag_pos, coords,
                           (const float *)coef, (const float *)load, (float *)values, (float *)rhs, status, nblk, E,
                           mp, me);
    return hipGetLastError();
}

}  // namespace tg
