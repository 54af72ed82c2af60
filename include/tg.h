/*
 * tg.h -- C ABI of libtg: batched Galerkin assembly on unstructured simplicial
 * meshes for AMD Instinct MI355X (gfx950), after TensorGalerkin
 * (arXiv 2602.05052).
 *
 * The method (Sec. 2 "The TensorGalerkin Framework"):
 *   Stage I, Batch-Map (Alg. 1, eq. kloc1): for every element e, the Jacobian J
 *     of the affine map from the reference simplex, |det J|, the physical basis
 *     gradients G = J^{-T} grad(phi_hat), and the quadrature-weighted local
 *     matrix K_e and vector F_e.
 *   Stage II, Sparse-Reduce (Alg. 2 and the two projections above it): the
 *     global CSR values and right-hand side as fixed 0/1 routing applied to the
 *     flattened local tensors, i.e. for every CSR entry the sum of the element
 *     slots that map to it.  The routing depends only on the mesh topology and
 *     is built once per mesh.
 * Sums here are deterministic: each CSR entry adds its element contributions in
 * ascending element order, with no atomics, so repeated calls give bitwise
 * identical results on the same inputs.
 *
 * Conventions for every function:
 *   - every function returns tg_status (0 = success, < 0 = error) and never
 *     throws; on error tg_last_error() describes it;
 *   - "host" pointers are CPU memory, read during the call only;
 *   - "device" pointers are GPU memory owned by the caller (e.g. torch tensors)
 *     that must stay alive until the work enqueued on `stream` has completed;
 *   - `stream` is a hipStream_t (NULL = the default stream); kernels are
 *     enqueued on it and the call returns without waiting unless stated;
 *   - the library allocates device memory in tg_pattern_create, for the
 *     pattern's scratch on first use by tg_adjoint_p1 / tg_heat_* (grown on
 *     demand, freed with the pattern), and for a server's slots;
 *   - all indices are 0-based int32; sizes are int64.
 */
#ifndef TG_H
#define TG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TG_OK = 0,
    TG_E_ARG = -1,        /* invalid argument (detected on the host, nothing enqueued) */
    TG_E_DEGENERATE = -2, /* a bad element: numerically singular (det J ~ 0) or with a */
                          /* non-finite coefficient or load (server results)          */
    TG_E_NONFINITE = -3,  /* a CG step length, inner product or residual is not finite */
    TG_E_NOMEM = -4,      /* hipMalloc or host allocation failed                      */
    TG_E_HIP = -5,        /* a HIP runtime call failed                                */
    TG_E_NOCONV = -6,     /* tg_pcg reached max_iter without meeting rtol             */
    TG_E_STATE = -7,      /* object in the wrong state (e.g. host-only pattern)       */
    TG_E_ACCURACY = -8    /* tg_pcg: the recursive residual met rtol but the true one  */
                          /* stays above it (below the dtype's attainable accuracy)   */
} tg_status;

typedef enum { TG_F64 = 0, TG_F32 = 1 } tg_dtype;

/*
 * Bilinear/linear forms (Sec. 2 eq. pde1 with the examples of SM A.2, SM A.1
 * and Sec. B.1.1):
 *   TG_LAPLACE    K_ij = int a grad(phi_j).grad(phi_i), F_i = int f phi_i
 *                 (P1, scalar; SM A.2)
 *   TG_MASS       M_ij = int phi_j phi_i  (P1, scalar; the mass inner product
 *                 of SM A.1); no right-hand side
 *   TG_ELASTICITY K_(i,c),(j,c') = int lambda div(phi_j e_c') div(phi_i e_c)
 *                 + 2 mu eps(phi_j e_c') : eps(phi_i e_c),  F_(i,c) = int b_c phi_i
 *                 (P2 tetrahedra, Hooke's law of Sec. B.1.1); DoF = 3*node + c
 *   TG_MASS_LAPLACE  A_ij = M_ij + int c grad(phi_j).grad(phi_i), F_i = int f phi_i
 *                 (P1, scalar): the matrix M + dt K(a) of an implicit Euler step
 *                 of the method-of-lines system of SM A.1 (pass c = dt a)
 */
typedef enum { TG_LAPLACE = 0, TG_MASS = 1, TG_ELASTICITY = 2, TG_MASS_LAPLACE = 3 } tg_form;

typedef struct tg_pattern tg_pattern; /* opaque, library-owned */

/* Pass as n_dirichlet (with dirichlet_vertices = NULL) to constrain every
 * vertex of the topological boundary (faces that belong to one element). */
#define TG_BOUNDARY_ALL (-1)

/* Value a device status word must hold before tg_assemble (see there). */
#define TG_STATUS_CLEAN INT32_MAX

/* tg_pattern_create flag: build host arrays only (no GPU needed); such a
 * pattern can be queried and copied out but not assembled or solved on. */
#define TG_PATTERN_HOST_ONLY 1u

typedef struct {
    int32_t dim, order, ncomp;
    int32_t nodes_per_element; /* k: 3 or 4 (P1), 10 (P2)                     */
    int64_t n_vertices, n_elements;
    int64_t n_nodes;           /* vertices (P1) or vertices + edges (P2)      */
    int64_t n_dofs;            /* ncomp * n_nodes: rows of K, length of F     */
    int64_t nnz;               /* scalar CSR entries (both triangles)         */
    int64_t n_constrained;     /* Dirichlet DoFs                              */
    int64_t n_blocks;          /* row blocks of the fused assembly kernel     */
    const int32_t *d_row_ptr;  /* device [n_dofs + 1], NULL if host-only     */
    const int32_t *d_col_idx;  /* device [nnz], NULL if host-only             */
    size_t device_bytes;       /* device memory owned by the pattern (host-only: what an upload would take) */
    int64_t n_slot;            /* length of the routing slot list             */
    size_t scratch_bytes;      /* the pattern's scratch grown by tg_adjoint_p1 / tg_heat_* (0 until used) */
    int64_t sell_index_bytes;  /* bytes per column index of the CG iterations' sliced-ELL
                                  pattern: 2 (offsets from the row, when every column lies
                                  within 32767 of it) or 4 */
    int64_t sell_uniform_len;  /* entries per row of every slice when all slices are padded
                                  to the longest row (at most 1/32 more entries; the CG
                                  iterations then locate slices without reading the slice
                                  offsets), else 0 */
} tg_pattern_info;

/* Text of the last error on the calling thread; valid until its next tg_ call. */
const char *tg_last_error(void);

/* Library version string. */
const char *tg_version(void);

/*
 * Build the CSR pattern and the routing of one mesh topology ("precompute
 * sparse binary routing matrices based solely on mesh topology", Sec. 2
 * Stage II).  Done once per mesh; every later call reuses it.
 *
 *   dim, order, ncomp : (2|3, 1, 1) for P1 scalar forms, (3, 2, 3) for P2
 *                       elasticity; anything else is TG_E_ARG.
 *   conn              : host [n_elements][dim+1] vertex ids of each simplex
 *                       (any orientation; |det J| is used, Sec. 2 eq. kloc1).
 *   dirichlet_vertices: host [n_dirichlet] constrained vertex ids, or NULL with
 *                       n_dirichlet = 0 (none) or TG_BOUNDARY_ALL.  For P2 an
 *                       edge node is constrained when its edge lies on a
 *                       boundary face whose three vertices are all constrained.
 *   flags             : 0 or TG_PATTERN_HOST_ONLY.
 *   out               : receives the new pattern (NULL on error).
 * Errors: TG_E_ARG for bad sizes, ids out of range, repeated vertices in an
 * element, vertices used by no element, or a node shared by more elements
 * than the kernel's block capacity (512 for P1, 64 for P2); TG_E_NOMEM; TG_E_HIP.
 * P1 nodes are the vertices; P2 nodes are the vertices followed by the edges
 * ranked by their (min vertex, max vertex) pair.
 */
tg_status tg_pattern_create(int32_t dim, int32_t order, int32_t ncomp, int64_t n_vertices, int64_t n_elements,
                            const int32_t *conn, const int32_t *dirichlet_vertices, int64_t n_dirichlet,
                            uint32_t flags, tg_pattern **out);

/* Fill *info (host struct). */
tg_status tg_pattern_query(const tg_pattern *p, tg_pattern_info *info);

/* Copy the scalar CSR structure to host arrays: h_row_ptr [n_dofs+1], h_col_idx [nnz]
 * (either may be NULL).  Columns are sorted; both triangles are stored; entries
 * whose value cancels to zero are kept. */
tg_status tg_pattern_copy_csr(const tg_pattern *p, int32_t *h_row_ptr, int32_t *h_col_idx);

/* Copy the constrained DoF ids (ascending) to host h_dofs [n_constrained]. */
tg_status tg_pattern_copy_constrained(const tg_pattern *p, int32_t *h_dofs);

/* Copy the global node ids of every element to host h_nodes [n_elements][k]
 * (P1: the vertices; P2: 4 vertices then the edge nodes of the local edges
 * (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)). */
tg_status tg_pattern_copy_element_nodes(const tg_pattern *p, int32_t *h_nodes);

/*
 * Copy the routing of Sec. 2 Stage II to host arrays (sizes from
 * tg_pattern_query: N = n_nodes, P = n_elements * nodes_per_element pairs,
 * B = n_blocks, Z = nnz / ncomp^2 node-level entries).  Any pointer may be NULL.
 *   h_inc_ptr [N+1], h_inc [P] : S_vec as segments: node i receives the pairs
 *       h_inc[h_inc_ptr[i] .. h_inc_ptr[i+1]) in ascending element order, each
 *       coded e * k + a (element e, local node a).
 *   h_blk_row [B+1] : row block b of the fused kernel covers nodes
 *       [h_blk_row[b], h_blk_row[b+1]).
 *   h_node_rp [N+1] : node-level CSR row pointers (node columns are the scalar
 *       CSR columns of component 0 divided by ncomp).
 *   h_seg_ptr [Z+1], h_slot [n_slot] : S_mat as segments: node-level entry z
 *       sums the local-matrix slots h_slot[h_seg_ptr[z] .. h_seg_ptr[z+1]) in
 *       ascending element order; a slot is b * n + (pair - f), where f is the
 *       first pair and n the number of pairs of the entry's row block: local
 *       entry (a, b) of the pair's element.  For ncomp = 3 each slot is a 3x3
 *       block, and b is the column node in the pair's frame: the element's
 *       vertices reordered as the pair's node's vertex (or its edge's two
 *       vertices, in local order), then the other vertices in local order, with
 *       frame nodes 0..3 these vertices and 4..9 the edges (0,1), (0,2), (0,3),
 *       (1,2), (1,3), (2,3) between them (the pair's node is frame node 0 or 4).
 *       The diagonal entry (i, i) has an empty segment: its value
 *       (P2: 3x3 block) is the sum of K_e[a][a] over the pairs (i, e, a) of
 *       node i, in their S_vec (ascending element) order.  n_slot (tg_pattern_info) is
 *       h_seg_ptr[Z] rounded up to a multiple of 4; the tail is unused.
 */
/*
 * The compact form of the P1 routing that the assembly kernel reads when every
 * node has at most 256 / k pairs and every row block at most 255 rows (*compact
 * receives 1; otherwise 0 and the kernel reads the form above).  It names the
 * same slots in the same order: the slots of node i start at inc_ptr[i] (k-1)
 * in h_slot8 [ceil4(P (k-1))], one byte each, coded (t - inc_ptr[i]) k + b for
 * pair t and local column b; node-level entry z of node i, the r-th row of its
 * block, is h_ent16[z] = r << 8 | (h_seg_ptr[z] - inc_ptr[i] (k-1)) (array
 * [Z]).  Either array may be NULL; nothing is copied when *compact is 0.
 * TG_E_ARG for a P2 pattern.
 */
tg_status tg_pattern_copy_compact_routing(const tg_pattern *p, int32_t *compact, uint16_t *h_ent16,
                                          uint8_t *h_slot8);

/*
 * The coordinate staging of the fused kernels.  Row block b reads the
 * coordinates of its elements' distinct vertices
 * h_blk_vert[h_blk_vptr[b] .. h_blk_vptr[b+1]) (ascending, at most 256) into
 * LDS once; pair t (in S_vec order) finds the vertices of its element at the
 * block-local positions (h_pair_lv[t] >> 8a) & 255, a = 0..dim (for P2 the
 * element's 4 vertex nodes in the pair's frame, see tg_pattern_copy_routing).
 * *n_vert receives the length of h_blk_vert (call
 * with NULL arrays first).  Any array may be NULL; h_blk_vptr [B+1],
 * h_pair_lv [P].
 */
tg_status tg_pattern_copy_block_vertices(const tg_pattern *p, int64_t *n_vert, int32_t *h_blk_vptr,
                                         int32_t *h_blk_vert, uint32_t *h_pair_lv);

tg_status tg_pattern_copy_routing(const tg_pattern *p, int32_t *h_inc_ptr, int32_t *h_inc, int32_t *h_blk_row,
                                  int32_t *h_node_rp, int32_t *h_seg_ptr, uint16_t *h_slot);

/*
 * The sliced-ELL pattern the CG iterations read: slice s holds the 64 scalar
 * rows [64 s, 64 s + 64); entry k of row r sits at h_sell_ptr[s] + 64 k + r % 64
 * (array [ceil(n_dofs / 64) + 1]); every row is padded to its slice's longest
 * row with the column min(r, n_dofs - 1) (value 0).  h_cols [*n_entries]
 * receives every entry's column (decoded); when sell_index_bytes
 * (tg_pattern_info) is 2 the kernels read h_offsets [*n_entries] instead, the
 * 16-bit offset of the column from min(r, n_dofs - 1) (not written otherwise).
 * *n_entries receives h_sell_ptr's last value (call with NULL arrays first).
 * Any pointer may be NULL.
 */
tg_status tg_pattern_copy_sell(const tg_pattern *p, int64_t *n_entries, int32_t *h_sell_ptr, int32_t *h_cols,
                               int16_t *h_offsets);

/* Free the pattern and its device memory.  Work using it must have completed. */
void tg_pattern_destroy(tg_pattern *p);

/*
 * Assemble the CSR values and the right-hand side of `form` on the pattern's
 * mesh: Stage I and Stage II fused in one kernel launch (Sec. 2 Alg. 1 and
 * Alg. 2).  Every entry is written (no accumulation into prior contents).
 *
 *   dtype    : value type of coef, load, values and rhs.  Geometry (J, det J,
 *              J^{-1}) is always computed in FP64.
 *   d_coords : device [n_vertices][dim] FP64 vertex coordinates.
 *   d_coef   : LAPLACE, MASS_LAPLACE: device [n_elements] coefficient per element;
 *              ELASTICITY: device [2][n_elements] (lambda row, then mu row);
 *              MASS: ignored (may be NULL).
 *   d_load   : LAPLACE, MASS_LAPLACE: device [n_elements] source f per element;
 *              ELASTICITY: device [n_elements][3] body force per element;
 *              may be NULL (then d_rhs is not written).  MASS: ignored.
 *   d_values : device [nnz] output values, CSR order of tg_pattern_copy_csr.
 *   d_rhs    : device [n_dofs] output right-hand side, or NULL.
 *   d_status : device int32 or NULL.  If given it must hold TG_STATUS_CLEAN
 *              before the call; after the kernel it holds the smallest index
 *              of an element that is numerically degenerate
 *              (|det J| <= 16 eps |x_1 - x_0| ... |x_d - x_0|) or has a
 *              non-finite value (det J, a coefficient or a load), or is
 *              unchanged.  It is the only
 *              word the library updates atomically.
 * Errors (host): TG_E_ARG (NULL required pointer, form/dtype not valid for the
 * pattern), TG_E_STATE (host-only pattern), TG_E_HIP (launch failure).
 */
tg_status tg_assemble(const tg_pattern *p, tg_form form, tg_dtype dtype, const double *d_coords, const void *d_coef,
                      const void *d_load, void *d_values, void *d_rhs, int32_t *d_status, void *stream);

/*
 * tg_assemble for nbatch coefficient sets on one pattern in one launch
 * (LAPLACE and MASS_LAPLACE; many right-hand sides / coefficient fields on a
 * fixed mesh, cf. the batched data generation of SM B.1.4).  The geometry and
 * the routing are read once; member m reads d_coef + m*E and d_load + m*E
 * (both [nbatch][n_elements]) and writes d_values + m*nnz and d_rhs + m*n_dofs
 * ([nbatch][nnz] and [nbatch][n_dofs]).  Each member is bitwise equal to a
 * single tg_assemble of its coefficients.  nbatch >= 1; other arguments and
 * errors as tg_assemble.
 */
tg_status tg_assemble_batched(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch,
                              const double *d_coords, const void *d_coef, const void *d_load, void *d_values,
                              void *d_rhs, int32_t *d_status, void *stream);

/*
 * Impose Dirichlet conditions on an assembled system by symmetric
 * elimination on the fixed pattern.  For a constrained DoF b with value g_b:
 * row b becomes e_b^T with rhs_b = g_b; for every other row i,
 * rhs_i -= K_ib g_b and K_ib = 0.  With x_0 = 0 the solution of the result
 * equals the condensed system of Sec. B.1.2 on the free DoFs and g on the
 * constrained ones.
 *   d_values, d_rhs : device, as written by tg_assemble (modified in place).
 *   d_g             : device [n_dofs] of dtype (only constrained entries are
 *                     read), or NULL for g = 0.
 * d_values may be NULL when d_g is NULL: then only rhs_b = 0 is written on the
 * constrained DoFs (the form an implicit step's right-hand side needs).
 */
tg_status tg_apply_dirichlet(const tg_pattern *p, tg_dtype dtype, void *d_values, void *d_rhs, const void *d_g,
                             void *stream);

/*
 * y = K x on the pattern's CSR (device arrays of dtype; rows accumulated in FP64).
 */
tg_status tg_spmv(const tg_pattern *p, tg_dtype dtype, const void *d_values, const void *d_x, void *d_y,
                  void *stream);

/*
 * Solve K x = b with Jacobi-preconditioned conjugate gradients, x_0 = 0, and
 * stop when ||r_k||_2 / ||b||_2 <= rtol for the recursive residual r_k (the
 * criterion of Sec. B.1.2; CG replaces the paper's BiCGSTAB because every
 * configured system is symmetric positive definite).  CG runs in the
 * single-reduction form of Chronopoulos and Gear (one kernel launch per
 * iteration).  Dot products and norms are accumulated in FP64 in a fixed order
 * (bitwise reproducible).
 *   d_values, d_rhs : device arrays of dtype (e.g. after tg_apply_dirichlet).
 *   d_x             : device [n_dofs] of dtype, output.
 *   check_every     : iterations per chunk between host checks of the stop test
 *                     (>= 1); the host reads one chunk's state while the next
 *                     chunk runs, launches after convergence do nothing, and
 *                     the iteration count reported is exact regardless.
 *   iters, relres   : host outputs: iterations done (all runs), and the final
 *                     TRUE relative residual ||b - K x|| / ||b|| (eq. linres).
 * TG_OK means the true residual met rtol.  When the recursive residual meets
 * rtol but the true one does not (rounding in the recurrences, mostly FP32),
 * CG restarts from the current x (residual replacement: r = b - K x formed
 * with FP64 sums), at most 4 times and only while each restart at least halves
 * the true residual; if it stays above rtol the call returns TG_E_ACCURACY
 * (rtol is below what the dtype can reach: in FP32 the rounding of x alone
 * leaves about 1e-7 to 1e-5 on Poisson and heat systems), with the best
 * iterate in d_x.  The values are copied once per call into a sliced-ELL
 * layout (64-row slices) that the iterations read.
 * Blocks until done (host syncs on `stream`).  Uses the pattern's own
 * workspace: calls on one pattern must not overlap.  Returns TG_E_NOCONV
 * (with the last iterate in d_x) if max_iter is reached, TG_E_NONFINITE if a
 * step length, inner product or the residual is not finite.
 */
tg_status tg_pcg(const tg_pattern *p, tg_dtype dtype, const void *d_values, const void *d_rhs, void *d_x, double rtol,
                 int32_t max_iter, int32_t check_every, int32_t *iters, double *relres, void *stream);

/*
 * Adjoint of P1 assembly (Sec. 2, eq. adj): the gradient of an assembled
 * system's bilinear quantity with respect to the element coefficients and the
 * vertex coordinates, for given adjoint and state vectors.  For members
 * m = 0 .. nbatch-1 it differentiates
 *     Phi = scale * sum_m lam_m^T (A u_m - M w_m),
 * with A = K(c) (TG_LAPLACE), M (TG_MASS) or M + K(c) (TG_MASS_LAPLACE) as
 * tg_assemble defines them and M the P1 mass matrix (the mass inner product of
 * SM A.1).  A gradient dL/du = A^T lam through a solve A u = b(w) gives
 * dL/dtheta = -dPhi/dtheta with scale = 1 (the relation dL/dK = -lam u^T of
 * eq. adj restricted to the pattern), so scale = -1 returns dL/dtheta.
 *   form           : TG_LAPLACE, TG_MASS or TG_MASS_LAPLACE on a P1 scalar pattern.
 *   d_coords       : device FP64 [n_vertices][dim], AoS.
 *   d_coef         : device [n_elements] of dtype, c_e (ignored for TG_MASS).
 *   d_lam, d_u     : device [nbatch][stride] of dtype; member m at offset m*stride.
 *   d_w            : as d_u, or NULL for w = 0.
 *   stride         : >= n_dofs (elements of dtype between members).
 *   d_dlogc        : device FP64 [n_elements] out, dPhi/d(log c_e) = scale *
 *                    sum_m lam_e^T K_e u_e (0 for TG_MASS), or NULL.
 *   d_dcoords      : device FP64 [n_vertices][dim] out, dPhi/dx, or NULL.
 *   d_status       : as in tg_assemble (numerically singular elements, non-finite c).
 * Arithmetic is FP64 for either dtype.  The vertex gradients are reduced over
 * each vertex's incident elements in ascending element order (no atomics), so
 * repeated calls give bitwise identical results.  Uses the pattern's scratch
 * (E*(dim+1)*dim doubles, allocated on first use): calls on one pattern must
 * not overlap.  Errors: TG_E_ARG (NULL inputs, no output, nbatch < 1,
 * stride < n_dofs, not P1 scalar, beyond 4 GiB), TG_E_NOMEM, TG_E_HIP.
 */
tg_status tg_adjoint_p1(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch, const double *d_coords,
                        const void *d_coef, const void *d_lam, const void *d_u, const void *d_w, int64_t stride,
                        double scale, double *d_dlogc, double *d_dcoords, int32_t *d_status, void *stream);

/*
 * tg_adjoint_p1 for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results (bitwise), but the kernels'
 * staging array [n_elements][dim+1][dim] of doubles lives in a fixed array of
 * the library (2^22 doubles = 32 MiB on each GPU the library runs on, held
 * until the process ends) instead of the pattern's scratch that tg_adjoint_p1
 * grows with hipMalloc; this call allocates nothing and frees nothing.
 * Limit: n_elements (dim+1) dim <= 4,194,304 (699,050 triangles or 349,525
 * tetrahedra); beyond it TG_E_ARG.  Every call on one GPU shares the array and
 * it keeps the last call's contents (each call overwrites the entries it
 * reads): calls that overlap on one GPU (different streams or threads) race
 * and give wrong results, so serialise them.  The current device must be the
 * pattern's (else TG_E_STATE).  Other errors as tg_adjoint_p1.
 */
tg_status tg_adjoint_p1_noalloc(const tg_pattern *p, tg_form form, tg_dtype dtype, int32_t nbatch,
                                const double *d_coords, const void *d_coef, const void *d_lam, const void *d_u,
                                const void *d_w, int64_t stride, double scale, double *d_dlogc, double *d_dcoords,
                                int32_t *d_status, void *stream);

/*
 * Implicit-Euler rollout of the method-of-lines system M U' + K(a) U = 0
 * (SM A.1, with no semilinear term and no source) on a P1 scalar pattern, U = 0
 * on the pattern's constrained DoFs:
 *     (M + dt K(a)) u^{k+1} = M u^k on the free DoFs,  k = 0 .. nsteps-1,
 * with a_e = exp(log_a_e).  Per step: one SpMV with M, then Jacobi-PCG on
 * A = M + dt K(a) (both assembled once per call by the Map-Reduce kernels),
 * started from u^k (its constrained entries set to 0); the stop test is
 * ||r|| <= rtol ||M u^k|| as in tg_pcg's recursive test (these solves do not
 * restart on the true residual: in FP32 its floor, about 1e-5 at 256^2, is
 * above the tolerances the gradients need, while the recursive test still
 * resolves the smooth error components).
 *   d_coords  : device FP64 [n_vertices][dim].   d_log_a : device FP64 [n_elements].
 *   d_u0      : device [n_dofs] of dtype (entries on constrained DoFs enter M u^0).
 *   d_states  : device [nsteps+1][n_dofs] of dtype, out: row k = u^k (row 0 = u^0).
 *   rtol, max_iter, check_every : per-step PCG controls as in tg_pcg.
 *   iters     : host out (may be NULL), PCG iterations summed over the steps.
 *   relres    : host out (may be NULL), the largest true relative residual.
 *   d_status  : as in tg_assemble.
 * Blocks until done.  Uses the pattern's scratch and PCG workspace: calls on
 * one pattern must not overlap.  Errors: as tg_pcg (TG_E_NOCONV stops the
 * rollout at that step), TG_E_ARG for dt <= 0 or nsteps < 0.
 */
tg_status tg_heat_rollout(const tg_pattern *p, tg_dtype dtype, const double *d_coords, const double *d_log_a,
                          double dt, int32_t nsteps, const void *d_u0, void *d_states, double rtol, int32_t max_iter,
                          int32_t check_every, int64_t *iters, double *relres, int32_t *d_status, void *stream);

/*
 * Discrete adjoint (Sec. 2, eq. adj) of tg_heat_rollout for a loss L with
 * d_g = dL/du^N (N = nsteps).  With A = M + dt K(a):
 *     A lam^N = g,   A lam^k = M lam^{k+1}  (k = N-1 .. 1)   on the free DoFs,
 *     dL/dtheta = -sum_k d/dtheta [lam^k^T (A u^k - M u^{k-1})],
 * evaluated by tg_adjoint_p1 over the N (lam^k, u^k, u^{k-1}) triples in one
 * launch, and dL/du^0 = M lam^1.  The solve for lam^k starts from lam^{k+1}
 * (lam^N from 0).
 *   d_states    : the rollout's [nsteps+1][n_dofs] of dtype (read only).
 *   d_g         : device [n_dofs] of dtype.
 *   d_dlog_a    : device FP64 [n_elements] out, dL/d(log a_e), or NULL.
 *   d_dcoords   : device FP64 [n_vertices][dim] out, dL/dx, or NULL.
 *   d_du0       : device [n_dofs] of dtype out, dL/du^0, or NULL.
 * Other arguments, blocking and errors as tg_heat_rollout.
 */
tg_status tg_heat_adjoint(const tg_pattern *p, tg_dtype dtype, const double *d_coords, const double *d_log_a,
                          double dt, int32_t nsteps, const void *d_states, const void *d_g, double *d_dlog_a,
                          double *d_dcoords, void *d_du0, double rtol, int32_t max_iter, int32_t check_every,
                          int64_t *iters, double *relres, int32_t *d_status, void *stream);

/*
 * Request server: continuous batching of assemble + solve requests with
 * iteration-level scheduling (the batched generation of many PDE instances of
 * SM B.1.4, served the way LLM servers batch generation steps).
 *
 * A request = assemble (tg_assemble's forms except TG_MASS), eliminate
 * Dirichlet data (tg_apply_dirichlet, with d_g or g = 0), and solve with
 * Jacobi-PCG (tg_pcg).  Requests are grouped by (pattern, dtype); a group keeps
 * up to max_slots systems in one batched CG (one launch per iteration for the
 * whole group; each group on its own stream, forked from and joined back to
 * `stream` in every tg_server_step).  Each tg_server_step admits queued requests into free
 * slots (a slot is allocated when the server's HBM budget allows), runs
 * check_every CG iterations, then retires the converged systems (or those at
 * max_iter).  Queued requests are admitted oldest first across groups.  A
 * request's solution and iteration count are bitwise the same as a solo
 * tg_assemble + tg_apply_dirichlet + tg_pcg of it: every slot's reductions are
 * its own, in the same fixed order, and a slot takes tg_pcg's decisions
 * (including its restarts from x when the true residual is above rtol).
 *
 * Memory: group tables, slots and the patterns the server builds
 * (tg_server_submit_mesh) count against hbm_budget_bytes.  A request that
 * needs memory the budget lacks first frees what no request uses, least
 * recently used first (idle slots of other groups, groups without slots,
 * cached patterns no request needs), else waits for running requests to
 * finish; it fails with TG_E_NOMEM only if one slot of it (with the group's
 * tables and its cached pattern) exceeds the whole budget.
 *
 * Ownership: the server owns the slot buffers and the patterns it builds
 * (freed by tg_server_destroy or when evicted).  The caller owns every pointer
 * of a request (coords, coef, load, g, x, and a mesh request's conn), which
 * must stay valid until the request's result has been polled, and a pattern
 * passed to tg_server_submit, which must outlive the server.  All work runs on
 * `stream` (NULL: the default stream); the server is not thread-safe.
 */
typedef struct tg_server tg_server; /* opaque */

typedef struct {
    int64_t request_id;
    int32_t status;      /* TG_OK, TG_E_NOCONV, TG_E_DEGENERATE (bad element), TG_E_NONFINITE (non-finite
                            CG scalars or residual), TG_E_NOMEM (one slot exceeds the budget), or a
                            submit_mesh topology's tg_pattern_create status */
    int32_t iters;       /* CG iterations, as tg_pcg reports them */
    double relres;       /* true relative residual ||b - K x|| / ||b|| */
    int32_t bad_element; /* first numerically singular element, or -1 */
    int32_t pad;
    double t_submit;     /* host seconds since tg_server_create */
    double t_done;
} tg_server_result;

typedef struct {
    int64_t n_queued, n_active, n_slots, n_groups, n_results;
    size_t hbm_used, hbm_budget;          /* bytes counted against the budget, and the budget */
    int64_t n_patterns;                   /* patterns the server holds for tg_server_submit_mesh */
    int64_t n_pattern_builds;             /* pattern builds so far (cache misses) */
    int64_t n_pattern_evictions;          /* cached patterns freed to make room */
    double pattern_build_s;               /* host seconds spent building them */
} tg_server_info;

/* hbm_budget_bytes: cap on slot memory (tg_server_slot_bytes per slot);
 * max_slots: slots per group (1..65535); check_every: CG iterations per
 * tg_server_step (>= 1). */
tg_status tg_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t check_every, void *stream,
                           tg_server **out);

/* Queue one request (arguments as tg_assemble / tg_apply_dirichlet / tg_pcg;
 * d_load is required, d_g may be NULL; d_x device [n_dofs] of dtype receives
 * the solution).  Nothing runs until tg_server_step. */
tg_status tg_server_submit(tg_server *srv, const tg_pattern *p, tg_form form, tg_dtype dtype, const double *d_coords,
                           const void *d_coef, const void *d_load, const void *d_g, void *d_x, double rtol,
                           int32_t max_iter, int64_t *request_id);

/* Queue one request on a mesh given by its connectivity: the server keeps the
 * CSR pattern of every topology it serves, keyed by (topology_key, dim,
 * order, n_vertices, n_elements) -- topology_key is the caller's name for the
 * connectivity, equal keys must mean equal connectivity -- and builds one on a
 * miss (host build plus device upload, during a later tg_server_step, with
 * homogeneous Dirichlet data on the whole boundary, as tg_pattern_create with
 * TG_BOUNDARY_ALL).  Cached patterns count against the HBM budget and the least
 * recently used one that no request needs is freed when memory is short.
 * form: TG_LAPLACE or TG_MASS_LAPLACE (P1, scalar, dim 2 or 3) or
 * TG_ELASTICITY (P2, dim 3); conn is host [n_elements][dim+1] and, like the
 * device arrays, must stay valid until the request's result has been polled.
 * A topology that tg_pattern_create rejects fails its requests with that
 * status; a request that one slot cannot hold within the budget fails with
 * TG_E_NOMEM. */
tg_status tg_server_submit_mesh(tg_server *srv, int32_t dim, int64_t n_vertices, int64_t n_elements,
                                const int32_t *conn, uint64_t topology_key, tg_form form, tg_dtype dtype,
                                const double *d_coords, const void *d_coef, const void *d_load, void *d_x,
                                double rtol, int32_t max_iter, int64_t *request_id);

/* One scheduling round (blocks until its iterations are done).  Optional outputs: systems in flight, queued. */
tg_status tg_server_step(tg_server *srv, int32_t *n_active, int32_t *n_queued);

/* Pop up to max_results finished requests, oldest first. */
tg_status tg_server_poll(tg_server *srv, int32_t max_results, tg_server_result *out, int32_t *n_out);

tg_status tg_server_query(const tg_server *srv, tg_server_info *info);

/* Device bytes of one server slot for systems on pattern p in dtype (values in
 * CSR and sliced-ELL layouts, right-hand side, Krylov vectors and partial sums),
 * the unit in which a server's HBM budget is spent.  Host-only; TG_E_ARG for a
 * NULL pattern or output, TG_E_STATE for a host-only pattern. */
tg_status tg_server_slot_bytes(const tg_pattern *p, tg_dtype dtype, size_t *bytes);

/* Synchronises the server's stream and frees its slots (NULL is a no-op). */
void tg_server_destroy(tg_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* TG_H */
