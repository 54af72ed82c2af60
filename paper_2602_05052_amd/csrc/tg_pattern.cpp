// Host construction of the CSR pattern and the routing tables of one mesh
// topology (TensorGalerkin Sec. 2, Stage II: routing matrices precomputed from
// the topology alone).
//
// The paper stores the routing as 0/1 matrices S_vec (N x E k) and
// S_mat (N_nnz x E k^2).  Every column of either has exactly one 1, so the
// products S_vec vec(F_local) and S_mat vec(K_local) are segmented sums.  This
// builder stores them in that form:
//   S_vec: for each node i, its (element, local node) pairs in ascending
//          element order  (inc_ptr / inc);
//   S_mat: for each off-diagonal node-level CSR entry (i, j), the element
//          slots (pair of row i, local column b) that land on it, in ascending
//          element order (seg_ptr / slot).  Slot ids are relative to the row
//          block of the fused kernel and index its local matrices in LDS,
//          stored column by column: slot = b * (pairs of the block) + (pair -
//          first pair).  A diagonal entry (i, i) sums exactly the blocks (a, a)
//          of row i's pairs in S_vec order, so it has no slots; the kernels sum
//          it per row.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "tg_internal.h"

namespace tg {
namespace {

constexpr int kP2Edge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// The local frame of a P2 pair (node i, element e, local node a): the element's
// vertices reordered so that i is vertex 0 (a vertex node) or edge (0, 1) (an
// edge node): its vertex, or its edge's two vertices in local order, then the
// element's other vertices in local order.  ord[k] = local vertex at frame
// position k.
void p2_frame_order(int a, int ord[4]) {
    bool used[4] = {false, false, false, false};
    int n = 0;
    auto put = [&](int v) {
        ord[n++] = v;
        used[v] = true;
    };
    if (a < 4) {
        put(a);
    } else {
        put(kP2Edge[a - 4][0]);
        put(kP2Edge[a - 4][1]);
    }
    for (int v = 0; v < 4; ++v)
        if (!used[v]) put(v);
}

// frame[a][b]: index in the frame of pair node a of the element's local node b
// (vertices 0..3, then edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) of the frame).
struct P2FrameTable {
    uint8_t frame[10][10];
    P2FrameTable() {
        for (int a = 0; a < 10; ++a) {
            int ord[4], pos[4];
            p2_frame_order(a, ord);
            for (int k = 0; k < 4; ++k) pos[ord[k]] = k;
            for (int b = 0; b < 10; ++b) {
                if (b < 4) {
                    frame[a][b] = (uint8_t)pos[b];
                    continue;
                }
                int p = pos[kP2Edge[b - 4][0]], q = pos[kP2Edge[b - 4][1]];
                if (p > q) std::swap(p, q);
                for (int m = 0; m < 6; ++m)
                    if (kP2Edge[m][0] == p && kP2Edge[m][1] == q) frame[a][b] = (uint8_t)(4 + m);
            }
        }
    }
};
const P2FrameTable kP2Frame;

struct FaceKey {
    int32_t v[3];
    bool operator<(const FaceKey &o) const {
        return std::lexicographical_compare(v, v + 3, o.v, o.v + 3);
    }
    bool operator==(const FaceKey &o) const { return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2]; }
};

// Faces (dim vertices, sorted) that belong to exactly one element.
std::vector<FaceKey> boundary_faces(int dim, int64_t E, const int32_t *conn) {
    const int nvtx = dim + 1;
    std::vector<FaceKey> faces;
    faces.reserve((size_t)E * nvtx);
    for (int64_t e = 0; e < E; ++e)
        for (int skip = 0; skip < nvtx; ++skip) {
            FaceKey f{{-1, -1, -1}};
            int m = 0;
            for (int a = 0; a < nvtx; ++a)
                if (a != skip) f.v[m++] = conn[e * nvtx + a];
            std::sort(f.v, f.v + dim);
            faces.push_back(f);
        }
    std::sort(faces.begin(), faces.end());
    std::vector<FaceKey> out;
    for (size_t t = 0; t < faces.size();) {
        size_t u = t + 1;
        while (u < faces.size() && faces[u] == faces[t]) ++u;
        if (u - t == 1) out.push_back(faces[t]);
        t = u;
    }
    return out;
}

}  // namespace

tg_status build_host_pattern(int dim, int order, int ncomp, int64_t nv, int64_t E, const int32_t *conn,
                             const int32_t *dirichlet, int64_t n_dirichlet, HostPattern &hp, std::string &msg) {
    const bool p1 = (order == 1 && ncomp == 1 && (dim == 2 || dim == 3));
    const bool p2 = (order == 2 && ncomp == 3 && dim == 3);
    if (!p1 && !p2) {
        msg = "unsupported (dim, order, ncomp); supported: (2|3, 1, 1) and (3, 2, 3)";
        return TG_E_ARG;
    }
    if (nv <= 0 || E <= 0 || !conn) {
        msg = "n_vertices and n_elements must be positive and conn non-NULL";
        return TG_E_ARG;
    }
    const int nvtx = dim + 1;
    const int k = p1 ? nvtx : 10;
    if (nv >= INT32_MAX || E * (int64_t)k >= INT32_MAX) {
        msg = "mesh too large for int32 indexing";
        return TG_E_ARG;
    }
    hp.dim = dim;
    hp.order = order;
    hp.ncomp = ncomp;
    hp.k = k;
    hp.nv = nv;
    hp.E = E;
    hp.conn.assign(conn, conn + E * nvtx);

    // ---- validate connectivity
    std::vector<uint8_t> used(nv, 0);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *g = conn + e * nvtx;
        for (int a = 0; a < nvtx; ++a) {
            if (g[a] < 0 || g[a] >= nv) {
                msg = "element " + std::to_string(e) + " has vertex id out of range";
                return TG_E_ARG;
            }
            for (int b = 0; b < a; ++b)
                if (g[a] == g[b]) {
                    msg = "element " + std::to_string(e) + " repeats a vertex";
                    return TG_E_ARG;
                }
            used[g[a]] = 1;
        }
    }
    for (int64_t v = 0; v < nv; ++v)
        if (!used[v]) {
            msg = "vertex " + std::to_string(v) + " is used by no element";
            return TG_E_ARG;
        }

    // ---- nodes: P1 = vertices; P2 = vertices, then edges by (min, max)
    std::vector<uint64_t> edges;
    hp.elem_nodes.resize((size_t)E * k);
    if (p1) {
        hp.n_nodes = nv;
        std::memcpy(hp.elem_nodes.data(), conn, sizeof(int32_t) * E * k);
    } else {
        edges.reserve((size_t)E * 6);
        for (int64_t e = 0; e < E; ++e)
            for (int m = 0; m < 6; ++m) {
                uint64_t p = (uint32_t)conn[e * 4 + kP2Edge[m][0]], q = (uint32_t)conn[e * 4 + kP2Edge[m][1]];
                edges.push_back(std::min(p, q) << 32 | std::max(p, q));
            }
        std::sort(edges.begin(), edges.end());
        edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
        hp.n_nodes = nv + (int64_t)edges.size();
        if (hp.n_nodes * 3 >= INT32_MAX) {
            msg = "mesh too large for int32 indexing";
            return TG_E_ARG;
        }
        for (int64_t e = 0; e < E; ++e) {
            for (int a = 0; a < 4; ++a) hp.elem_nodes[e * 10 + a] = conn[e * 4 + a];
            for (int m = 0; m < 6; ++m) {
                uint64_t p = (uint32_t)conn[e * 4 + kP2Edge[m][0]], q = (uint32_t)conn[e * 4 + kP2Edge[m][1]];
                uint64_t key = std::min(p, q) << 32 | std::max(p, q);
                int64_t r = std::lower_bound(edges.begin(), edges.end(), key) - edges.begin();
                hp.elem_nodes[e * 10 + 4 + m] = (int32_t)(nv + r);
            }
        }
    }
    const int64_t N = hp.n_nodes;
    hp.n_dofs = N * ncomp;

    // ---- S_vec routing: pairs grouped by node, ascending element inside a node
    hp.inc_ptr.assign(N + 1, 0);
    for (int64_t t = 0; t < E * k; ++t) hp.inc_ptr[hp.elem_nodes[t] + 1]++;
    const int cap = p1 ? kP1BlockCap : kP2BlockCap;
    for (int64_t i = 0; i < N; ++i) {
        if (hp.inc_ptr[i + 1] > cap) {
            msg = "node " + std::to_string(i) + " belongs to " + std::to_string(hp.inc_ptr[i + 1]) +
                  " elements, more than the kernel block capacity " + std::to_string(cap);
            return TG_E_ARG;
        }
        hp.inc_ptr[i + 1] += hp.inc_ptr[i];
    }
    hp.inc.resize((size_t)E * k);
    {
        std::vector<int32_t> fill(hp.inc_ptr.begin(), hp.inc_ptr.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < k; ++a) hp.inc[fill[hp.elem_nodes[e * k + a]]++] = (int32_t)(e * k + a);
    }

    // ---- node-level CSR: row i holds every node sharing an element with i (sorted)
    hp.node_rp.assign(N + 1, 0);
    hp.node_ci.clear();
    hp.node_ci.reserve((size_t)E * k * 2);
    std::vector<int32_t> mark(N, -1), pos(N, 0), cols, cnt;
    for (int64_t i = 0; i < N; ++i) {
        cols.clear();
        for (int32_t t = hp.inc_ptr[i]; t < hp.inc_ptr[i + 1]; ++t) {
            const int64_t e = hp.inc[t] / k;
            for (int b = 0; b < k; ++b) {
                int32_t j = hp.elem_nodes[e * k + b];
                if (mark[j] != (int32_t)i) {
                    mark[j] = (int32_t)i;
                    cols.push_back(j);
                }
            }
        }
        std::sort(cols.begin(), cols.end());
        hp.node_ci.insert(hp.node_ci.end(), cols.begin(), cols.end());
        hp.node_rp[i + 1] = (int32_t)hp.node_ci.size();
        if ((int64_t)hp.node_ci.size() * ncomp * ncomp >= INT32_MAX) {
            msg = "too many nonzeros for int32 indexing";
            return TG_E_ARG;
        }
    }

    // ---- P2: vertex-node columns per row, as a prefix (the Reduce handles a
    // block's vertex-column and edge-column entries in separate passes)
    hp.node_vp.clear();
    if (p2) {
        hp.node_vp.assign(N + 1, 0);
        for (int64_t i = 0; i < N; ++i) {
            int32_t c = 0;
            for (int32_t z = hp.node_rp[i]; z < hp.node_rp[i + 1] && hp.node_ci[z] < hp.nv; ++z) ++c;
            hp.node_vp[i + 1] = hp.node_vp[i] + c;
        }
    }

    // ---- row blocks: consecutive rows while the pairs fit the target (and, for
    // P1, the node-level entries fit one thread each); a single row may exceed
    // the target up to the capacity
    // the target up to the capacity.  P1 blocks also keep their elements'
    // distinct vertices within kP1BlockVerts (8-bit local ids).
    const int target = p1 ? kP1BlockTarget : kP2BlockTarget;
    const int entry_target = p1 ? kP1Threads - 1 : INT32_MAX;
    hp.blk_row.clear();
    hp.blk_row.push_back(0);
    std::vector<int64_t> vstamp(p1 ? hp.nv : 0, -1);
    // distinct vertices that row r adds to the block stamped `stamp` (marks them)
    auto row_new_verts = [&](int64_t r, int64_t stamp, std::vector<int32_t> *added) {
        int n = 0;
        for (int32_t t = hp.inc_ptr[r]; t < hp.inc_ptr[r + 1]; ++t) {
            const int64_t e = hp.inc[t] / k;
            for (int b = 0; b < k; ++b) {
                const int32_t v = hp.elem_nodes[e * k + b];
                if (vstamp[v] != stamp) {
                    vstamp[v] = stamp;
                    ++n;
                    if (added) added->push_back(v);
                }
            }
        }
        return n;
    };
    std::vector<int32_t> added;
    for (int64_t i = 0; i < N;) {
        const int32_t first = hp.inc_ptr[i], first_entry = hp.node_rp[i];
        int64_t j = i + 1;
        if (p1) {
            int nverts = row_new_verts(i, i, nullptr);
            if (nverts > kP1BlockVerts) {
                msg = "the elements of node " + std::to_string(i) + " have " + std::to_string(nverts) +
                      " distinct vertices, more than the kernel block capacity " + std::to_string(kP1BlockVerts);
                return TG_E_ARG;
            }
            while (j < N && hp.inc_ptr[j + 1] - first <= target && hp.node_rp[j + 1] - first_entry <= entry_target) {
                added.clear();
                const int extra = row_new_verts(j, i, &added);
                if (nverts + extra > kP1BlockVerts) {
                    for (int32_t v : added) vstamp[v] = -1;  // row j starts the next block
                    break;
                }
                nverts += extra;
                ++j;
            }
        } else {  // P2 blocks also hold at most kP2BlockCap rows (nodes of no element add rows, not pairs)
            while (j < N && j - i < kP2BlockCap && hp.inc_ptr[j + 1] - first <= target &&
                   hp.node_rp[j + 1] - first_entry <= entry_target)
                ++j;
        }
        hp.blk_row.push_back((int32_t)j);
        i = j;
    }

    // ---- S_mat routing, row by row
    hp.seg_ptr.clear();
    hp.seg_ptr.reserve((size_t)hp.node_ci.size() + 1);
    // Diagonal entries take no slots: the kernels sum the pairs' own diagonal
    // entries (P1) or 3x3 diagonal blocks (P2) row by row, the same terms in
    // the same order.
    const bool skip_diag = true;
    hp.slot.resize((size_t)E * k * (skip_diag ? k - 1 : k) + 3);
    int64_t slot_fill = 0;
    int64_t blk = 0;
    for (int64_t i = 0; i < N; ++i) {
        while (hp.blk_row[blk + 1] <= i) ++blk;
        const int32_t blk_first_pair = hp.inc_ptr[hp.blk_row[blk]];
        const int32_t blk_pairs = hp.inc_ptr[hp.blk_row[blk + 1]] - blk_first_pair;
        const int32_t c0 = hp.node_rp[i], m = hp.node_rp[i + 1] - c0;
        for (int32_t c = 0; c < m; ++c) pos[hp.node_ci[c0 + c]] = c;
        // counts per entry, then slots in (pair ascending, b) order -> ascending element per entry
        cnt.assign(m + 1, 0);
        const int diag = skip_diag ? pos[i] : -1;
        for (int32_t t = hp.inc_ptr[i]; t < hp.inc_ptr[i + 1]; ++t) {
            const int64_t e = hp.inc[t] / k;
            for (int b = 0; b < k; ++b) {
                const int c = pos[hp.elem_nodes[e * k + b]];
                if (c != diag) cnt[c + 1]++;
            }
        }
        for (int32_t c = 0; c < m; ++c) cnt[c + 1] += cnt[c];
        for (int32_t c = 0; c < m; ++c) hp.seg_ptr.push_back((int32_t)(slot_fill + cnt[c]));
        for (int32_t t = hp.inc_ptr[i]; t < hp.inc_ptr[i + 1]; ++t) {
            const int64_t e = hp.inc[t] / k;
            const int a = hp.inc[t] % k;
            for (int b = 0; b < k; ++b) {
                const int c = pos[hp.elem_nodes[e * k + b]];
                const int bf = p2 ? kP2Frame.frame[a][b] : b;  // P2: the column in the pair's frame
                if (c != diag) hp.slot[slot_fill + cnt[c]++] = (uint16_t)(bf * blk_pairs + (t - blk_first_pair));
            }
        }
        slot_fill += cnt[m];
    }
    hp.seg_ptr.push_back((int32_t)slot_fill);
    // the kernels copy whole 4-slot units: pad to a multiple of 4 (never referenced)
    hp.slot.resize(((size_t)slot_fill + 3) & ~(size_t)3, 0);
    hp.nnz_nodes = (int64_t)hp.node_ci.size();
    hp.max_block_pairs = hp.max_block_entries = hp.max_block_rows = 0;
    hp.blk_desc.assign((hp.blk_row.size() - 1) * kBlkDesc, 0);
    for (int64_t b = 0; b + 1 < (int64_t)hp.blk_row.size(); ++b) {
        const int32_t r0 = hp.blk_row[b], r1 = hp.blk_row[b + 1];
        int32_t *dsc = &hp.blk_desc[b * kBlkDesc];
        dsc[0] = r0;
        dsc[1] = r1;
        dsc[2] = hp.inc_ptr[r0];
        dsc[3] = hp.inc_ptr[r1];
        dsc[4] = hp.node_rp[r0];
        dsc[5] = hp.node_rp[r1];
        dsc[8] = hp.seg_ptr[hp.node_rp[r0]];
        dsc[9] = hp.seg_ptr[hp.node_rp[r1]];
        if (p2) {
            dsc[10] = hp.node_vp[r0];
            dsc[11] = hp.node_vp[r1];
        }
        hp.max_block_pairs = std::max(hp.max_block_pairs, hp.inc_ptr[r1] - hp.inc_ptr[r0]);
        hp.max_block_entries = std::max(hp.max_block_entries, hp.node_rp[r1] - hp.node_rp[r0]);
        hp.max_block_rows = std::max(hp.max_block_rows, r1 - r0);
    }
    // ---- compact P1 routing (same slots and order, one byte per slot, two per entry)
    hp.compact = false;
    hp.ent16.clear();
    hp.slot8.clear();
    if (p1) {
        int32_t max_row_pairs = 0;
        for (int64_t i = 0; i < N; ++i) max_row_pairs = std::max(max_row_pairs, hp.inc_ptr[i + 1] - hp.inc_ptr[i]);
        hp.compact = max_row_pairs <= compact_row_pairs(k) && hp.max_block_rows <= 255;
    }
    if (hp.compact) {
        hp.ent16.resize((size_t)hp.nnz_nodes);
        hp.slot8.assign(((size_t)hp.n_pairs() * (k - 1) + 3) & ~(size_t)3, 0);
        for (int64_t b = 0; b + 1 < (int64_t)hp.blk_row.size(); ++b) {
            const int32_t r0 = hp.blk_row[b], r1 = hp.blk_row[b + 1];
            const int32_t bf = hp.inc_ptr[r0], bp = hp.inc_ptr[r1] - bf;  // first pair, pairs of the block
            for (int32_t i = r0; i < r1; ++i) {
                const int32_t rs = hp.inc_ptr[i] * (k - 1);  // the row's first slot (wide and compact alike)
                for (int32_t z = hp.node_rp[i]; z < hp.node_rp[i + 1]; ++z) {
                    hp.ent16[z] = (uint16_t)(((i - r0) << 8) | (hp.seg_ptr[z] - rs));
                    for (int32_t g = hp.seg_ptr[z]; g < hp.seg_ptr[z + 1]; ++g) {
                        const int32_t t = bf + hp.slot[g] % bp, bb = hp.slot[g] / bp;
                        hp.slot8[g] = (uint8_t)((t - hp.inc_ptr[i]) * k + bb);
                    }
                }
            }
        }
    }
    // ---- block vertex lists and the per-pair block-local ids of the element's
    // vertices (its first dim + 1 nodes; P2 blocks hold at most 64 pairs, so
    // at most 256 vertices)
    hp.blk_vert.clear();
    hp.pair_lv.clear();
    hp.max_block_verts = 0;
    {
        const int kv = dim + 1;
        hp.pair_lv.assign((size_t)E * k, 0u);
        std::vector<int32_t> local(hp.nv, -1), verts;
        for (int64_t b = 0; b + 1 < (int64_t)hp.blk_row.size(); ++b) {
            int32_t *dsc = &hp.blk_desc[b * kBlkDesc];
            const int32_t q0 = dsc[2], q1 = dsc[3];
            verts.clear();
            for (int32_t t = q0; t < q1; ++t) {
                const int64_t e = hp.inc[t] / k;
                for (int a = 0; a < kv; ++a) verts.push_back(hp.elem_nodes[e * k + a]);
            }
            std::sort(verts.begin(), verts.end());
            verts.erase(std::unique(verts.begin(), verts.end()), verts.end());
            if ((int)verts.size() > kP1BlockVerts) {  // the block partition above prevents this
                msg = "internal error: block vertex capacity exceeded";
                return TG_E_ARG;
            }
            dsc[6] = (int32_t)hp.blk_vert.size();
            for (size_t l = 0; l < verts.size(); ++l) {
                local[verts[l]] = (int32_t)l;
                hp.blk_vert.push_back(verts[l]);
            }
            dsc[7] = (int32_t)hp.blk_vert.size();
            hp.max_block_verts = std::max(hp.max_block_verts, (int32_t)verts.size());
            for (int32_t t = q0; t < q1; ++t) {
                const int64_t e = hp.inc[t] / k;
                int ord[4] = {0, 1, 2, 3};  // P1: local order; P2: the pair's frame
                if (p2) p2_frame_order(hp.inc[t] % k, ord);
                uint32_t w = 0;
                for (int a = 0; a < kv; ++a) w |= (uint32_t)local[hp.elem_nodes[e * k + ord[a]]] << (8 * a);
                hp.pair_lv[t] = w;
            }
            for (int32_t v : verts) local[v] = -1;
        }
    }
    hp.nnz = hp.nnz_nodes * ncomp * ncomp;

    // ---- scalar CSR (DoF = ncomp * node + c; the 3 rows of a node share its node columns)
    if (ncomp == 1) {
        hp.row_ptr = hp.node_rp;
        hp.col_idx = hp.node_ci;
    } else {
        hp.row_ptr.assign(hp.n_dofs + 1, 0);
        hp.col_idx.resize(hp.nnz);
        for (int64_t i = 0; i < N; ++i) {
            const int32_t m = hp.node_rp[i + 1] - hp.node_rp[i];
            for (int c = 0; c < ncomp; ++c) {
                const int64_t r = i * ncomp + c;
                const int64_t base = (int64_t)ncomp * ncomp * hp.node_rp[i] + (int64_t)c * ncomp * m;
                hp.row_ptr[r] = (int32_t)base;
                for (int32_t q = 0; q < m; ++q)
                    for (int cc = 0; cc < ncomp; ++cc)
                        hp.col_idx[base + q * ncomp + cc] = hp.node_ci[hp.node_rp[i] + q] * ncomp + cc;
            }
        }
        hp.row_ptr[hp.n_dofs] = (int32_t)hp.nnz;
    }
    hp.diag_pos.resize(hp.n_dofs);
    for (int64_t r = 0; r < hp.n_dofs; ++r) {
        auto b = hp.col_idx.begin() + hp.row_ptr[r], e = hp.col_idx.begin() + hp.row_ptr[r + 1];
        hp.diag_pos[r] = (int32_t)(std::lower_bound(b, e, (int32_t)r) - hp.col_idx.begin());
    }

    // ---- sliced-ELL copy of the CSR pattern for the CG iterations: slice s holds
    // rows [64 s, 64 s + 64) (one row per lane of a wave); entry k of row r sits at
    // sell_ptr[s] + 64 k + (r - 64 s), and every row of a slice is padded to the
    // slice's longest row (at least one entry) with its own index as column; when
    // padding every slice to the longest row of all adds at most 1/32 of the
    // entries, every slice is (sell_len)
    {
        const int64_t nsl = (hp.n_dofs + kSellRows - 1) / kSellRows;
        hp.sell_ptr.assign(nsl + 1, 0);
        std::vector<int32_t> slen(nsl, 1);
        int64_t total = 0;
        int32_t lmax = 1;
        for (int64_t s = 0; s < nsl; ++s) {
            for (int64_t r = s * kSellRows; r < std::min<int64_t>(hp.n_dofs, (s + 1) * kSellRows); ++r)
                slen[s] = std::max(slen[s], hp.row_ptr[r + 1] - hp.row_ptr[r]);
            total += slen[s];
            lmax = std::max(lmax, slen[s]);
        }
        hp.sell_len = 0;
        if (nsl > 0 && (int64_t)lmax * nsl * 32 <= total * 33) {
            hp.sell_len = lmax;
            std::fill(slen.begin(), slen.end(), lmax);
        }
        int64_t off = 0;
        for (int64_t s = 0; s < nsl; ++s) {
            const int32_t len = slen[s];
            hp.sell_ptr[s] = (int32_t)off;
            off += (int64_t)len * kSellRows;
            if (off > INT32_MAX) {
                msg = "the padded sliced-ELL pattern exceeds 2^31 entries";
                return TG_E_ARG;
            }
        }
        hp.sell_ptr[nsl] = (int32_t)off;
        hp.sell_col.assign(off, 0);
        for (int64_t s = 0; s < nsl; ++s) {
            const int64_t len = (hp.sell_ptr[s + 1] - hp.sell_ptr[s]) / kSellRows;
            for (int64_t l = 0; l < kSellRows; ++l) {
                const int64_t r = s * kSellRows + l;
                const int32_t p0 = r < hp.n_dofs ? hp.row_ptr[r] : 0, m = r < hp.n_dofs ? hp.row_ptr[r + 1] - p0 : 0;
                for (int64_t q = 0; q < len; ++q)
                    hp.sell_col[hp.sell_ptr[s] + q * kSellRows + l] =
                        q < m ? hp.col_idx[p0 + q] : (int32_t)std::min<int64_t>(r, hp.n_dofs - 1);
            }
        }
        // 16-bit offsets from the clamped row when they all fit (banded numberings:
        // half the index bytes the CG iterations read)
        bool fits = true;
        for (int64_t s = 0; s < nsl && fits; ++s)
            for (int64_t q = hp.sell_ptr[s]; q < hp.sell_ptr[s + 1]; ++q) {
                const int64_t d = (int64_t)hp.sell_col[q] - std::min<int64_t>(s * kSellRows + (q % kSellRows), hp.n_dofs - 1);
                if (d < -32767 || d > 32767) {
                    fits = false;
                    break;
                }
            }
        hp.sell_off.clear();
        if (fits && off > 0) {
            hp.sell_off.resize(off);
            for (int64_t s = 0; s < nsl; ++s)
                for (int64_t q = hp.sell_ptr[s]; q < hp.sell_ptr[s + 1]; ++q)
                    hp.sell_off[q] = (int16_t)((int64_t)hp.sell_col[q] -
                                               std::min<int64_t>(s * kSellRows + (q % kSellRows), hp.n_dofs - 1));
            hp.sell_col.clear();
            hp.sell_col.shrink_to_fit();
        }
    }

    // ---- Dirichlet DoFs
    std::vector<uint8_t> cvert(nv, 0);
    std::vector<FaceKey> bfaces;
    if (n_dirichlet == TG_BOUNDARY_ALL || p2) bfaces = boundary_faces(dim, E, conn);
    if (n_dirichlet == TG_BOUNDARY_ALL) {
        if (dirichlet) {
            msg = "dirichlet_vertices must be NULL with TG_BOUNDARY_ALL";
            return TG_E_ARG;
        }
        for (const FaceKey &f : bfaces)
            for (int a = 0; a < dim; ++a) cvert[f.v[a]] = 1;
    } else if (n_dirichlet > 0) {
        if (!dirichlet) {
            msg = "dirichlet_vertices is NULL";
            return TG_E_ARG;
        }
        for (int64_t t = 0; t < n_dirichlet; ++t) {
            if (dirichlet[t] < 0 || dirichlet[t] >= nv) {
                msg = "Dirichlet vertex id out of range";
                return TG_E_ARG;
            }
            cvert[dirichlet[t]] = 1;
        }
    } else if (n_dirichlet < 0) {
        msg = "n_dirichlet must be >= 0 or TG_BOUNDARY_ALL";
        return TG_E_ARG;
    }
    std::vector<uint8_t> cnode(N, 0);
    for (int64_t v = 0; v < nv; ++v) cnode[v] = cvert[v];
    if (p2) {
        for (const FaceKey &f : bfaces) {
            if (!(cvert[f.v[0]] && cvert[f.v[1]] && cvert[f.v[2]])) continue;
            for (int m = 0; m < 3; ++m) {
                uint64_t p = (uint32_t)f.v[m], q = (uint32_t)f.v[(m + 1) % 3];
                uint64_t key = std::min(p, q) << 32 | std::max(p, q);
                int64_t r = std::lower_bound(edges.begin(), edges.end(), key) - edges.begin();
                cnode[nv + r] = 1;
            }
        }
    }
    hp.constrained.assign(hp.n_dofs, 0);
    hp.constrained_list.clear();
    for (int64_t i = 0; i < N; ++i)
        if (cnode[i])
            for (int c = 0; c < ncomp; ++c) {
                hp.constrained[i * ncomp + c] = 1;
                hp.constrained_list.push_back((int32_t)(i * ncomp + c));
            }
    hp.dirichlet_rows.clear();
    for (int64_t r = 0; r < hp.n_dofs; ++r) {
        bool touched = hp.constrained[r] != 0;
        for (int32_t q = hp.row_ptr[r]; !touched && q < hp.row_ptr[r + 1]; ++q) touched = hp.constrained[hp.col_idx[q]];
        if (touched) hp.dirichlet_rows.push_back((int32_t)r);
    }
    return TG_OK;
}

}  // namespace tg
