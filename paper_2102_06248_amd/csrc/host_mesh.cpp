// Host-side mesh build of libfepic (see host_mesh.h).
#include "host_mesh.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

namespace fepic {

namespace {

constexpr int kLE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
constexpr int kLF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

// local edge index of local vertex pair (a, b), a < b
inline int local_edge(int a, int b) {
    static const int t[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
    return t[a][b];
}

inline void cross(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Morton code of a point of the box [lo, hi]: 21 bits per axis, interleaved x y z.
uint64_t morton_key(const double* p, const double* lo, const double* hi) {
    auto spread = [](uint64_t v) {  // 21 bits -> every third bit
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffull;
        v = (v | v << 16) & 0x1f0000ff0000ffull;
        v = (v | v << 8) & 0x100f00f00f00f00full;
        v = (v | v << 4) & 0x10c30c30c30c30c3ull;
        v = (v | v << 2) & 0x1249249249249249ull;
        return v;
    };
    uint64_t q[3];
    for (int d = 0; d < 3; ++d) {
        const double ext = hi[d] - lo[d];
        const double f = ext > 0 ? (p[d] - lo[d]) / ext : 0.0;
        q[d] = (uint64_t)std::min(2097151.0, std::max(0.0, f * 2097151.0));
    }
    return spread(q[0]) | spread(q[1]) << 1 | spread(q[2]) << 2;
}

}  // namespace

// Nodal auxiliary space of the Newmark preconditioner: the interior nodes in Morton order
// of their positions (ties in node order; runs of 8 and 64 consecutive nodes are the
// aggregates of the coarser levels), each with the list of its interior edges in SELL-64
// layout, and per edge the half edge vector and the auxiliary indices of its ends.
void build_aux_space(HostMesh& m) {
    const int64_t nn = m.n_nodes, ne = m.n_edges;
    double lo3[3] = {1e300, 1e300, 1e300}, hi3[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < nn; ++v)
        for (int d = 0; d < 3; ++d) {
            lo3[d] = std::min(lo3[d], m.xyz[3 * v + d]);
            hi3[d] = std::max(hi3[d], m.xyz[3 * v + d]);
        }
    // interior edges of every node, device edge ids ascending
    std::vector<int64_t> start(nn + 1, 0);
    for (int64_t d = 0; d < ne; ++d)
        if (!m.dev_bedge[d]) {
            start[m.dev_edges[2 * d] + 1]++;
            start[m.dev_edges[2 * d + 1] + 1]++;
        }
    for (int64_t v = 0; v < nn; ++v) start[v + 1] += start[v];
    std::vector<int32_t> code(start[nn]);
    {
        std::vector<int64_t> pos(start.begin(), start.end() - 1);
        for (int64_t d = 0; d < ne; ++d)
            if (!m.dev_bedge[d]) {
                code[pos[m.dev_edges[2 * d]]++] = ~(int32_t)d;   // tail: -1 in the gradient
                code[pos[m.dev_edges[2 * d + 1]]++] = (int32_t)d;  // head: +1
            }
    }
    std::vector<int32_t> order;
    std::vector<uint64_t> key(nn, 0);
    for (int64_t v = 0; v < nn; ++v)
        if (!m.bnode[v]) {
            order.push_back((int32_t)v);
            key[v] = morton_key(&m.xyz[3 * v], lo3, hi3);
        }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    auto deg = [&](int32_t v) { return start[v + 1] - start[v]; };
    const int64_t na = (int64_t)order.size();
    m.n_aux = na;
    m.aux_node = order;
    std::vector<int32_t> aux_of(nn, (int32_t)na);   // wall nodes -> the zero entry
    for (int64_t a = 0; a < na; ++a) aux_of[order[a]] = (int32_t)a;
    const int64_t nsl = (na + kSell - 1) / kSell;
    m.aux_sp.assign(nsl + 1, 0);
    for (int64_t s = 0; s < nsl; ++s) {
        int64_t w = 0;
        for (int l = 0; l < kSell && s * kSell + l < na; ++l) w = std::max(w, deg(order[s * kSell + l]));
        m.aux_sp[s + 1] = m.aux_sp[s] + w * kSell;
    }
    m.aux_inc.assign(m.aux_sp[nsl], kAuxPad);
    for (int64_t a = 0; a < na; ++a) {
        const int32_t v = order[a];
        const int64_t s = a / kSell, l = a % kSell;
        for (int64_t k = 0; k < deg(v); ++k) m.aux_inc[m.aux_sp[s] + k * kSell + l] = code[start[v] + k];
    }
    double scale = 0.0;
    for (int64_t d = 0; d < ne; ++d) {
        if (m.dev_bedge[d]) continue;
        const int32_t a = m.dev_edges[2 * d], b = m.dev_edges[2 * d + 1];
        for (int k = 0; k < 3; ++k) scale = std::max(scale, std::fabs(0.5 * (m.xyz[3 * b + k] - m.xyz[3 * a + k])));
    }
    const double inv = scale > 0 ? 1.0 / scale : 1.0;
    m.aux_th.assign(ne, EdgeVec{});
    m.aux_ends.assign(2 * ne, (int32_t)na);
    for (int64_t d = 0; d < ne; ++d) {
        if (m.dev_bedge[d]) continue;
        const int32_t a = m.dev_edges[2 * d], b = m.dev_edges[2 * d + 1];
        EdgeVec& t = m.aux_th[d];
        t.x = (_Float16)(0.5 * (m.xyz[3 * b] - m.xyz[3 * a]) * inv);
        t.y = (_Float16)(0.5 * (m.xyz[3 * b + 1] - m.xyz[3 * a + 1]) * inv);
        t.z = (_Float16)(0.5 * (m.xyz[3 * b + 2] - m.xyz[3 * a + 2]) * inv);
        m.aux_ends[2 * d] = aux_of[a];
        m.aux_ends[2 * d + 1] = aux_of[b];
    }
}

// The edge matrices over the unknown edges (those not in `fixed`, device order) in SELL-64:
// M = [*eps0] and S = [curl]^T [*mu0^-1] [curl] element by element in closed form, rows of
// fixed edges reduced to a unit diagonal; with absorbing faces (abc_face, canonical face
// ids) also their boundary matrix K in the same pattern.
int assemble_edge_matrices(HostMesh& m, const std::vector<uint8_t>& fixed, const std::vector<uint8_t>& abc_face,
                           std::string& err) {
    const std::vector<int32_t>& TE = m.dev_tet_edges;
    const std::vector<uint8_t>& BE = fixed;
    const int64_t n_tets = m.n_tets;

    // ---- assembly pattern (device order): row e couples to the interior edges of every
    // tet holding e
    const int64_t ne = m.n_edges;
    std::vector<int64_t> et_start(ne + 1, 0);
    for (int64_t j = 0; j < 6 * n_tets; ++j) et_start[TE[j] + 1]++;
    for (int64_t e = 0; e < ne; ++e) et_start[e + 1] += et_start[e];
    std::vector<int32_t> et(6 * n_tets);
    {
        std::vector<int64_t> pos(et_start.begin(), et_start.end() - 1);
        for (int64_t j = 0; j < 6 * n_tets; ++j) et[pos[TE[j]]++] = (int32_t)(j / 6);
    }
    SellMatrix& A = m.mat;
    A.n_rows = ne;
    A.n_slices = (ne + kSell - 1) / kSell;
    std::vector<int32_t> rlen(A.n_slices * kSell, 0);
    std::vector<int64_t> rstart(ne + 1, 0);
    std::vector<int32_t> rcols;
    rcols.reserve(ne * 17);
    std::vector<int32_t> tmp;
    for (int64_t e = 0; e < ne; ++e) {
        rstart[e] = (int64_t)rcols.size();
        rcols.push_back((int32_t)e);  // diagonal first
        if (!BE[e]) {
            tmp.clear();
            for (int64_t j = et_start[e]; j < et_start[e + 1]; ++j) {
                const int t = et[j];
                for (int i = 0; i < 6; ++i) {
                    const int32_t c = TE[6 * t + i];
                    if (c != e && !BE[c]) tmp.push_back(c);
                }
            }
            std::sort(tmp.begin(), tmp.end());
            tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
            rcols.insert(rcols.end(), tmp.begin(), tmp.end());
        }
        rlen[e] = (int32_t)(rcols.size() - rstart[e]);
    }
    rstart[ne] = (int64_t)rcols.size();
    A.slice_ptr.assign(A.n_slices + 1, 0);
    for (int64_t s = 0; s < A.n_slices; ++s) {
        int32_t w = 0;
        for (int l = 0; l < kSell; ++l) w = std::max(w, rlen[s * kSell + l]);
        A.slice_ptr[s + 1] = A.slice_ptr[s] + (int64_t)w * kSell;
    }
    const int64_t total = A.slice_ptr[A.n_slices];
    A.col.assign(total, 0);
    A.M.assign(total, 0.0);
    A.S.assign(total, 0.0);
    for (int64_t s = 0; s < A.n_slices; ++s) {
        const int64_t w = (A.slice_ptr[s + 1] - A.slice_ptr[s]) / kSell;
        for (int l = 0; l < kSell; ++l) {
            const int64_t r = s * kSell + l;
            for (int64_t k = 0; k < w; ++k) {
                int32_t c = 0;
                if (r < ne) c = (k < rlen[r]) ? rcols[rstart[r] + k] : (int32_t)r;
                A.col[A.slice_ptr[s] + k * kSell + l] = c;
            }
        }
    }
    auto slot = [&](int64_t r, int32_t c) -> int64_t {
        const int64_t s = r / kSell, l = r % kSell;
        if (c == r) return A.slice_ptr[s] + l;
        // columns after the diagonal are ascending
        int64_t lo = 1, hi = rlen[r] - 1;
        while (lo <= hi) {
            const int64_t mid = (lo + hi) / 2;
            const int32_t v = rcols[rstart[r] + mid];
            if (v == c) return A.slice_ptr[s] + mid * kSell + l;
            if (v < c) lo = mid + 1; else hi = mid - 1;
        }
        return -1;
    };
    // element matrices, closed form:
    //   M_(ab)(cd) = eps0 V/20 [(1+d_ac) g_b.g_d - (1+d_ad) g_b.g_c - (1+d_bc) g_a.g_d + (1+d_bd) g_a.g_c]
    //   S_(ab)(cd) = 4 V / mu0 (g_a x g_b) . (g_c x g_d)
    for (int64_t t = 0; t < n_tets; ++t) {
        double g[4][3];
        for (int k = 1; k < 4; ++k)
            for (int d = 0; d < 3; ++d) g[k][d] = m.grad[9 * t + 3 * (k - 1) + d];
        for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        double gg[4][4], cr[6][3];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) gg[a][b] = dot(g[a], g[b]);
        for (int i = 0; i < 6; ++i) cross(g[kLE[i][0]], g[kLE[i][1]], cr[i]);
        const double V = m.vol[t];
        const double mc = kEps0 * V / 20.0, sc = 4.0 * V / kMu0;
        for (int i = 0; i < 6; ++i) {
            const int32_t ei = TE[6 * t + i];
            if (BE[ei]) continue;
            const int a = kLE[i][0], b = kLE[i][1];
            for (int j = 0; j < 6; ++j) {
                const int32_t ej = TE[6 * t + j];
                if (BE[ej]) continue;
                const int c = kLE[j][0], d = kLE[j][1];
                const double Mv = mc * ((1 + (a == c)) * gg[b][d] - (1 + (a == d)) * gg[b][c] -
                                        (1 + (b == c)) * gg[a][d] + (1 + (b == d)) * gg[a][c]);
                const double Sv = sc * dot(cr[i], cr[j]);
                const int64_t p = slot(ei, ej);
                if (p < 0) {
                    err = "internal: assembly pattern miss";
                    return FEPIC_E_MESH;
                }
                A.M[p] += Mv;
                A.S[p] += Sv;
            }
        }
    }
    // absorbing faces: K = int over the face of (n x W_a) . (n x W_b), the tangential traces
    // being the triangle's own Whitney functions mu_a grad mu_b - mu_b grad mu_a, with
    // int mu_i mu_j = A (1 + delta_ij) / 12 and surface gradients grad mu_i = N x (edge
    // opposite i, taken around the triangle) / |N|^2, N = (p1 - p0) x (p2 - p0)
    A.K.clear();
    if (!abc_face.empty()) {
        A.K.assign(total, 0.0);
        constexpr int kTE[3][2] = {{0, 1}, {1, 2}, {0, 2}};   // face_edges order: (i,j), (j,k), (i,k)
        for (int64_t f = 0; f < m.n_faces; ++f) {
            if (!abc_face[f]) continue;
            const double* p[3] = {&m.xyz[3 * m.faces[3 * f]], &m.xyz[3 * m.faces[3 * f + 1]],
                                  &m.xyz[3 * m.faces[3 * f + 2]]};
            double u[3], v[3], N[3];
            for (int d = 0; d < 3; ++d) {
                u[d] = p[1][d] - p[0][d];
                v[d] = p[2][d] - p[0][d];
            }
            cross(u, v, N);
            const double n2 = dot(N, N), area = 0.5 * std::sqrt(n2);
            double gm[3][3];
            for (int i = 0; i < 3; ++i) {
                const double* a = p[(i + 1) % 3];
                const double* b = p[(i + 2) % 3];
                double ed[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, t[3];
                cross(N, ed, t);
                for (int d = 0; d < 3; ++d) gm[i][d] = t[d] / n2;
            }
            const double kc = area / 12.0;
            for (int i = 0; i < 3; ++i) {
                const int32_t ei = m.dev_face_edges[3 * f + i];
                if (BE[ei]) continue;
                const int a = kTE[i][0], b = kTE[i][1];
                for (int j = 0; j < 3; ++j) {
                    const int32_t ej = m.dev_face_edges[3 * f + j];
                    if (BE[ej]) continue;
                    const int cc = kTE[j][0], d = kTE[j][1];
                    const double Kv = kc * ((1 + (a == cc)) * dot(gm[b], gm[d]) - (1 + (a == d)) * dot(gm[b], gm[cc]) -
                                            (1 + (b == cc)) * dot(gm[a], gm[d]) + (1 + (b == d)) * dot(gm[a], gm[cc]));
                    const int64_t q = slot(ei, ej);
                    if (q < 0) {
                        err = "internal: boundary pattern miss";
                        return FEPIC_E_MESH;
                    }
                    A.K[q] += Kv;
                }
            }
        }
    }
    // fixed rows: keep a unit mass on the diagonal (identity rows after scaling)
    for (int64_t e = 0; e < ne; ++e)
        if (BE[e]) A.M[slot(e, (int32_t)e)] = 1.0;
    return FEPIC_OK;
}

int build_host_mesh(HostMesh& m, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets_in,
                    std::string& err) {
    if (n_nodes <= 0 || n_tets <= 0 || !xyz || !tets_in) {
        err = "empty mesh";
        return FEPIC_E_ARG;
    }
    if (n_nodes >= (int64_t)1 << 31 || n_tets >= (int64_t)1 << 29) {
        err = "mesh too large for 32-bit ids";
        return FEPIC_E_ARG;
    }
    m.n_nodes = n_nodes;
    m.n_tets = n_tets;
    m.xyz.assign(xyz, xyz + 3 * n_nodes);
    m.tets.resize(4 * n_tets);
    for (int64_t t = 0; t < n_tets; ++t) {
        std::array<int32_t, 4> v = {tets_in[4 * t], tets_in[4 * t + 1], tets_in[4 * t + 2], tets_in[4 * t + 3]};
        for (int k = 0; k < 4; ++k)
            if (v[k] < 0 || v[k] >= n_nodes) {
                err = "tet " + std::to_string(t) + " has an out-of-range node id";
                return FEPIC_E_MESH;
            }
        std::sort(v.begin(), v.end());
        if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) {
            err = "tet " + std::to_string(t) + " repeats a node";
            return FEPIC_E_MESH;
        }
        for (int k = 0; k < 4; ++k) m.tets[4 * t + k] = v[k];
    }

    // ---- geometry: J = [r1-r0, r2-r0, r3-r0] (columns); grad lambda_1..3 = rows of J^-1
    m.grad.resize(9 * n_tets);
    m.vol.resize(n_tets);
    double hmax = 0.0;
    for (int64_t t = 0; t < n_tets; ++t) {
        const double* r0 = &m.xyz[3 * m.tets[4 * t]];
        double c[3][3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) c[k][d] = m.xyz[3 * m.tets[4 * t + k + 1] + d] - r0[d];
        double bc[3], ca[3], ab[3];
        cross(c[1], c[2], bc);
        cross(c[2], c[0], ca);
        cross(c[0], c[1], ab);
        const double det = dot(c[0], bc);
        double len = 0.0;
        for (int k = 0; k < 3; ++k) len = std::max(len, std::sqrt(dot(c[k], c[k])));
        hmax = std::max(hmax, len);
        if (!(std::fabs(det) > 1e-12 * len * len * len)) {
            err = "tet " + std::to_string(t) + " is degenerate";
            return FEPIC_E_MESH;
        }
        for (int d = 0; d < 3; ++d) {
            m.grad[9 * t + d] = bc[d] / det;
            m.grad[9 * t + 3 + d] = ca[d] / det;
            m.grad[9 * t + 6 + d] = ab[d] / det;
        }
        m.vol[t] = std::fabs(det) / 6.0;
    }

    // ---- edges: sorted unique node pairs
    {
        const int64_t ni = 6 * n_tets;
        std::vector<uint64_t> key(ni);
        for (int64_t t = 0; t < n_tets; ++t)
            for (int i = 0; i < 6; ++i)
                key[6 * t + i] = (uint64_t)m.tets[4 * t + kLE[i][0]] * (uint64_t)n_nodes + m.tets[4 * t + kLE[i][1]];
        std::vector<int64_t> ord(ni);
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        m.tet_edges.resize(ni);
        m.edges.clear();
        int64_t ne = -1;
        uint64_t prev = ~0ull;
        for (int64_t j = 0; j < ni; ++j) {
            const uint64_t k = key[ord[j]];
            if (k != prev) {
                ++ne;
                prev = k;
                m.edges.push_back((int32_t)(k / n_nodes));
                m.edges.push_back((int32_t)(k % n_nodes));
            }
            m.tet_edges[ord[j]] = (int32_t)ne;
        }
        m.n_edges = ne + 1;
    }

    // ---- faces: sorted unique node triples; neighbours across them
    {
        const int64_t ni = 4 * n_tets;
        std::vector<std::array<int32_t, 3>> key(ni);
        for (int64_t t = 0; t < n_tets; ++t)
            for (int k = 0; k < 4; ++k)
                key[4 * t + k] = {m.tets[4 * t + kLF[k][0]], m.tets[4 * t + kLF[k][1]], m.tets[4 * t + kLF[k][2]]};
        std::vector<int64_t> ord(ni);
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        m.tet_faces.resize(ni);
        m.nbr.assign(ni, -1);
        m.nbr_far.assign(ni, -1);
        m.faces.clear();
        std::vector<int64_t> first_inst;
        int64_t nf = -1;
        for (int64_t j = 0; j < ni; ++j) {
            const int64_t inst = ord[j];
            if (j == 0 || key[inst] != key[ord[j - 1]]) {
                ++nf;
                for (int d = 0; d < 3; ++d) m.faces.push_back(key[inst][d]);
                first_inst.push_back(inst);
            } else {
                if (j >= 2 && key[inst] == key[ord[j - 2]]) {
                    err = "non-conforming mesh: a face is shared by more than two tets";
                    return FEPIC_E_MESH;
                }
                const int64_t a = first_inst[nf], b = inst;
                m.nbr[a] = (int32_t)(b / 4);
                m.nbr[b] = (int32_t)(a / 4);
                m.nbr_far[a] = (int8_t)(b % 4);
                m.nbr_far[b] = (int8_t)(a % 4);
            }
            m.tet_faces[inst] = (int32_t)nf;
        }
        m.n_faces = nf + 1;
        // face -> edges, from the tet that first listed it
        m.face_edges.resize(3 * m.n_faces);
        for (int64_t f = 0; f < m.n_faces; ++f) {
            const int64_t inst = first_inst[f];
            const int64_t t = inst / 4;
            const int k = (int)(inst % 4);
            const int i = kLF[k][0], jj = kLF[k][1], l = kLF[k][2];
            m.face_edges[3 * f] = m.tet_edges[6 * t + local_edge(i, jj)];
            m.face_edges[3 * f + 1] = m.tet_edges[6 * t + local_edge(jj, l)];
            m.face_edges[3 * f + 2] = m.tet_edges[6 * t + local_edge(i, l)];
        }
    }

    // ---- wall entities
    m.bedge.assign(m.n_edges, 0);
    m.bnode.assign(n_nodes, 0);
    for (int64_t t = 0; t < n_tets; ++t)
        for (int k = 0; k < 4; ++k) {
            if (m.nbr[4 * t + k] >= 0) continue;
            const int i = kLF[k][0], j = kLF[k][1], l = kLF[k][2];
            m.bnode[m.tets[4 * t + i]] = m.bnode[m.tets[4 * t + j]] = m.bnode[m.tets[4 * t + l]] = 1;
            m.bedge[m.tet_edges[6 * t + local_edge(i, j)]] = 1;
            m.bedge[m.tet_edges[6 * t + local_edge(j, l)]] = 1;
            m.bedge[m.tet_edges[6 * t + local_edge(i, l)]] = 1;
        }
    m.int_edges.clear();
    for (int64_t e = 0; e < m.n_edges; ++e)
        if (!m.bedge[e]) m.int_edges.push_back((int32_t)e);
    m.n_int_edges = (int64_t)m.int_edges.size();
    m.n_int_nodes = 0;
    for (int64_t v = 0; v < n_nodes; ++v) m.n_int_nodes += !m.bnode[v];

    // ---- device edge numbering: Morton order of edge midpoints, rows of equal length
    // grouped within windows of kSortWindow rows
    constexpr int64_t kSortWindow = 8 * kSell;
    {
        const int64_t ne0 = m.n_edges;
        double lo3[3] = {1e300, 1e300, 1e300}, hi3[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < n_nodes; ++v)
            for (int d = 0; d < 3; ++d) {
                lo3[d] = std::min(lo3[d], m.xyz[3 * v + d]);
                hi3[d] = std::max(hi3[d], m.xyz[3 * v + d]);
            }
        std::vector<uint64_t> key(ne0);
        for (int64_t e = 0; e < ne0; ++e) {
            double mid[3];
            for (int d = 0; d < 3; ++d)
                mid[d] = 0.5 * (m.xyz[3 * m.edges[2 * e] + d] + m.xyz[3 * m.edges[2 * e + 1] + d]);
            key[e] = morton_key(mid, lo3, hi3);
        }
        m.eiperm.resize(ne0);
        std::iota(m.eiperm.begin(), m.eiperm.end(), 0);
        std::stable_sort(m.eiperm.begin(), m.eiperm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        // Within windows of kSortWindow consecutive rows, order rows by their stored length
        // (stable, so Morton order is kept among equal lengths): slices of 64 rows then
        // hold rows of one length and carry little padding.
        {
            std::vector<int64_t> ets(ne0 + 1, 0);
            for (int64_t j = 0; j < 6 * n_tets; ++j) ets[m.tet_edges[j] + 1]++;
            for (int64_t e = 0; e < ne0; ++e) ets[e + 1] += ets[e];
            std::vector<int32_t> etl(6 * n_tets);
            std::vector<int64_t> pos(ets.begin(), ets.end() - 1);
            for (int64_t j = 0; j < 6 * n_tets; ++j) etl[pos[m.tet_edges[j]]++] = (int32_t)(j / 6);
            std::vector<int32_t> len(ne0, 1), nb;
            for (int64_t e = 0; e < ne0; ++e) {
                if (m.bedge[e]) continue;
                nb.clear();
                for (int64_t j = ets[e]; j < ets[e + 1]; ++j)
                    for (int i = 0; i < 6; ++i) {
                        const int32_t c = m.tet_edges[6 * etl[j] + i];
                        if (c != e && !m.bedge[c]) nb.push_back(c);
                    }
                std::sort(nb.begin(), nb.end());
                len[e] = 1 + (int32_t)(std::unique(nb.begin(), nb.end()) - nb.begin());
            }
            for (int64_t w0 = 0; w0 < ne0; w0 += kSortWindow) {
                const int64_t w1 = std::min<int64_t>(ne0, w0 + kSortWindow);
                std::stable_sort(m.eiperm.begin() + w0, m.eiperm.begin() + w1,
                                 [&](int32_t a, int32_t b) { return len[a] > len[b]; });
            }
        }
        m.eperm.resize(ne0);
        for (int64_t d = 0; d < ne0; ++d) m.eperm[m.eiperm[d]] = (int32_t)d;
        m.dev_edges.resize(2 * ne0);
        m.dev_bedge.resize(ne0);
        for (int64_t d = 0; d < ne0; ++d) {
            const int32_t e = m.eiperm[d];
            m.dev_edges[2 * d] = m.edges[2 * e];
            m.dev_edges[2 * d + 1] = m.edges[2 * e + 1];
            m.dev_bedge[d] = m.bedge[e];
        }
        m.dev_tet_edges.resize(m.tet_edges.size());
        for (size_t j = 0; j < m.tet_edges.size(); ++j) m.dev_tet_edges[j] = m.eperm[m.tet_edges[j]];
        m.dev_face_edges.resize(m.face_edges.size());
        for (size_t j = 0; j < m.face_edges.size(); ++j) m.dev_face_edges[j] = m.eperm[m.face_edges[j]];
        m.dev_int_edges.clear();
        for (int64_t d = 0; d < ne0; ++d)
            if (!m.dev_bedge[d]) m.dev_int_edges.push_back((int32_t)d);
    }
    {
        m.dev_fixed = m.dev_bedge;
        m.abc_face.clear();
        const int rc = assemble_edge_matrices(m, m.dev_fixed, m.abc_face, err);
        if (rc != FEPIC_OK) return rc;
    }

    build_aux_space(m);

    // ---- point-location grid
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < n_nodes; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], m.xyz[3 * v + d]);
            hi[d] = std::max(hi[d], m.xyz[3 * v + d]);
        }
    double ext[3], volb = 1.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = std::max(hi[d] - lo[d], 1e-300);
        volb *= ext[d];
    }
    const double target_cells = std::max(1.0, (double)n_tets / 2.0);
    const double h = std::cbrt(volb / target_cells);
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        m.grid_n[d] = (int32_t)std::max(1.0, std::min(1024.0, std::ceil(ext[d] / h)));
        m.grid_lo[d] = lo[d];
        m.grid_inv_h[d] = m.grid_n[d] / ext[d];
        ncell *= m.grid_n[d];
    }
    auto cell_of = [&](double x, int d) {
        int c = (int)std::floor((x - m.grid_lo[d]) * m.grid_inv_h[d]);
        return std::min(std::max(c, 0), m.grid_n[d] - 1);
    };
    std::vector<std::array<int, 6>> rng(n_tets);
    m.cell_start.assign(ncell + 1, 0);
    for (int64_t t = 0; t < n_tets; ++t) {
        double tl[3] = {1e300, 1e300, 1e300}, th[3] = {-1e300, -1e300, -1e300};
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) {
                tl[d] = std::min(tl[d], m.xyz[3 * m.tets[4 * t + k] + d]);
                th[d] = std::max(th[d], m.xyz[3 * m.tets[4 * t + k] + d]);
            }
        auto& r = rng[t];
        for (int d = 0; d < 3; ++d) {
            const double pad = 1e-9 * ext[d];
            r[2 * d] = cell_of(tl[d] - pad, d);
            r[2 * d + 1] = cell_of(th[d] + pad, d);
        }
        for (int z = r[4]; z <= r[5]; ++z)
            for (int y = r[2]; y <= r[3]; ++y)
                for (int x = r[0]; x <= r[1]; ++x) m.cell_start[x + m.grid_n[0] * (y + (int64_t)m.grid_n[1] * z) + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) m.cell_start[c + 1] += m.cell_start[c];
    m.cell_tets.assign(m.cell_start[ncell], 0);
    {
        std::vector<int32_t> pos(m.cell_start.begin(), m.cell_start.end() - 1);
        for (int64_t t = 0; t < n_tets; ++t) {
            const auto& r = rng[t];
            for (int z = r[4]; z <= r[5]; ++z)
                for (int y = r[2]; y <= r[3]; ++y)
                    for (int x = r[0]; x <= r[1]; ++x)
                        m.cell_tets[pos[x + m.grid_n[0] * (y + (int64_t)m.grid_n[1] * z)]++] = (int32_t)t;
        }
    }
    (void)hmax;
    return FEPIC_OK;
}

void face_area_vectors(const HostMesh& m, std::vector<double>& out) {
    out.resize(3 * m.n_faces);
    for (int64_t f = 0; f < m.n_faces; ++f) {
        const double* a = &m.xyz[3 * m.faces[3 * f]];
        const double* b = &m.xyz[3 * m.faces[3 * f + 1]];
        const double* c = &m.xyz[3 * m.faces[3 * f + 2]];
        double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double w[3];
        cross(u, v, w);
        for (int d = 0; d < 3; ++d) out[3 * f + d] = 0.5 * w[d];
    }
}

}  // namespace fepic
