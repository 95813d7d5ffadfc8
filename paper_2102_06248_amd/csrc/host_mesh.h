// Host-side mesh build of libfepic: canonical topology, barycentric geometry, assembly of
// the edge mass and curl-curl matrices (Sec. II-A) into sliced-ELLPACK, and the bucket
// grid used for point location.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fepic_internal.h"

namespace fepic {

struct HostMesh {
    int64_t n_nodes = 0, n_tets = 0, n_edges = 0, n_faces = 0;
    int64_t n_int_edges = 0, n_int_nodes = 0;
    std::vector<double> xyz;          // [n_nodes][3]
    std::vector<int32_t> tets;        // [n_tets][4], node ids ascending
    std::vector<int32_t> edges;       // [n_edges][2]
    std::vector<int32_t> faces;       // [n_faces][3]
    std::vector<int32_t> tet_edges;   // [n_tets][6]
    std::vector<int32_t> tet_faces;   // [n_tets][4], face opposite local vertex k
    std::vector<int32_t> nbr;         // [n_tets][4], -1 on the wall
    std::vector<int8_t> nbr_far;      // [n_tets][4], neighbour's local index of its far vertex
    std::vector<int32_t> face_edges;  // [n_faces][3]: (i,j), (j,k), (i,k)
    std::vector<uint8_t> bedge, bnode;
    std::vector<int32_t> int_edges;   // interior edge ids, ascending
    // Device numbering of edges: canonical edges re-ordered along a Morton curve of their
    // midpoints, so consecutive matrix rows (and the columns they gather) are close in
    // space and in memory.  All device arrays use it; the C ABI converts at its boundary.
    std::vector<int32_t> eperm;        // canonical edge id -> device edge id
    std::vector<int32_t> eiperm;       // device edge id -> canonical edge id
    std::vector<int32_t> dev_edges;       // [n_edges][2] node pairs, device order
    std::vector<int32_t> dev_tet_edges;   // [n_tets][6] device edge ids
    std::vector<int32_t> dev_face_edges;  // [n_faces][3] device edge ids
    std::vector<uint8_t> dev_bedge;       // wall flag, device order
    std::vector<uint8_t> dev_fixed;       // fixed (PEC) edges, device order: the wall edges
                                          // not on an absorbing face
    std::vector<uint8_t> abc_face;        // [n_faces] absorbing wall faces (empty: none)
    std::vector<int32_t> dev_int_edges;   // interior edges, device ids ascending
    std::vector<double> grad;         // [n_tets][9] grad lambda_1..3
    std::vector<double> vol;          // [n_tets]
    SellMatrix mat;                   // M and S over all edge rows in device order (boundary rows:
                                      // diagonal only)
    // Nodal auxiliary space of the Newmark preconditioner: interior nodes in Morton order.
    int64_t n_aux = 0;
    std::vector<int32_t> aux_node;    // auxiliary index -> node id
    std::vector<int64_t> aux_sp;      // SELL-64 slice offsets of the node incidence lists
    std::vector<int32_t> aux_inc;     // device edge id (node is its head) or ~id (its tail);
                                      // kAuxPad in padding
    std::vector<EdgeVec> aux_th;      // [n_edges] (r_head - r_tail) / 2 over the largest
                                      // component, FP16; zero on wall edges
    std::vector<int32_t> aux_ends;    // [n_edges][2] auxiliary index of tail, head; n_aux for
                                      // wall nodes (and both ends of wall edges)
    // point-location grid
    double grid_lo[3] = {0, 0, 0}, grid_inv_h[3] = {1, 1, 1};
    int32_t grid_n[3] = {1, 1, 1};
    std::vector<int32_t> cell_start, cell_tets;
};

// Returns FEPIC_OK or FEPIC_E_MESH/FEPIC_E_ARG with a message in err.
int build_host_mesh(HostMesh& m, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets,
                    std::string& err);

// The edge matrices over the unknown edges (not `fixed`, device order), and with absorbing
// faces (abc_face per canonical face, or empty) their boundary matrix K; see host_mesh.cpp.
int assemble_edge_matrices(HostMesh& m, const std::vector<uint8_t>& fixed, const std::vector<uint8_t>& abc_face,
                           std::string& err);

// Face area vectors 1/2 (r_j - r_i) x (r_k - r_i).
void face_area_vectors(const HostMesh& m, std::vector<double>& out);

}  // namespace fepic
