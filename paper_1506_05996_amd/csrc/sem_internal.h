// Internal state of a sem_mesh handle, shared by the host set-up (sem_setup.cpp)
// and the device side (sem_device.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sem.h"

namespace sem {

// Status carrier for internal code: never crosses the C ABI as an exception.
struct Error {
  int status;
  std::string msg;
};

void set_error(const std::string& msg);

// --- entity records ---------------------------------------------------------
// Each element has 27 node classes: class c = cx + 3 cy + 9 cz with
// cx = 0 (i = 0), 1 (0 < i < N), 2 (i = N), likewise cy, cz.  Class 13 is the
// element interior, the 8 corner classes are vertices, 12 are edges and 6 faces.
// For every class the global id of local node (i,j,k) is affine:
//     gid = gbase + ai*i + aj*j + ak*k,
// and so is its slot in the shared-node work array w (faces: 2 slots per face
// node, edges and vertices: one slot per incident element):
//     wid = wbase + ai*i + aj*j + ak*k.
// Record layout (int32 x4): gbase, packed coefficients (three signed 10-bit
// fields), wbase, flags.
constexpr int kRecInts = 4;  // kernels read a record as one int4
constexpr int kClasses = 27;
constexpr int kInteriorClass = 13;
constexpr int kFlagOwned = 1;     // this element holds the first local copy of the node
constexpr int kFlagInterior = 2;  // interior node: written straight to the global vector
constexpr int kFlagMaskedInterior = 4;  // (interior record) some interior node of the element is Dirichlet

inline int32_t pack_coef(int ai, int aj, int ak) {
  return (ai & 0x3FF) | ((aj & 0x3FF) << 10) | ((ak & 0x3FF) << 20);
}

// Coarse solve by nested dissection.  The free-vertex graph of each connected
// component is split recursively by separators (one BFS level across the
// longest extent); the separators and the final small parts are the nodes of
// a forest, numbered in post-order, and each node's own vertices form one
// contiguous range of coarse indices.  A node t holds its own vertices I and
// the boundary B: the vertices of its ancestors coupled to its subtree once
// the subtree is eliminated.  After elimination of the subtree, the front
// [F_II F_IB; F_BI F_BB] gives S = F_II and W = F_BI S^-1.
// Nodes with s <= kSmallFront are "small": their forward product runs one lane
// per row (the forward matrix is stored transposed so that lanes read
// consecutive rows); larger nodes, and every backward product, use one wave
// per row.
constexpr int kSmallFront = 128;

struct FrontNode {
  int64_t off;     // first coarse index of the node's own vertices
  int64_t fwd;     // offset of [S^-1 ; W] in the forward pool: (s + b) x s row-major,
                   // or column-major (leading dimension s + b) for a small node
  int64_t bwd;     // offset of W^T (s x b, row-major) in the backward pool
  int64_t bidx;    // offset of the boundary list (ascending coarse indices) in fb_idx
  int64_t coff;    // offset of the node's contribution W y in the contribution vector
  int32_t s;       // own vertices
  int32_t b;       // boundary vertices
  int32_t parent;  // -1 for a root
  int32_t height;  // 0 for a leaf, else 1 + the largest height of its children
  int32_t small;   // 1 when s <= kSmallFront
  int32_t pad;
};

// Tile shape of the sweeps for a row length L: rows per wave (4 for short
// rows, whose node vector serves four rows; 2 beyond 256) and, beyond 1024
// columns, rows split across the workgroup's 4 waves (more waves in flight
// for the long rows of the upper heights).  A tile holds rw rows when split,
// else 4 rw.
struct CoarseTileShape {
  int32_t rw;
  int32_t split;
};
inline CoarseTileShape coarse_tile_shape(int64_t L) {
  if (L <= 256) return CoarseTileShape{4, 0};
  return CoarseTileShape{2, L > 1024 ? 1 : 0};
}
inline int32_t coarse_tile_rows(const CoarseTileShape& t) { return t.split ? t.rw : 4 * t.rw; }

// one row of a per-height work list: (node, row or column of that node)
struct RowItem {
  int32_t node;
  int32_t row;
};

struct HostTables {
  int N = 0, n1 = 0, np = 0;  // order, N+1, N+3
  int64_t E = 0, n_global = 0, n_local = 0;
  int64_t V = 0, n_edges = 0, n_faces = 0;
  int64_t base_e = 0, base_f = 0, base_i = 0;  // first global id of edges, faces, interiors

  // reference data
  std::vector<double> t, rho, D;  // D[i*(N+1)+j] = phi_j'(t_i)
  std::vector<double> S, lam;     // fast-diagonalisation basis by parity (packed, [(N+3)/2 rows][N+3] + middle row), eigenvalues [N+3]

  // numbering and gather
  std::vector<int32_t> rec;              // [E][27][4]
  std::vector<uint8_t> dir;              // [n_global] 1 = Dirichlet
  std::vector<int32_t> vinc_off;         // [V+1]   vertex incidences (slot = index)
  std::vector<int32_t> einc_off;         // [n_edges+1]
  std::vector<uint8_t> fcount;           // [n_faces] 1 or 2 hexahedra
  int64_t wedge_off = 0, wvert_off = 0, w_size = 0;
  std::vector<int32_t> owner;            // [n_global] local index of the first copy

  // faces and patches
  std::vector<int32_t> face_nbr;         // [E][6][2] (element, local face) or -1
  std::vector<int32_t> ip;               // [E][(N+3)^3] global id or -1
  // the nx = (N+3)^3 - (N+1)^3 patch slots outside the element: their ordinal
  // (xord[slot] >= 0, grouped by face plane, edge line and corner; inside:
  // -(local index) - 1; the device derives the slot of an ordinal in closed
  // form) and, per patch, where each
  // lands in the consumer layout [E][nx] of the element that holds it:
  // 6 face planes [(N+1)^2] at one layer in from that face (in-plane index
  // x_lo + (N+1) x_hi over the other two axes in increasing order), 12 edge
  // lines [N+1] at one layer in from both faces of the edge (edge id
  // 4 axis + side_lo + 2 side_hi, position along the axis), 8 corner points
  // (id = side_x + 2 side_y + 4 side_z); -1 where the slot is NULL
  int64_t nx = 0;
  std::vector<int32_t> xord;             // [(N+3)^3]
  std::vector<int32_t> xdest;            // [E][nx]

  // geometry
  std::vector<double> G;     // [E][6][(N+1)^3]
  std::vector<double> X8;    // [E][8][3] vertex coordinates in tensor corner order
  std::vector<double> mass;  // [E][(N+1)^3]
  std::vector<double> mN;    // [n_global]
  std::vector<double> xN;    // [n_global][3]
  std::vector<double> h;     // [E][3]
  std::vector<int32_t> order;  // element traversal order: Morton order of the centroids

  // coarse space (order-1 operator on the free vertices, nested-dissection order)
  std::vector<int32_t> cidx;             // [V] coarse index or -1 (Dirichlet vertex)
  int64_t nc = 0;                        // number of free vertices
  std::vector<int32_t> ac_off, ac_col;   // CSR of A_c in coarse order
  std::vector<double> ac_val;
  std::vector<FrontNode> fnodes;         // post-order
  std::vector<std::vector<int32_t>> fchildren;  // children of each node, ascending
  std::vector<int32_t> fb_idx;           // boundary lists
  std::vector<int32_t> ct_off, ct_pos;   // [nc + 1]: contribution slots subtracted from each row
  int64_t fwd_size = 0, bwd_size = 0, c_size = 0;
  int64_t ustack_size = 0;               // largest sum of pending update matrices (set-up)
  int32_t max_front = 0;                 // largest s + b
  int32_t n_heights = 0;
  std::vector<int32_t> fy_off, fy_items;  // per height: coarse rows of large nodes to assemble
  std::vector<int64_t> fr_off, br_off;    // per height: ranges of fr_items (large nodes) / br_items (all)
  // forward tiles of large nodes (rows r.. of [S^-1; W], s + b rows per node) and
  // backward tiles of every node (rows r.. of W^T, s per node): one workgroup
  // per tile, the tile shape chosen per height
  std::vector<RowItem> fr_items, br_items;
  std::vector<CoarseTileShape> fr_shape, br_shape;  // per height: tile shape of the forward / backward launch
  std::vector<int64_t> fs_off;            // per height: range of fs_items (small nodes)
  std::vector<RowItem> fs_items;          // 64-row chunks of small nodes' forward rows
  std::vector<double> corner_K;          // [E][8][8] order-1 element stiffness matrices
  std::vector<double> corner_M;          // [E][8] order-1 element mass (|J| at the corners, diagonal)
  std::vector<int64_t> coarse_vid;       // [E][8] global id of each element's corner vertices

  // coefficients of the model problem c u - div(kappa grad u) = s: constants,
  // or one value per element (kap_e, c_e non-empty; kappa, cmass are then NaN)
  double kappa = 1.0, cmass = 0.0;
  std::vector<double> kap_e, c_e;
};

// aggregation AMG hierarchy of the coarse system (sem_amg.cpp); level 0 holds
// the free vertices in ascending vertex id
struct AmgLevel {
  int64_t n = 0;
  std::vector<int32_t> off, col;  // CSR, columns ascending
  std::vector<double> val, diag;
  std::vector<int32_t> agg;       // [n] aggregate (row of the next level); empty on the coarsest
  std::vector<int32_t> moff, mem; // members of each aggregate, ascending
};

struct AmgHierarchy {
  std::vector<AmgLevel> levels;
  std::vector<double> coarse_inv;  // dense inverse of the coarsest matrix, row-major
  std::vector<int32_t> nd_of;      // level-0 unknown -> coarse (nested-dissection) index
};

void build_amg(const HostTables& T, AmgHierarchy& H);

// host set-up entry points (sem_setup.cpp)
void build_reference(HostTables& T, int N);
void build_numbering(HostTables& T, const int64_t* hex, int64_t n_hex, int64_t n_vtx);
void build_geometry(HostTables& T, const double* vtx, const int64_t* hex);
void build_patches(HostTables& T, const int64_t* hex);
void build_coarse_matrices(HostTables& T, const double* vtx, const int64_t* hex);
void build_coarse_tree(HostTables& T, int leaf_max = 0);
void assemble_coarse_matrix(HostTables& T);
void boundary_face_mass(const HostTables& T, const int64_t* faces, int64_t n_faces, double* ws);
void export_l2g(const HostTables& T, int32_t* l2g);
void update_interior_mask_flags(HostTables& T);
int64_t gid_of(const HostTables& T, int64_t e, int i, int j, int k);

}  // namespace sem
