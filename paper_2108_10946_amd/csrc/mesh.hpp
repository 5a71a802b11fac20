// Mesh preprocessing for the patch-scheduled GPU kernels (host side).
#pragma once
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "element.hpp"

namespace kmv {

constexpr int kMaxShare = 2;  // inline partial slots per shared ref (DOFs on one patch interface)
constexpr uint32_t kListMark = 0xFFFFu;  // high half of a gather word that points into a list

// A point inside the mesh: containing (internal) cell and basis weights.
struct PointLoc {
  int64_t cell;              // internal cell index
  std::vector<double> phi;   // [nd] phi_a(xi)
};

struct Mesh {
  int dim = 0, degree = 0, nd = 0, ng = 0;  // ng: geometry entries per cell (3 / 6)
  const Element* el = nullptr;
  int64_t n_vertices = 0, n_cells = 0, n_dofs = 0;
  std::vector<double> coords;        // [n_vertices*dim]
  std::vector<int32_t> cells_in;     // [n_cells*(dim+1)], input order
  // internal cell order (patch-major, recursive-bisection order inside a patch)
  std::vector<int64_t> cell_input;   // internal -> input cell id
  std::vector<int64_t> cell_dofs;    // [n_cells*nd] internal order, final DOF ids
  std::vector<double> x0;            // [n_cells*dim] first vertex (internal order)
  std::vector<double> jac;           // [n_cells*dim*dim] J (row-major [i][r])
  std::vector<double> jinv;          // [n_cells*dim*dim] J^-1 (row-major [r][i])
  std::vector<double> absdet;        // [n_cells]
  std::vector<double> geom;          // [n_cells*ng] |det J| J^-1 J^-T, upper triangle
  std::vector<double> dof_coords;    // [n_dofs*dim]
  std::vector<double> mass;          // [n_dofs]
  // node classes: interior nodes (the DOF belongs to that cell alone) and the
  // rest, each in ascending local-node order
  int ni = 0, nb = 0;
  std::vector<int> int_nodes, bnd_nodes;
  // patches.  The DOFs touched by one patch only ("owned") come first, patch by
  // patch: the patch's interior DOFs, interior node j of its t-th cell at
  // own_start + j*nc + t (nc cells in the patch), then its other owned DOFs.
  // DOFs touched by several patches ("shared") follow all owned ones.
  int patch_cells = 0;
  int64_t n_patches = 0, n_own_total = 0, n_shared = 0, n_shared_refs = 0;
  int max_nbl = 0, max_patch_cells = 0;
  std::vector<int32_t> patch_cell_start;  // [n_patches+1]
  std::vector<int32_t> patch_own_start;   // [n_patches+1]
  std::vector<int32_t> patch_sh_start;    // [n_patches+1] into sh_idx / partial slots
  std::vector<int32_t> sh_idx;            // [n_shared_refs] global DOF id
  std::vector<int32_t> shp_ptr;           // [n_shared+1]
  std::vector<int32_t> shp_slot;          // [n_shared_refs]
  // per shared ref: {first slot (the designated patch's), second slot} when two
  // patches touch the DOF, else {first slot, -count} (walk the CSR list)
  std::vector<int32_t> ref_slots;         // [n_shared_refs*kMaxShare]
  int max_share = 0;                      // most patches touching one DOF
  // Patch-local numbering of the non-interior DOFs: the owned ones in global
  // order (0..nbo-1), then the patch's shared refs (nbo + j).
  std::vector<uint16_t> lmap;             // [nb*n_cells] SoA: local DOF of non-interior node b of cell e
  // Cell-node slots: non-interior node b of the patch's t-th cell writes slot
  // b*slot_stride + t; slot nb*slot_stride holds zero.  Gather word of a local
  // DOF: s0 | s1 << 16 for one or two contributions (s1 = the zero slot for one),
  // or off | kListMark << 16 for more: glist[off] = count, then the slots.
  int slot_stride = 0;
  std::vector<uint32_t> gword;            // per patch, per local non-interior DOF
  std::vector<int32_t> gword_off;         // [n_patches+1]
  std::vector<uint16_t> glist;            // per patch, 8-entry aligned regions
  std::vector<int32_t> glist_off;         // [n_patches+1]
  int max_glist = 0;                      // longest per-patch glist region
  // point location grid
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int grid_n[3] = {1, 1, 1};
  std::vector<int64_t> grid_ptr, grid_cells;

  // boundary mass, computed on first use (see boundary_of); shared by the problems
  // and server requests on this mesh
  mutable std::once_flag bnd_once;
  mutable std::vector<int32_t> bnd_dof;
  mutable std::vector<double> bnd_b;

  // Find the cell containing x (barycentric >= -tol, lowest input id among ties).
  // Returns false if none.
  bool locate(const double* x, PointLoc& out) const;
};

// Build; throws std::invalid_argument (bad input), kmv::MeshError (bad mesh).
struct MeshError {
  const char* what;
};
Mesh* build_mesh(int dim, int degree, const double* coords, int64_t nv, const int32_t* cells,
                 int64_t ne, int patch_cells);

// Boundary mass of the absorbing boundary term (the boundary integral of
// c phi_i phi_j in the damping matrix M_{u,1} of the appendix, lumped by rows with c
// at node i): b_i = integral over the mesh boundary of phi_i, for the DOFs where it
// is not zero.  Facets (edges / triangles) that belong to one cell are the
// boundary; on each, the cell's basis is integrated by Gauss quadrature.
void boundary_weights(const Mesh& m, std::vector<int32_t>& dofs, std::vector<double>& b);
// The mesh's boundary DOFs and b_i, computed once (thread-safe) and kept with it.
void boundary_of(const Mesh& m, const std::vector<int32_t>** dofs, const std::vector<double>** b);

// Row sums of |K(c)| divided by M (Gershgorin radii of M^-1 K).
double gershgorin_rho(const Mesh& m, const double* c);

// Check the invariants the kernels rely on; false with a reason on violation.
bool validate_mesh(const Mesh& m, std::string& why);

}  // namespace kmv
