// KMV reference element tables for the GPU path (host side).
#pragma once
#include <array>
#include <vector>

namespace kmv {

// Where a reference node sits: on a vertex, an edge, a face (3D) or inside.
enum Entity { ENT_VERTEX = 0, ENT_EDGE = 1, ENT_FACE = 2, ENT_CELL = 3 };

struct Element {
  int dim = 0, degree = 0, n = 0;  // n = nodes per cell (= quadrature points)
  std::vector<double> nodes;       // [n*dim] reference coordinates
  std::vector<double> bary;        // [n*(dim+1)] barycentric coordinates
  std::vector<double> weights;     // [n] nodal quadrature weights
  std::vector<double> grads;       // [(q*n + a)*dim + r] d phi_a / d xi_r at node q
  std::vector<int> entity;         // [n] Entity of each node
  std::vector<int> entity_id;      // [n] local vertex / edge / face id (cell: 0)
  int n_vertex = 0, n_edge = 0, n_face = 0, n_cell = 0;  // nodes per entity
  // basis evaluation at arbitrary reference points
  void eval(const double* xi, double* phi) const;
  // internals: coefficients of the nodal basis in the spanning polynomials
  std::vector<std::vector<long double>> span_polys;  // dense monomial coefficients
  std::vector<std::array<int, 3>> mono;              // exponent of each monomial
  std::vector<long double> coef;                     // [j*n + a]
};

// Build (and cache) the element.  Throws std::invalid_argument on an unsupported
// (dim, degree).
const Element& element(int dim, int degree);
bool element_supported(int dim, int degree);

}  // namespace kmv
