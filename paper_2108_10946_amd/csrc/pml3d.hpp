// The perfectly matched layer on tetrahedra: per-cell contractions and per-DOF
// update rows (pml3d.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kmv {

// Per-cell pass.  Forward: u = u^n, y = omega^n, p = p^n ([3][n_dofs]); writes
// components 0-2 (D_k u), 3-5 (D_k omega), 6 (sum_k D_k^T p_k).  Adjoint: u =
// lambda^{m+1}, p = mu^{m+1}, c2, sig; writes 0-2 (D_k lambda), 3 (sum_k D_k^T C_k
// mu_k), 4 (sum_k D_k^T E_k mu_k) and, when uf (u^m) is set, 5 (the stiffness
// pairing of lambda^{m+1} with u^m), 6-8 (D_k u^m), 9-11 (D_k omega^m, yf).
// out: [component][n_cells*nd]; node q of cell e writes to place cpos[q*n_cells + e],
// inside its DOF's range of the per-DOF pass.
template <typename T>
struct Pml3CellArgs {
  int64_t n_cells = 0, n_dofs = 0;
  const int32_t* cdof = nullptr;  // [nd][n_cells] DOF of node q of cell e
  const int32_t* cpos = nullptr;  // [nd][n_cells] its place in out
  const T* b3 = nullptr;          // [9][n_cells] |det J| J^-T, entry (k, r) at 3k + r
  const T* geom = nullptr;        // [6][n_cells] |det J| J^-1 J^-T, upper triangle
  const T* u = nullptr;
  const T* y = nullptr;
  const T* p = nullptr;
  const T* c2 = nullptr;
  const T* sig = nullptr;  // [3][n_dofs] sigma_x, sigma_y, sigma_z
  const T* uf = nullptr;
  const T* yf = nullptr;
  T* out = nullptr;
};

// Per-DOF pass: sums DOF i's cell-node values (places csr_ptr[i] .. csr_ptr[i+1] of
// each component, ascending (cell, node)) and applies the update rows.
// Forward: u = u^n, u_prev = u^{n-1} (NULL: zero), y = omega^n, p_io = p^{n-1} in,
// p^{n+1} out; u_out = u^{n+1}, y_out = omega^{n+1}; amp = w(t_n) (one value),
// svec = the source's nodal load vector.  Adjoint: u = lambda^{m+1}, u_prev =
// lambda^{m+2} in, lambda^m out (u_out may alias it), y = nu^{m+1}, y_out = nu^m,
// p_in = mu^{m+1}, p_io = mu^{m+2} in, mu^m out; resid_row = y^m per receiver with
// the transposed receiver rows rec_ptr / rec_idx / rec_w; gacc (float64, NULL: no
// pairing at this step).
template <typename T>
struct Pml3UpdateArgs {
  int64_t n_dofs = 0, n_slots = 0;
  const int32_t* csr_ptr = nullptr;
  const T* cell_out = nullptr;
  const T* sig = nullptr;
  const T* mass = nullptr;
  const T* c2 = nullptr;
  T dt = 0;
  const T* ku = nullptr;  // K(c) u^n or K(c) lambda^{m+1}
  const T* u = nullptr;
  const T* u_prev = nullptr;
  const T* y = nullptr;
  T* u_out = nullptr;
  T* y_out = nullptr;
  const T* p_in = nullptr;
  T* p_io = nullptr;
  const T* amp = nullptr;
  const T* svec = nullptr;
  const int32_t* rec_ptr = nullptr;
  const int32_t* rec_idx = nullptr;
  const T* rec_w = nullptr;
  const T* resid_row = nullptr;
  double* gacc = nullptr;
};

template <typename T>
hipError_t launch_pml3_cell(int nd, bool adjoint, const Pml3CellArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_pml3_update(bool adjoint, const Pml3UpdateArgs<T>& a, hipStream_t s);

}  // namespace kmv
