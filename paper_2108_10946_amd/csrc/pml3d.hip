// The perfectly matched layer on tetrahedra (auxiliary p_x, p_y, p_z and omega):
// the terms the layer adds to the leapfrog of the acoustic wave equation, and the
// exact transpose of the coupled recursion for the adjoint, as per-cell and per-DOF
// kernels beside the stiffness apply.
//
// With nodal quadrature, (D_k)_ij = integral of phi_i dphi_j/dx_k reduces on a cell
// to w_i |det J| dphi_j/dx_k (x_i), so every PML operator is a per-cell
// reference-gradient contraction at the nodes:
//   (D_k v)_i      <- w_q (B g_v)_k        at node q of the cell, i = its DOF,
//   (D_k^T v_k)_j  <- sum_q sum_r D[q][j][r] (w_q B^T v_q)_r,
// with g_v the reference gradient of v at the node (sum_b D[q][b][.] v_b) and
// B = |det J| J^-T.  One thread per cell writes its cell-node values, each to its
// place in its DOF's contiguous range; one thread per DOF then sums its range in a
// fixed (cell, node) order (no atomics) and applies the update rows of the scheme.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "kmv_tables.inc"
#include "pml3d.hpp"

namespace kmv {
namespace {

// Damping coefficients at a DOF from sigma_x, sigma_y, sigma_z (component-major
// [3][n]): Psi_2^kk = sigma_k - sum_{j != k} sigma_j, Psi_3^kk = prod_{j != k}
// sigma_j, s = tr Psi_3, d1 = det Psi_1.
template <typename T>
struct Damp3 {
  T sg[3], p2[3], p3[3], tr, s, d1;
  __device__ Damp3(const T* sig, int64_t n, int64_t i) {
#pragma unroll
    for (int k = 0; k < 3; ++k) sg[k] = sig[k * n + i];
    tr = sg[0] + sg[1] + sg[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) p2[k] = T(2) * sg[k] - tr;
    p3[0] = sg[1] * sg[2];
    p3[1] = sg[0] * sg[2];
    p3[2] = sg[0] * sg[1];
    s = p3[0] + p3[1] + p3[2];
    d1 = sg[0] * sg[1] * sg[2];
  }
};

// w_q B g_v at every node q of the cell for the nodal values v, written to
// components c0..c0+2 at the node's slot pos[q].
template <typename T, int ND>
__device__ __forceinline__ void put_grads(const T (&v)[ND], const T (&B)[9], T* out, int64_t ns, int c0,
                                          const int32_t (&pos)[ND]) {
  using Tab = KmvTab<T, 3, ND>;
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    T g[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int b = 0; b < ND; ++b)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T dv = Tab::D[(q * ND + b) * 3 + r];
        if (dv != T(0)) g[r] += dv * v[b];
      }
    const T wq = Tab::W[q];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      out[(c0 + k) * ns + pos[q]] = wq * (B[3 * k] * g[0] + B[3 * k + 1] * g[1] + B[3 * k + 2] * g[2]);
  }
}

// Accumulate sum_r D[q][j][r] (w_q B^T v)_r into t[j] for the vector v at node q:
// node q's part of the cell's sum_k D_k^T v_k.
template <typename T, int ND>
__device__ __forceinline__ void add_div_t(int q, const T (&v)[3], const T (&B)[9], T (&t)[ND]) {
  using Tab = KmvTab<T, 3, ND>;
  const T wq = Tab::W[q];
  T z[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) z[r] = wq * (B[r] * v[0] + B[3 + r] * v[1] + B[6 + r] * v[2]);
#pragma unroll
  for (int j = 0; j < ND; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const T dv = Tab::D[(q * ND + j) * 3 + r];
      if (dv != T(0)) t[j] += dv * z[r];
    }
}

template <typename T, int ND>
__global__ void __launch_bounds__(256) k_pml3_cell_fwd(const Pml3CellArgs<T> A) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A.n_cells) return;
  const int64_t N = A.n_dofs, ns = A.n_cells * ND;
  int dof[ND];
  int32_t pos[ND];
  T B[9], v[ND];
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    dof[a] = A.cdof[a * A.n_cells + e];
    pos[a] = A.cpos[a * A.n_cells + e];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) B[k] = A.b3[k * A.n_cells + e];
#pragma unroll
  for (int a = 0; a < ND; ++a) v[a] = A.u[dof[a]];
  put_grads<T, ND>(v, B, A.out, ns, 0, pos);  // (D_k u^n)
#pragma unroll
  for (int a = 0; a < ND; ++a) v[a] = A.y[dof[a]];
  put_grads<T, ND>(v, B, A.out, ns, 3, pos);  // (D_k omega^n)
  T t[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) t[j] = T(0);
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    T pq[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) pq[k] = A.p[k * N + dof[q]];
    add_div_t<T, ND>(q, pq, B, t);  // sum_k D_k^T p_k^n
  }
#pragma unroll
  for (int q = 0; q < ND; ++q) A.out[6 * ns + pos[q]] = t[q];
}

template <typename T, int ND>
__global__ void __launch_bounds__(256) k_pml3_cell_adj(const Pml3CellArgs<T> A) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A.n_cells) return;
  const int64_t N = A.n_dofs, ns = A.n_cells * ND;
  int dof[ND];
  int32_t pos[ND];
  T B[9];
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    dof[a] = A.cdof[a * A.n_cells + e];
    pos[a] = A.cpos[a * A.n_cells + e];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) B[k] = A.b3[k * A.n_cells + e];
  {
    T l[ND];
#pragma unroll
    for (int a = 0; a < ND; ++a) l[a] = A.u[dof[a]];  // lambda^{m+1}
    put_grads<T, ND>(l, B, A.out, ns, 0, pos);          // (D_k lambda^{m+1})
  }
  {
    T t1[ND], t2[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) t1[j] = t2[j] = T(0);
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      const int i = dof[q];
      const Damp3<T> d(A.sig, N, i);
      const T c2 = A.c2[i];
      T vc[3], ve[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T mu = A.p[k * N + i];  // mu_k^{m+1}
        vc[k] = c2 * d.p2[k] * mu;
        ve[k] = c2 * d.p3[k] * mu;
      }
      add_div_t<T, ND>(q, vc, B, t1);  // sum_k D_k^T C_k mu_k
      add_div_t<T, ND>(q, ve, B, t2);  // sum_k D_k^T E_k mu_k
    }
#pragma unroll
    for (int q = 0; q < ND; ++q) {
      A.out[3 * ns + pos[q]] = t1[q];
      A.out[4 * ns + pos[q]] = t2[q];
    }
  }
  if (A.uf == nullptr) return;
  // gradient: the stiffness pairing w_q |det J| grad lambda . grad u^m at the node,
  // and (D_k u^m), (D_k omega^m) for the PML terms
  using Tab = KmvTab<T, 3, ND>;
  T G[6], v[ND], l[ND];
#pragma unroll
  for (int k = 0; k < 6; ++k) G[k] = A.geom[k * A.n_cells + e];
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    l[a] = A.u[dof[a]];
    v[a] = A.uf[dof[a]];
  }
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    T gl[3] = {T(0), T(0), T(0)}, gu[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int b = 0; b < ND; ++b)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T dv = Tab::D[(q * ND + b) * 3 + r];
        if (dv != T(0)) {
          gl[r] += dv * l[b];
          gu[r] += dv * v[b];
        }
      }
    const T v0 = G[0] * gu[0] + G[1] * gu[1] + G[2] * gu[2];
    const T v1 = G[1] * gu[0] + G[3] * gu[1] + G[4] * gu[2];
    const T v2 = G[2] * gu[0] + G[4] * gu[1] + G[5] * gu[2];
    A.out[5 * ns + pos[q]] = Tab::W[q] * (gl[0] * v0 + gl[1] * v1 + gl[2] * v2);
  }
  put_grads<T, ND>(v, B, A.out, ns, 6, pos);  // (D_k u^m)
#pragma unroll
  for (int a = 0; a < ND; ++a) v[a] = A.yf[dof[a]];
  put_grads<T, ND>(v, B, A.out, ns, 9, pos);  // (D_k omega^m)
}

// Sum of component c of DOF i's cell-node values, which the per-cell pass wrote to
// the DOF's own contiguous range [lo, hi), in ascending (cell, node) order.
template <typename T>
__device__ __forceinline__ T slot_sum(const T* x, int64_t ns, int c, int32_t lo, int32_t hi) {
  T y = T(0);
  for (int32_t k = lo; k < hi; ++k) y += x[c * ns + k];
  return y;
}

// Forward rows at DOF i (level n -> n+1):
//   (1+a) u^{n+1} = 2u^n - (1-a) u^{n-1} + dt^2/M (w_n s - K u^n - M s u^n - M d1 om^n - sum_k D_k^T p_k^n)
//   (1+b_k) p_k^{n+1} = (1-b_k) p_k^{n-1} - 2 dt/M c^2 (Psi_2^kk D_k u^n - Psi_3^kk D_k om^n)
//   om^{n+1} = om^n + dt (u^{n+1} + u^n)/2,    a = dt tr Psi_1 / 2, b_k = dt sigma_k.
template <typename T>
__global__ void __launch_bounds__(256) k_pml3_fwd_update(const Pml3UpdateArgs<T> A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_dofs) return;
  const int64_t N = A.n_dofs, ns = A.n_slots;
  const int32_t lo = A.csr_ptr[i], hi = A.csr_ptr[i + 1];
  T du[3], dy[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    du[k] = slot_sum(A.cell_out, ns, k, lo, hi);
    dy[k] = slot_sum(A.cell_out, ns, 3 + k, lo, hi);
  }
  const T dtp = slot_sum(A.cell_out, ns, 6, lo, hi);
  const Damp3<T> d(A.sig, N, i);
  const T M = A.mass[i], c2 = A.c2[i], dt = A.dt;
  const T a = T(0.5) * dt * d.tr;
  const T u = A.u[i], um = A.u_prev ? A.u_prev[i] : T(0), om = A.y[i];
  const T rhs = A.amp[0] * A.svec[i] - A.ku[i] - M * d.s * u - M * d.d1 * om - dtp;
  const T un = (T(2) * u - (T(1) - a) * um + dt * dt * rhs / M) / (T(1) + a);
  A.u_out[i] = un;
  A.y_out[i] = om + T(0.5) * dt * (un + u);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T b = dt * d.sg[k];
    A.p_io[k * N + i] = ((T(1) - b) * A.p_io[k * N + i] - T(2) * dt / M * c2 * (d.p2[k] * du[k] - d.p3[k] * dy[k])) /
                        (T(1) + b);
  }
}

// Reverse rows at DOF i (m = N_t .. 1), the exact transpose of the forward:
//   nu^m = nu^{m+1} - 2 dt d1 lam^{m+1} + 2 dt/M sum_k D_k^T E_k mu_k^{m+1}
//   (1+a) lam^m = 2 lam^{m+1} - (1-a) lam^{m+2} + (P^T y^m)/M + dt^2 (nu^m + nu^{m+1})/4
//                 - dt^2/M (K lam^{m+1} + M s lam^{m+1} + sum_k D_k^T C_k mu_k^{m+1})
//   (1+b_k) mu_k^m = (1-b_k) mu_k^{m+2} - 2 dt/M D_k lam^{m+1}
// and, at the paired steps, the float64 gradient accumulator gains the stiffness
// pairing plus sum_k mu_k^{m+1} (Psi_2^kk D_k u^m - Psi_3^kk D_k om^m).
template <typename T>
__global__ void __launch_bounds__(256) k_pml3_adj_update(const Pml3UpdateArgs<T> A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_dofs) return;
  const int64_t N = A.n_dofs, ns = A.n_slots;
  const int32_t lo = A.csr_ptr[i], hi = A.csr_ptr[i + 1];
  T dl[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) dl[k] = slot_sum(A.cell_out, ns, k, lo, hi);
  const T t1 = slot_sum(A.cell_out, ns, 3, lo, hi);
  const T t2 = slot_sum(A.cell_out, ns, 4, lo, hi);
  const Damp3<T> d(A.sig, N, i);
  const T M = A.mass[i], dt = A.dt;
  const T a = T(0.5) * dt * d.tr;
  const T l1 = A.u[i], l2 = A.u_prev[i], nu1 = A.y[i];
  const T nu = nu1 - T(2) * dt * d.d1 * l1 + T(2) * dt / M * t2;
  A.y_out[i] = nu;
  T rho = T(0);
  for (int32_t k = A.rec_ptr[i]; k < A.rec_ptr[i + 1]; ++k) rho += A.rec_w[k] * A.resid_row[A.rec_idx[k]];
  A.u_out[i] = (T(2) * l1 - (T(1) - a) * l2 + rho / M + T(0.25) * dt * dt * (nu + nu1) -
                dt * dt / M * (A.ku[i] + M * d.s * l1 + t1)) /
               (T(1) + a);
  T mu1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mu1[k] = A.p_in[k * N + i];
    const T b = dt * d.sg[k];
    A.p_io[k * N + i] = ((T(1) - b) * A.p_io[k * N + i] - T(2) * dt / M * dl[k]) / (T(1) + b);
  }
  if (A.gacc == nullptr) return;
  T g = slot_sum(A.cell_out, ns, 5, lo, hi);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T duk = slot_sum(A.cell_out, ns, 6 + k, lo, hi);
    const T dyk = slot_sum(A.cell_out, ns, 9 + k, lo, hi);
    g += mu1[k] * (d.p2[k] * duk - d.p3[k] * dyk);
  }
  A.gacc[i] += (double)g;
}

template <typename T, int ND>
hipError_t cell_t(bool adjoint, const Pml3CellArgs<T>& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.n_cells + 255) / 256);
  if (adjoint)
    hipLaunchKernelGGL((k_pml3_cell_adj<T, ND>), dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_pml3_cell_fwd<T, ND>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_pml3_cell(int nd, bool adjoint, const Pml3CellArgs<T>& a, hipStream_t s) {
  if (a.n_cells <= 0) return hipSuccess;
  switch (nd) {
    case 4: return cell_t<T, 4>(adjoint, a, s);
    case 15: return cell_t<T, 15>(adjoint, a, s);
    case 32: return cell_t<T, 32>(adjoint, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_pml3_update(bool adjoint, const Pml3UpdateArgs<T>& a, hipStream_t s) {
  if (a.n_dofs <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((a.n_dofs + 255) / 256);
  if (adjoint)
    hipLaunchKernelGGL((k_pml3_adj_update<T>), dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_pml3_fwd_update<T>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_pml3_cell<float>(int, bool, const Pml3CellArgs<float>&, hipStream_t);
template hipError_t launch_pml3_cell<double>(int, bool, const Pml3CellArgs<double>&, hipStream_t);
template hipError_t launch_pml3_update<float>(bool, const Pml3UpdateArgs<float>&, hipStream_t);
template hipError_t launch_pml3_update<double>(bool, const Pml3UpdateArgs<double>&, hipStream_t);

}  // namespace kmv
