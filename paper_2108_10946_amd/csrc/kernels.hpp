// Device kernels of the KMV hot path and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kmv {

constexpr int kColStride = 65;  // colour_start row stride (max colours + 1)

// Arguments of the patch kernel.  One workgroup processes one patch of cells:
// it stages the patch's DOF values in LDS, applies the element stiffness of every
// cell, scatters colour by colour (no two cells of a colour share a DOF), adds the
// point-source terms of the DOFs it owns, then either finishes the leapfrog update
// of the DOFs no other patch touches or writes y = K u for them, and writes its
// partial sums for DOFs shared with other patches.
template <typename T>
struct PatchArgs {
  const uint16_t* lmap;        // [nd * n_cells] patch-local DOF of node a of cell e
  const T* geom;               // [n_cells * gstride] |det J| J^-1 J^-T (upper triangle)
  const T* D;                  // [nd*nd*dim] reference gradients at the nodes
  const T* W;                  // [nd] nodal quadrature weights
  const int32_t* cell_start;   // [np+1]
  const int32_t* own_start;    // [np+1]
  const int32_t* sh_start;     // [np+1]
  const int32_t* sh_idx;       // [n_shared_refs] global id of each shared ref
  const int32_t* colour_start; // [np*kColStride]
  const int32_t* ncol;         // [np]
  int64_t n_cells;
  int nloc_max;                // LDS array stride
  int mode;                    // 0: leapfrog step, 1: y = K u
  const T* u_in;               // u^n (or lambda^{m+1})
  T* u_out;                    // u^{n+1} (or lambda^m)
  T* du;                       // increment, updated in place
  const T* c2;                 // c^2 at the DOFs
  const T* gamma;              // dt^2 / (M (1+a))
  const T* beta;               // (1-a)/(1+a), or nullptr (no damping)
  T* partial;                  // [n_shared_refs] partial K u of shared DOFs
  T* y_out;                    // mode 1: K u
  // point injection: groups of entries per patch, one group per local DOF
  const int32_t* grp_ptr;      // [np+1] or nullptr
  const int32_t* grp_local;    // [n_groups]
  const int32_t* grp_eptr;     // [n_groups+1]
  const int32_t* ent_pt;       // [n_entries] amplitude index
  const T* ent_w;              // [n_entries] phi_a(x_point)
  const T* amp;                // amplitudes (wavelet sample or adjoint data row)
  T amp_scale;
  // adjoint + gradient
  const T* uf;                 // forward state u^m
  T* partial_r;                // [n_shared_refs] partial gradient pairing
  double* gacc;                // [n_dofs] float64 gradient accumulator
};

template <typename T>
struct SharedArgs {
  int64_t n_own, n_shared;
  const int32_t* shp_ptr;
  const int32_t* shp_slot;
  int mode;
  const T* partial;
  const T* u_in;
  T* u_out;
  T* du;
  const T* gamma;
  const T* beta;
  T* y_out;
  const T* partial_r;
  double* gacc;
};

// Launchers (return hipError_t of the launch).
template <typename T>
hipError_t launch_patch(int dim, int nd, bool adjoint, const PatchArgs<T>& a, int n_patches,
                        int block, hipStream_t s);
template <typename T>
hipError_t launch_shared(bool adjoint, const SharedArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_sample(const T* u, const int32_t* dof, const T* w, int npts, int nd, T* out,
                         hipStream_t s);
template <typename T>
hipError_t launch_square(const double* c, T* c2, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* x, T v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* x, double v, int64_t n, hipStream_t s);
// r = obs - d (element type T), J partial sums in float64 (deterministic order);
// final J at *J_out (device).
template <typename T>
hipError_t launch_misfit(const T* d, const T* obs, T* resid, int64_t n, double* scratch,
                         int nblocks, double* J_out, hipStream_t s);
hipError_t launch_finalize_grad(const double* c, const double* gacc, double scale, double* g,
                                int64_t n, hipStream_t s);
// power iteration helpers
template <typename T>
hipError_t launch_scale(const T* x, const T* s, T* y, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_dot(const T* x, const T* y, int64_t n, double* scratch, int nblocks,
                      double* out, hipStream_t s);
template <typename T>
hipError_t launch_axpby_norm(T* v, const T* w, const double* dot_ww, int64_t n, hipStream_t s);
template <typename T>
hipError_t set_patch_lds_limit(int dim, int nd, bool adjoint, int bytes);

}  // namespace kmv
