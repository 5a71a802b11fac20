// Device kernels of the KMV hot path and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kmv {

constexpr int kColStride = 65;  // colour_start row stride (max colours + 1)
constexpr int kRefStride = 2;   // inline partial slots per shared ref

// Arguments of the fused step kernel.  One workgroup processes one patch of cells
// per time step:
//   1. it finishes the DOFs it shares with other patches for the current level:
//      their K u of the previous step is the fixed-order sum of the patches'
//      partials, and every touching patch repeats the same arithmetic, so all
//      copies agree bit for bit; the first touching patch stores the result;
//   2. it stages the patch's values in LDS (owned DOFs are a contiguous range);
//   3. it samples the receivers whose cell lies in the patch;
//   4. it applies the element stiffness of its cells; each cell writes its own
//      LDS slots and each DOF sums its slots in a fixed order (deterministic);
//   5. it adds the point sources of the DOFs it is designated for;
//   6. it finishes the leapfrog update (or writes y = K u) of the DOFs only it
//      touches and writes its partial sums of the shared ones.
// The adjoint variant also gathers the forward state u^m and accumulates the
// gradient pairing in float64.
template <typename T>
struct StepArgs {
  // mesh
  const uint16_t* lmap;        // [nd * n_cells] patch-local DOF of node a of cell e
  const T* geom;               // [ng * n_cells] |det J| J^-1 J^-T (upper triangle)
  const int32_t* cell_start;   // [np+1]
  const int32_t* own_start;    // [np+1]
  const int32_t* sh_start;     // [np+1]
  const int32_t* sh_idx;       // [n_shared_refs] global id of each shared ref
  const uint16_t* gl_ptr;      // gather pointers per patch (16-byte aligned regions)
  const uint16_t* gl_ent;      // gather entries per patch (16-byte aligned regions)
  const int32_t* gl_ptr_off;   // [np+1]
  const int32_t* gl_ent_off;   // [np+1]
  const int32_t* shp_ptr;      // [n_shared+1] partial slots of each shared DOF
  const int32_t* shp_slot;     // [n_shared_refs], in patch order
  const int32_t* ref_slots;    // [n_shared_refs*kRefStride] the same lists per ref, -1 padded
  int64_t n_cells, n_own;
  int nloc_max, cells_max;     // LDS sizing
  int mode;                    // 0: leapfrog step, 1: y = K u
  int prev;                    // 1: shared DOFs of this level are finished here
  // state (level n -> n+1; the adjoint runs the same recursion backwards)
  const T* u_in;               // level n: owned entries (and shared ones if !prev)
  T* u_in_sh;                  // same buffer: finished shared entries are stored here
  const T* u_prev;             // level n-1: shared entries
  T* u_out;                    // level n+1: owned entries
  T* du;                       // owned increments, updated in place
  const T* dsh_prev;           // [n_shared] shared increments of level n-1
  T* dsh_cur;                  // [n_shared] shared increments of level n
  const T* part_prev;          // [n_shared_refs] partial K u of the previous step
  T* part_cur;                 // [n_shared_refs] partial K u of this step
  const T* c2;                 // c^2 at the DOFs
  const T* gamma;              // dt^2 / (M (1+a))
  const T* beta;               // (1-a)/(1+a), or nullptr (no damping)
  const int32_t* damp_patch;   // [np] 1 if a DOF of the patch is damped (beta read only there)
  T* y_out;                    // mode 1
  // point injection: groups of entries per patch, one group per local DOF
  const int32_t* grp_ptr;      // [np+1] or nullptr
  const int32_t* grp_local;
  const int32_t* grp_eptr;
  const int32_t* ent_pt;       // amplitude index of each entry
  const T* ent_w;              // phi_a(x_point)
  const T* amp;                // amplitudes (wavelet sample or adjoint data row)
  T amp_scale;
  // receivers sampled from LDS (level n), per patch
  const int32_t* rp_ptr;       // [np+1]
  const int32_t* rp_rec;       // receiver index
  const uint16_t* rp_loc;      // [n*nd] patch-local DOFs
  const T* rp_w;               // [n*nd] phi_a(x_r)
  T* trace_row;                // d^n row, or nullptr
  // adjoint + gradient
  const T* uf;                 // forward state u^m
  const T* partr_prev;         // pairing partials of the previous step
  T* partr_cur;
  double* gacc;                // [n_dofs] float64 gradient accumulator
};

// Finisher: the shared DOFs of a level from the last step's partials (end of a
// sweep, checkpoints, segment ends), or y = K u for them (mode 1).
template <typename T>
struct FinishArgs {
  int64_t n_own, n_shared;
  const int32_t* shp_ptr;
  const int32_t* shp_slot;
  int mode;
  const T* part_prev;
  const T* u_prev;
  T* u_cur;
  const T* dsh_prev;
  T* dsh_cur;
  const T* gamma;
  const T* beta;
  T* y_out;
  const T* partr_prev;
  double* gacc;
};

template <typename T>
// e0/e1: optional events recorded by the dispatch itself at kernel start and end.
hipError_t launch_step(int dim, int nd, bool adjoint, const StepArgs<T>& a, int n_patches, int block,
                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Dynamic LDS bytes of one k_step workgroup.
size_t step_lds_bytes(int nloc_max, int cells_max, int nd, size_t elem_size);
template <typename T>
hipError_t launch_finish(bool adjoint, const FinishArgs<T>& a, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_sample(const T* u, const int32_t* dof, const T* w, int npts, int nd, T* out,
                         hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <typename T>
hipError_t launch_square(const double* c, T* c2, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* x, T v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* x, double v, int64_t n, hipStream_t s);
// r = obs - d (element type T), J = 1/2 sum r^2 in float64 (fixed order) at *J_out.
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
hipError_t launch_normalize(T* v, const T* w, const double* dot_ww, int64_t n, hipStream_t s);
template <typename T>
hipError_t set_step_lds_limit(int dim, int nd, bool adjoint, int bytes);

}  // namespace kmv
