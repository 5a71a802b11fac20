// Device kernels of the KMV hot path and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kmv {

constexpr int kRefStride = 2;          // inline partial slots per shared ref
constexpr uint32_t kGatherList = 0xFFFFu;  // high half of a gather word that points into a list

// Arguments of the fused step kernel.  One workgroup processes one patch of cells
// per time step, one thread per cell:
//   1. it finishes the DOFs it shares with other patches for the current level:
//      their K u of the previous step is the fixed-order sum of the patches'
//      partials, and every touching patch repeats the same arithmetic, so all
//      copies agree bit for bit; the first touching patch stores the result;
//   2. it stages the level of the patch's non-interior DOFs in LDS (the owned
//      ones are a contiguous range); each thread loads its cell's interior DOFs
//      straight into registers;
//   3. each thread samples the receivers in its cell, applies its element
//      stiffness, subtracts the point sources in its cell and finishes its
//      interior DOFs (leapfrog update, or y = K u);
//   4. the non-interior contributions go to per-cell LDS slots and each DOF sums
//      its slots in a fixed order (deterministic); owned DOFs are updated, shared
//      ones write this patch's partial sum.
// The adjoint variant also stages the forward state u^m and accumulates the
// gradient pairing in float64.
template <typename T>
struct StepArgs {
  // mesh
  const uint32_t* lmap;        // [ceil(nb/2) * n_cells] local non-interior DOFs of nodes 2q, 2q+1 of cell e
  const T* geom;               // [ng * n_cells] |det J| J^-1 J^-T (upper triangle)
  const T* gdet;               // [n_cells] dt^2 / |det J|
  const int32_t* cell_start;   // [np+1]
  const int32_t* own_start;    // [np+1] interior DOFs, then the other owned DOFs
  const int32_t* sh_start;     // [np+1]
  const int32_t* sh_idx;       // [n_shared_refs + 1] global id of each shared ref (+ padding)
  const uint32_t* gword;       // gather word per local non-interior DOF, per patch
  const int32_t* gword_off;    // [np+1]
  const uint16_t* glist;       // gather lists of DOFs with more than two slots (8-aligned regions, + 8 padding)
  const int32_t* glist_off;    // [np+1]
  const int32_t* shp_ptr;      // [n_shared+1] partial slots of each shared DOF
  const int32_t* shp_slot;     // [n_shared_refs], in patch order
  const int32_t* ref_slots;    // [(n_shared_refs+1)*kRefStride] {first, second} or {first, -count}
  int64_t n_cells, n_own, n_dofs;
  int nbl_max, slot_stride, glist_max;  // LDS sizing; cell-node slot = b*slot_stride + t
  int mode;                    // 0: leapfrog step, 1: y = K u
  int prev;                    // 1: shared DOFs of this level are finished here
  int pair_prev;               // adjoint: 1 if the previous launch's pairing partials are finished here
                               // (0 when a separate pass finishes them, as with gradient subsampling)
  // state (level n -> n+1; the adjoint runs the same recursion backwards).  A
  // level vector holds the n_dofs DOF values, then one copy per shared ref of its
  // DOF's value (index n_dofs + r), kept by the patch of ref r.
  const T* u_in;               // level n (apply mode: a plain n_dofs vector)
  T* u_in_sh;                  // same buffer: finished shared entries are stored here
  const T* u_prev;             // level n-1 (its shared-ref copies are read)
  T* u_out;                    // level n+1: owned entries
  T* du;                       // owned increments, updated in place
  const T* dsh_prev;           // [n_shared_refs] increment of each ref's DOF, level n-1
  T* dsh_cur;                  // [n_shared_refs] the same, level n
  const T* part_prev;          // [n_shared_refs] partial K u of each ref, previous step
  T* part_cur;                 // [n_shared_refs] partial K u of each ref, this step
  const T* c2;                 // c^2 at the DOFs
  const T* c2_ref;             // [n_shared_refs] c^2 at each ref's DOF
  const T* gamma;              // dt^2 / (M (1+a)) (read for non-interior DOFs)
  const T* gamma_ref;          // [n_shared_refs]
  const T* beta;               // (1-a)/(1+a), or nullptr (no damping)
  const T* beta_ref;           // [n_shared_refs], or nullptr
  const int32_t* damp_patch;   // [np] 1 if a DOF of the patch is damped (beta read only there)
  T* y_out;                    // mode 1
  // point sources: entries (cell, point, phi_a(x_point) per node) per patch
  const int32_t* inj_ptr;      // [np+1] or nullptr
  const int32_t* inj_cell;     // patch-local cell of the entry
  const int32_t* inj_pt;       // point index
  const T* inj_w;              // [n*nd]
  const T* amp;                // amplitude of point j: amp[j * amp_stride]
  int amp_stride;
  T amp_scale;
  // receivers sampled from level n, entries as for the sources
  const int32_t* rec_ptr;
  const int32_t* rec_cell;
  const int32_t* rec_pt;
  const T* rec_w;
  T* trace_row;                // d^n row, or nullptr
  // adjoint + gradient
  const T* uf;                 // forward state u^m (a level vector)
  const T* partr_prev;         // pairing partials of the previous step
  T* partr_cur;
  double* gacc;                // [n_dofs] float64 gradient accumulator
  // shots stepped together: the launch has n_patches * n_shots workgroups, work
  // item i being (patch i / n_shots, shot i % n_shots).  Every per-shot buffer of
  // shot s starts s times its stride after shot 0's; mesh tables and coefficients
  // are shared.  A stride of 0 shares the buffer between shots.
  int n_shots;                 // >= 1 (1 in apply mode)
  int64_t ss_level;            // u_in, u_in_sh, u_prev, u_out, uf
  int64_t ss_dof;              // du, gacc
  int64_t ss_ref;              // dsh_prev, dsh_cur, part_prev, part_cur, partr_prev, partr_cur
  int64_t ss_amp;              // amp
  int64_t ss_trace;            // trace_row
  int64_t ss_inj;              // inj_ptr (a [np+1] block per shot, or shared)
  // work items: patch_list[i] is the patch of item i (nullptr: item i is patch i)
  const int32_t* patch_list;
  // PML (2D, the k_step<..., PML = true> instances, launched on the patches with a
  // DOF in the layer)
  const T* pml_b;              // [4 * n_cells] B_e = |det J_e| J_e^-T, entry (k, r) at (2k + r) * n_cells + e
  const T* sig;                // [2 * n_dofs] sigma_x then sigma_z at the DOFs
  const T* sig_ref;            // [2 * n_shared_refs] the same at each shared ref
  const T* pp_in;              // auxiliary level n: [2][ls] (component k at k * ls), DOF values then ref copies
  T* pp_in_sh;                 // same buffer: finished shared entries are stored here
  T* pp_io;                    // auxiliary level n-1, overwritten by level n+1 (owned DOFs)
  const T* pt_prev;            // [2][rs] partial sums of the gradient term t of the previous step
  T* pt_cur;                   // [2][rs] this step's
  int64_t pml_ls, pml_rs;      // component strides of pp_* (ls) and pt_* (rs)
  int64_t ss_pml, ss_pt;       // per-shot strides (2 ls, 2 rs)
  T pml_dt, inv_dt;            // dt, 1 / dt
  int pml_trans;               // 1: the transposed (adjoint) PML couplings, with or without the gradient pairing
};

// Finisher: the shared DOFs of a level from the last step's partials (end of a
// sweep, checkpoints, segment ends), or y = K u for them (mode 1), or (adjoint,
// mode 2) only the gradient pairing partials of the last step, added to the
// accumulators of the shared DOFs.
template <typename T>
struct FinishArgs {
  int64_t n_own, n_shared, n_dofs;
  const int32_t* shp_ptr;
  const int32_t* shp_slot;
  int mode;
  const T* part_prev;
  const T* u_prev;             // level vectors (shared-ref copies after n_dofs)
  T* u_cur;
  const T* dsh_prev;           // per shared ref
  T* dsh_cur;
  const T* gamma;
  const T* beta;
  T* y_out;
  const T* partr_prev;
  double* gacc;
  // shots: blockIdx.y; per-shot strides as in StepArgs
  int n_shots;
  int64_t ss_level, ss_dof, ss_ref;
};

// e0/e1: optional events recorded by the dispatch itself at kernel start and end.
// n_items: patches in the launch (a.patch_list's length when it is set).  pml:
// the PML instance (2D only).
template <typename T>
hipError_t launch_step(int dim, int nd, bool adjoint, const StepArgs<T>& a, int n_items, int block,
                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, bool pml = false);
// Threads per workgroup of k_step for patches of up to max_patch_cells cells (one
// thread per cell, whole wavefronts).
int step_block(int max_patch_cells);
// Shared refs a k_step workgroup of `block` threads finishes in its first batch of
// loads; a patch with more goes through the loop over the remaining refs.
int step_first_batch_refs(int dim, int nd, bool adjoint, int block);
// Dynamic LDS bytes of one k_step workgroup.
size_t step_lds_bytes(int dim, int nd, int nbl_max, int slot_stride, int nb, int glist_max, bool adjoint,
                      size_t elem_size, bool pml = false);
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
hipError_t launch_fill_i32(int* x, int v, int64_t n, hipStream_t s);
// r = obs - d (element type T), J = 1/2 sum r^2 in float64 (fixed order) at *J_out.
template <typename T>
hipError_t launch_misfit(const T* d, const T* obs, T* resid, int64_t n, double* scratch,
                         int nblocks, double* J_out, hipStream_t s);
// g = scale * c * sum_s gacc[s*n + i], shots summed in order; with accumulate the
// result is added to g instead of replacing it
hipError_t launch_finalize_grad(const double* c, const double* gacc, int n_shots, double scale, double* g,
                                int64_t n, hipStream_t s, bool accumulate = false);
// Non-finite sentinel: sets *flag = 1 if any of x[v*stride + i], i < n, v < nvec is
// NaN or infinite (flag untouched otherwise).
template <typename T>
hipError_t launch_check_finite(const T* x, int64_t n, int64_t stride, int nvec, int* flag, hipStream_t s);
// out[r] = x[idx[r]], r < n (per-ref copies of a DOF vector)
template <typename T>
hipError_t launch_gather(const T* x, const int32_t* idx, T* out, int64_t n, hipStream_t s);
// power iteration helpers
template <typename T>
hipError_t launch_scale(const T* x, const T* s, T* y, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_dot(const T* x, const T* y, int64_t n, double* scratch, int nblocks,
                      double* out, hipStream_t s);
template <typename T>
hipError_t launch_normalize(T* v, const T* w, const double* dot_ww, int64_t n, hipStream_t s);
template <typename T>
hipError_t set_step_lds_limit(int dim, int nd, bool adjoint, int bytes, bool pml = false);

}  // namespace kmv
