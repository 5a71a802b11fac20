// Device-side problem state and the forward / adjoint / gradient drivers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mesh.hpp"

namespace kmv {

struct Status {
  int code;
  std::string msg;
};

// Stream for the device allocations of problems created or destroyed on this
// thread (nullptr: plain hipMalloc / hipFree).  Set by the server's workers.
hipStream_t alloc_stream();
struct AllocStreamScope {
  explicit AllocStreamScope(hipStream_t s);
  ~AllocStreamScope();
  hipStream_t prev;
};

// Point tables on the device: per patch, the entries (patch-local cell, point
// index, phi_a(x_point) per node) of the points whose cell lies in the patch, used
// for injection and for sampling inside k_step; and global sampling rows (DOF
// ids and weights) for k_sample.
struct PointTables {
  int npts = 0;                 // all points (shot-major when the table is per shot)
  int64_t shot_stride = 0;      // np+1 when each shot has its own pp_ptr block, else 0
  int32_t* pp_ptr = nullptr;    // [np+1]
  int32_t* pp_cell = nullptr;   // patch-local cell
  int32_t* pp_pt = nullptr;     // point index
  void* pp_w = nullptr;         // [n*nd]
  int32_t* s_dof = nullptr;     // [npts*nd] global DOFs
  void* s_w = nullptr;          // [npts*nd]
  std::vector<int32_t> h_dof;   // host copies of s_dof, s_w
  std::vector<double> h_w;
};

// Event-based timing of sampled kernel launches (see kmv_profile_enable).
struct Probe {
  static constexpr int kVariants = 5;
  int every = 0;
  int64_t launches[kVariants] = {0, 0, 0, 0, 0};
  int64_t timed[kVariants] = {0, 0, 0, 0, 0};
  double total_ms[kVariants] = {0, 0, 0, 0, 0};
  struct Pending {
    int variant;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};

// Lagged state of one sweep: owned increments, the shared-ref increments of the
// two most recent levels and the partial sums of the two most recent steps.
struct Sweep {
  void* d = nullptr;                    // [n_dofs] owned increments
  void* dsh[2] = {nullptr, nullptr};    // [n_shared_refs] by level parity
  void* part[2] = {nullptr, nullptr};   // [n_shared_refs] by step parity
  void* partr[2] = {nullptr, nullptr};  // adjoint pairing partials
};

struct Problem {
  Probe probe;
  Mesh* mesh = nullptr;
  int prec = 0;        // 0 fp64, 1 fp32
  size_t ts = 8;       // element size
  double dt = 0;
  int64_t nt = 0;
  int64_t ckpt_every = 0;
  int64_t grad_every = 1;  // gradient subsampling ratio r: pair (and keep states) every r-th step
  size_t budget = 0;
  int device = 0;
  int block = 64;
  // mesh data
  uint32_t* d_lmap = nullptr;
  void* d_geom = nullptr;
  int32_t *d_cell_start = nullptr, *d_own_start = nullptr, *d_sh_start = nullptr, *d_sh_idx = nullptr,
          *d_shp_ptr = nullptr, *d_shp_slot = nullptr, *d_ref_slots = nullptr, *d_gword_off = nullptr,
          *d_glist_off = nullptr;
  uint32_t* d_gword = nullptr;
  uint16_t* d_glist = nullptr;
  int64_t nref = 0;             // shared refs
  int64_t rs = 1;               // per-shot length of the per-ref arrays: max(1, nref)
  int64_t ls = 0;               // level vector length: n_dofs + nref (copies per ref)
  // Shots stepped together.  Every per-shot buffer holds n_shots copies, shot s
  // at s times the per-shot length (level vectors ls, DOF vectors n_dofs, ref
  // arrays rs, traces n_steps * n_rec); mesh tables, coefficients, the wavelet
  // and the receivers are shared.
  int nshot = 1;
  // coefficients
  std::vector<double> eta;      // host damping (empty = none)
  void* d_gamma = nullptr;
  void* d_gdet = nullptr;       // [n_cells] dt^2 / |det J|
  void* d_beta = nullptr;
  int32_t* d_damp_patch = nullptr;  // [np] patch touches a damped DOF
  void* d_c2 = nullptr;
  void *d_c2_ref = nullptr, *d_gamma_ref = nullptr, *d_beta_ref = nullptr;  // [nref]
  void* d_minv_sqrt = nullptr;  // for the power iteration
  // absorbing boundary term (off unless enabled): the boundary DOFs' damping
  // a_i = eta_i dt/2 + dt c_i b_i/(2 M_i) is rebuilt from c at every solve
  bool absorb = false;
  std::vector<int32_t> bnd_dof;  // boundary DOFs (b_i != 0), ascending
  std::vector<double> bnd_b;     // b_i = boundary integral of phi_i
  int nbd = 0, nbr = 0;          // boundary DOFs, shared refs of boundary DOFs
  int32_t* d_bnd_dof = nullptr;  // [nbd]
  int32_t* d_bnd_ref = nullptr;  // [2*nbr] (shared ref, boundary index)
  double* d_bnd_coef = nullptr;  // [3*nbd] (eta dt/2, dt b/(2M), dt^2/M)
  double* d_bnd_hb = nullptr;    // [nbd] dt b / 2
  void *d_ub = nullptr, *d_lb = nullptr;  // [n_shots][nt+1][nbd] u^n, lambda^n at the boundary DOFs
  size_t bnd_rec_bytes = 0;
  double* d_bnd_part = nullptr;  // [kBndChunks*nbd] ordered partial sums of the gradient term
  // PML (triangles): per-axis damping functions sigma_x, sigma_z; its tr Psi_1 is
  // the damping eta.  Off while sigma is empty.
  std::vector<double> sigma;    // [2*n_dofs] host, sigma_x then sigma_z
  void* d_sig = nullptr;        // [2*n_dofs]
  void* d_sig_ref = nullptr;    // [2*rs] per shared ref
  void* d_pml_b = nullptr;      // [4*n_cells] |det J| J^-T
  int32_t* d_list[2] = {nullptr, nullptr};  // patches without / with a DOF in the layer
  int n_list[2] = {0, 0};
  void* d_pp[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [sweep][level parity]: [n_shots][2][ls]
  void* d_pt[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [sweep][step parity]: [n_shots][2][rs]
  bool pml() const { return !sigma.empty(); }
  // PML on tetrahedra (pml3d.hip): sigma holds sigma_x, sigma_y, sigma_z; per-cell
  // contractions and per-DOF update rows beside the stiffness apply, one shot, the
  // forward states (u and omega) kept for the reverse sweep
  bool pml3 = false;
  int32_t* d_cdof = nullptr;                    // [nd][n_cells] DOF of each cell node
  void* d_b3 = nullptr;                         // [9*n_cells] |det J| J^-T
  int32_t *d_csr_ptr = nullptr, *d_cpos = nullptr;  // DOF -> its range of cell-node values; their places
  void* d_mass = nullptr;                       // [n_dofs] lumped mass
  void* d_cellout = nullptr;                    // [12*n_cells*nd] cell-node values
  void* d_ku = nullptr;                         // [n_dofs] K u
  void* d_p3[2] = {nullptr, nullptr};           // [3*n_dofs] p (forward) or mu (reverse), by parity
  void* d_nu3[2] = {nullptr, nullptr};          // [n_dofs] nu by parity
  void* d_y3 = nullptr;                         // omega levels [n_y3][n_dofs]
  int64_t n_y3 = 0;
  void* d_svec = nullptr;                       // [n_dofs] the source's load vector
  int32_t *d_rptr = nullptr, *d_ridx = nullptr;  // DOF -> receiver rows (transposed sampling)
  void* d_rw = nullptr;
  bool p3_points_dirty = true;
  // sweeps
  Sweep fwd, adj;
  void* d_lam[2] = {nullptr, nullptr};
  // With the absorbing boundary's records the adjoint levels rotate through a ring of
  // lam_k levels instead (lam_k - 1 complete levels recorded per gather launch).
  void* d_lam_ring = nullptr;
  int lam_k = 2;
  double* d_gacc = nullptr;
  double* d_red = nullptr;      // reduction scratch
  int* d_flag = nullptr;        // non-finite sentinel of the most recent solve (see check_every)
  int red_blocks = 256;
  void* d_slots = nullptr;      // forward state slots
  int64_t n_slots = 0;
  void* d_ck_u = nullptr;
  void* d_ck_du = nullptr;
  int64_t n_ck = 0, seg = 0;
  bool store_all = false;
  bool store_sub = false;       // r > 1: slots 0, 1 a ring, slot 2 + n/r holds level n (n % r == 0)
  void* d_resid = nullptr;      // [nt*nrec]
  void* d_traces_tmp = nullptr; // [nt*nrec]
  // sources / receivers
  bool has_src = false;
  PointTables src, rec;
  void* d_wavelet = nullptr;    // [nt], or [n_shots][nt] when wavelet_per_shot
  bool wavelet_per_shot = false;
  std::vector<double> wavelet;

  ~Problem();
};

Status problem_create(Mesh* m, int prec, double dt, int64_t nt, int64_t ckpt_every, size_t budget,
                      int n_shots, int64_t grad_every, Problem** out);
Status set_damping(Problem* p, const double* eta);
// PML damping functions sigma [n_dofs*2] (sigma_x, sigma_z per DOF), or NULL = off.
Status set_pml(Problem* p, const double* sigma);
Status set_absorbing_boundary(Problem* p, bool on);
Status set_sources(Problem* p, const double* xs, int nsrc, double f0, double t0, double amp);
Status set_wavelet(Problem* p, const double* w);
Status set_wavelets(Problem* p, const double* w);
Status set_receivers(Problem* p, const double* xr, int nrec);
Status forward(Problem* p, const double* c_dev, void* traces_dev, hipStream_t s);
// As forward, with its two level buffers in the library's static per-device
// workspace instead of the problem's (no device allocation in the call).
Status forward_noalloc(Problem* p, const double* c_dev, void* traces_dev, hipStream_t s);
// J and, unless grad_dev is NULL, dJ/dc.  accumulate: *J and grad_dev receive the
// sums of their old values and this problem's (several problems summed in place).
Status misfit_gradient(Problem* p, const double* c_dev, const void* obs_dev, double* J,
                       double* grad_dev, void* traces_dev, hipStream_t s, bool accumulate = false);
// Misfit only: the forward solve and J, no adjoint sweep.
Status misfit(Problem* p, const double* c_dev, const void* obs_dev, double* J, void* traces_dev, hipStream_t s);
// Synchronise s and report the non-finite sentinel of the most recent solve:
// KMV_ECFL if it tripped and dt exceeds the Gershgorin step bound for the solve's
// wave speed, KMV_ENUMERIC if it tripped otherwise, else KMV_OK.
Status solve_status(Problem* p, hipStream_t s);
Status adjoint(Problem* p, const double* c_dev, const void* adj_dev, void* lambda_out,
               void* src_trace_out, hipStream_t s);
Status stiffness_apply(Problem* p, const double* c_dev, const void* u_dev, void* y_dev, hipStream_t s);
Status spectral_radius(Problem* p, const double* c_dev, int iters, uint64_t seed, double* rho,
                       hipStream_t s);
Status profile_enable(Problem* p, int every);
Status profile_read(Problem* p, int variant, int64_t* launches, int64_t* timed, double* mean_ms);

}  // namespace kmv
