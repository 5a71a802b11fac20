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

// Point tables on the device: injection groups (per patch) and sampling rows.
struct PointTables {
  int npts = 0;
  int32_t* grp_ptr = nullptr;   // [np+1]
  int32_t* grp_local = nullptr;
  int32_t* grp_eptr = nullptr;
  int32_t* ent_pt = nullptr;
  void* ent_w = nullptr;
  int32_t* s_dof = nullptr;     // [npts*nd] sampling
  void* s_w = nullptr;          // [npts*nd]
  std::vector<double> host_xyz;
};

struct Problem {
  Mesh* mesh = nullptr;
  int prec = 0;        // 0 fp64, 1 fp32
  size_t ts = 8;       // element size
  double dt = 0;
  int64_t nt = 0;
  int64_t ckpt_every = 0;
  size_t budget = 0;
  int device = 0;
  int block = 64;
  int nloc = 0;
  // mesh data
  uint16_t* d_lmap = nullptr;
  void* d_geom = nullptr;
  void* d_D = nullptr;
  void* d_W = nullptr;
  int32_t *d_cell_start = nullptr, *d_own_start = nullptr, *d_sh_start = nullptr, *d_sh_idx = nullptr,
          *d_colour_start = nullptr, *d_ncol = nullptr, *d_shp_ptr = nullptr, *d_shp_slot = nullptr;
  // coefficients
  std::vector<double> eta;      // host damping (empty = none)
  void* d_gamma = nullptr;
  void* d_beta = nullptr;
  void* d_c2 = nullptr;
  void* d_minv_sqrt = nullptr;  // for the power iteration
  // state
  void* d_du = nullptr;
  void* d_partial = nullptr;
  void* d_partial_r = nullptr;
  void* d_lam[2] = {nullptr, nullptr};
  void* d_dlam = nullptr;
  double* d_gacc = nullptr;
  double* d_red = nullptr;      // reduction scratch
  int red_blocks = 256;
  void* d_slots = nullptr;      // state slots
  int64_t n_slots = 0;
  void* d_ck_u = nullptr;
  void* d_ck_du = nullptr;
  int64_t n_ck = 0, seg = 0;
  bool store_all = false;
  void* d_resid = nullptr;      // [nt*nrec]
  void* d_traces_tmp = nullptr; // [nt*nrec]
  // sources / receivers
  bool has_src = false;
  PointTables src, rec;
  void* d_wavelet = nullptr;    // [nt]
  std::vector<double> wavelet;
  double f0 = 0, t0 = 0, amp = 0;

  ~Problem();
};

Status problem_create(Mesh* m, int prec, double dt, int64_t nt, int64_t ckpt_every, size_t budget,
                      Problem** out);
Status set_damping(Problem* p, const double* eta);
Status set_sources(Problem* p, const double* xs, int nsrc, double f0, double t0, double amp);
Status set_wavelet(Problem* p, const double* w);
Status set_receivers(Problem* p, const double* xr, int nrec);
Status forward(Problem* p, const double* c_dev, void* traces_dev, hipStream_t s);
Status misfit_gradient(Problem* p, const double* c_dev, const void* obs_dev, double* J,
                       double* grad_dev, void* traces_dev, hipStream_t s);
Status adjoint(Problem* p, const double* c_dev, const void* adj_dev, void* lambda_out,
               void* src_trace_out, hipStream_t s);
Status stiffness_apply(Problem* p, const double* c_dev, const void* u_dev, void* y_dev, hipStream_t s);
Status spectral_radius(Problem* p, const double* c_dev, int iters, uint64_t seed, double* rho,
                       hipStream_t s);

}  // namespace kmv
