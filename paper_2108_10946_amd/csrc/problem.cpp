// Device-side problem state and the forward / adjoint / gradient drivers.
//
// Forward (eqs. Leapfrog, forward3): per step n, k_patch + k_shared advance
// u^n -> u^{n+1} in increment form (du^{n+1} = beta du^n + gamma (b^n - K u^n),
// u^{n+1} = u^n + du^{n+1}, beta = (1-a)/(1+a), gamma = dt^2 / (M (1+a)), a =
// eta dt / 2), and k_sample records d^{n+1} = P u^{n+1}.
// Reverse sweep (eq. acoustic_pml_FEM_adj, transposed scheme): per step m = N_t..1,
// dlam^m = beta dlam^{m+1} + gamma (P^T y^m / dt^2 - K lambda^{m+1}),
// lambda^m = lambda^{m+1} + dlam^m, with the same kernels, fused with the gradient
// pairing of lambda^{m+1} and u^m (eq. gradient3), accumulated in float64.
// Forward states are either all kept (when they fit the memory budget) or
// checkpointed every S steps and recomputed segment by segment.
#include "problem.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "../../include/kmvwave.h"
#include "boundary.hpp"
#include "kernels.hpp"
#include "pml3d.hpp"

namespace kmv {

namespace {
thread_local hipStream_t t_alloc_stream = nullptr;
}
hipStream_t alloc_stream() { return t_alloc_stream; }
AllocStreamScope::AllocStreamScope(hipStream_t s) : prev(t_alloc_stream) { t_alloc_stream = s; }
AllocStreamScope::~AllocStreamScope() { t_alloc_stream = prev; }

namespace {

#define HIPTRY(expr)                                                                       \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return Status{KMV_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)};      \
  } while (0)

#define STTRY(expr)                      \
  do {                                   \
    Status _s = (expr);                  \
    if (_s.code != KMV_OK) return _s;    \
  } while (0)

const Status OK{KMV_OK, ""};

// Device memory of a problem.  On a thread that set an allocation stream (the
// server's workers), allocations and frees are stream-ordered (hipMallocAsync /
// hipFreeAsync), so creating or destroying a problem does not wait for work that
// other streams have in flight.
Status dmalloc(void** dst, size_t bytes) {
  const hipError_t e = alloc_stream() ? hipMallocAsync(dst, bytes, alloc_stream()) : hipMalloc(dst, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return Status{KMV_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  return OK;
}

void dfree(void* p) {
  if (!p) return;
  if (alloc_stream())
    (void)hipFreeAsync(p, alloc_stream());
  else
    (void)hipFree(p);
}

template <typename V>
Status upload(void** dst, const V* src, size_t count) {
  dfree(*dst);
  *dst = nullptr;
  if (count == 0) return OK;
  STTRY(dmalloc(dst, count * sizeof(V)));
  if (alloc_stream()) {
    HIPTRY(hipMemcpyAsync(*dst, src, count * sizeof(V), hipMemcpyHostToDevice, alloc_stream()));
    HIPTRY(hipStreamSynchronize(alloc_stream()));  // the host source is a temporary
  } else {
    HIPTRY(hipMemcpy(*dst, src, count * sizeof(V), hipMemcpyHostToDevice));
  }
  return OK;
}

template <typename V>
Status upload_i(V** dst, const std::vector<V>& v) {
  void* p = *dst;
  Status s = upload(&p, v.data(), v.size());
  *dst = (V*)p;
  return s;
}

Status upload_real(void** dst, const std::vector<double>& v, int prec) {
  if (prec == KMV_FP64) return upload(dst, v.data(), v.size());
  std::vector<float> f(v.begin(), v.end());
  return upload(dst, f.data(), f.size());
}

Status alloc(void** dst, size_t bytes) {
  dfree(*dst);
  *dst = nullptr;
  if (bytes == 0) return OK;
  return dmalloc(dst, bytes);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

Status upload_coefficients(Problem* p) {
  const Mesh& m = *p->mesh;
  std::vector<double> gamma(m.n_dofs), beta;
  const double dt2 = p->dt * p->dt;
  // boundary DOFs carry c-dependent damping when the absorbing boundary is on
  std::vector<int32_t> bix(p->absorb ? m.n_dofs : 0, -1);
  for (int t = 0; p->absorb && t < p->nbd; ++t) bix[p->bnd_dof[t]] = t;
  auto damped = [&](int64_t i) { return (!p->eta.empty() && p->eta[i] != 0.0) || (p->absorb && bix[i] >= 0); };
  if (!p->eta.empty() || p->absorb) beta.resize(m.n_dofs);
  for (int64_t i = 0; i < m.n_dofs; ++i) {
    const double a = p->eta.empty() ? 0.0 : p->eta[i] * p->dt / 2.0;
    gamma[i] = dt2 / (m.mass[i] * (1.0 + a));
    if (!beta.empty()) beta[i] = (1.0 - a) / (1.0 + a);
  }
  STTRY(upload_real(&p->d_gamma, gamma, p->prec));
  {
    std::vector<double> gr(std::max<int64_t>(1, m.n_shared_refs), 0.0), br;
    for (int64_t r = 0; r < m.n_shared_refs; ++r) gr[r] = gamma[m.sh_idx[r]];
    STTRY(upload_real(&p->d_gamma_ref, gr, p->prec));
    if (!beta.empty()) {
      br.assign(gr.size(), 0.0);
      for (int64_t r = 0; r < m.n_shared_refs; ++r) br[r] = beta[m.sh_idx[r]];
    }
    if (br.empty()) {
      dfree(p->d_beta_ref);
      p->d_beta_ref = nullptr;
    } else {
      STTRY(upload_real(&p->d_beta_ref, br, p->prec));
    }
  }
  {
    std::vector<double> gd(m.n_cells);
    for (int64_t e = 0; e < m.n_cells; ++e) gd[e] = dt2 / m.absdet[e];
    STTRY(upload_real(&p->d_gdet, gd, p->prec));
  }
  if (beta.empty()) {
    dfree(p->d_beta);
    p->d_beta = nullptr;
  } else {
    STTRY(upload_real(&p->d_beta, beta, p->prec));
  }
  // patches that touch a damped DOF (owned or shared)
  std::vector<int32_t> flag(m.n_patches, 0);
  if (!beta.empty()) {
    for (int64_t q = 0; q < m.n_patches; ++q) {
      for (int32_t i = m.patch_own_start[q]; i < m.patch_own_start[q + 1] && !flag[q]; ++i)
        if (damped(i)) flag[q] = 1;
      for (int32_t r = m.patch_sh_start[q]; r < m.patch_sh_start[q + 1] && !flag[q]; ++r)
        if (damped(m.sh_idx[r])) flag[q] = 1;
    }
  }
  STTRY(upload_i(&p->d_damp_patch, flag));
  if (p->absorb) {
    std::vector<double> coef(3 * (size_t)p->nbd), hb(p->nbd);
    for (int t = 0; t < p->nbd; ++t) {
      const int32_t i = p->bnd_dof[t];
      coef[3 * t] = p->eta.empty() ? 0.0 : p->eta[i] * p->dt / 2.0;
      coef[3 * t + 1] = p->dt * p->bnd_b[t] / (2.0 * m.mass[i]);
      coef[3 * t + 2] = dt2 / m.mass[i];
      hb[t] = p->dt * p->bnd_b[t] / 2.0;
    }
    std::vector<int32_t> refs;
    for (int64_t r = 0; r < m.n_shared_refs; ++r)
      if (bix[m.sh_idx[r]] >= 0) {
        refs.push_back((int32_t)r);
        refs.push_back(bix[m.sh_idx[r]]);
      }
    p->nbr = (int)(refs.size() / 2);
    if (refs.empty()) refs.assign(2, 0);
    STTRY(upload_i(&p->d_bnd_coef, coef));
    STTRY(upload_i(&p->d_bnd_hb, hb));
    STTRY(upload_i(&p->d_bnd_ref, refs));
  }
  return OK;
}

// Point tables: each point is located in one cell (lowest input id on ties); its
// entry (patch-local cell, point index, phi_a(x) per node) goes to the patch of
// that cell, entries in point order.  Global rows: DOF ids and weights.  With
// nshot > 1 the points are shot-major, npts/nshot per shot, and each shot gets its
// own [np+1] block of patch offsets (into the shared entry arrays) and point
// indices counted within the shot.
Status build_points(Problem* p, const double* xyz, int npts, int nshot, PointTables& T) {
  const Mesh& m = *p->mesh;
  const int nd = m.nd, dim = m.dim;
  std::vector<int32_t> sdof((size_t)npts * nd);
  std::vector<double> sw((size_t)npts * nd);
  std::vector<int64_t> cell_of(npts);
  for (int j = 0; j < npts; ++j) {
    PointLoc loc;
    if (!m.locate(xyz + (size_t)j * dim, loc))
      return Status{KMV_EOUTSIDE, "point " + std::to_string(j) + " lies outside the mesh"};
    cell_of[j] = loc.cell;
    for (int a = 0; a < nd; ++a) {
      sdof[(size_t)j * nd + a] = (int32_t)m.cell_dofs[loc.cell * nd + a];
      sw[(size_t)j * nd + a] = loc.phi[a];
    }
  }
  std::vector<int32_t> order(npts), patch_of(npts);
  for (int j = 0; j < npts; ++j) {
    order[j] = j;
    patch_of[j] = (int32_t)(std::upper_bound(m.patch_cell_start.begin(), m.patch_cell_start.end(),
                                             (int32_t)cell_of[j]) - m.patch_cell_start.begin() - 1);
  }
  const int nps = npts / nshot;
  const int64_t np1 = m.n_patches + 1;
  std::vector<int32_t> ptr((size_t)nshot * np1, 0), pcell(npts), ppt(npts);
  std::vector<double> pw((size_t)npts * nd);
  for (int s = 0; s < nshot; ++s) {
    const int j0 = s * nps;
    std::stable_sort(order.begin() + j0, order.begin() + j0 + nps,
                     [&](int32_t a, int32_t b) { return patch_of[a] < patch_of[b]; });
    int32_t* pt = ptr.data() + (size_t)s * np1;
    for (int k = j0; k < j0 + nps; ++k) {
      const int j = order[k];
      pt[patch_of[j] + 1]++;
      pcell[k] = (int32_t)(cell_of[j] - m.patch_cell_start[patch_of[j]]);
      ppt[k] = j - j0;
      for (int a = 0; a < nd; ++a) pw[(size_t)k * nd + a] = sw[(size_t)j * nd + a];
    }
    pt[0] = j0;
    for (int64_t q = 0; q < m.n_patches; ++q) pt[q + 1] += pt[q];
  }
  T.npts = npts;
  T.shot_stride = nshot > 1 ? np1 : 0;
  STTRY(upload_i(&T.pp_ptr, ptr));
  STTRY(upload_i(&T.pp_cell, pcell));
  STTRY(upload_i(&T.pp_pt, ppt));
  STTRY(upload_real(&T.pp_w, pw, p->prec));
  STTRY(upload_i(&T.s_dof, sdof));
  STTRY(upload_real(&T.s_w, sw, p->prec));
  T.h_dof = sdof;
  T.h_w = sw;
  p->p3_points_dirty = true;
  return OK;
}

void free_points(PointTables& T) {
  for (void* q : {(void*)T.pp_ptr, (void*)T.pp_cell, (void*)T.pp_pt, T.pp_w, (void*)T.s_dof, T.s_w}) dfree(q);
  T = PointTables();
}

// Launch through the timing probe: every probe.every-th launch of a variant gets
// start/stop events recorded by its own dispatch (resolved in profile_read).  The
// launcher is called as launch(e0, e1) with null events for untimed launches.
template <typename F>
Status probed(Problem* p, int variant, hipStream_t s, F&& launch) {
  Probe& pr = p->probe;
  const bool timed = pr.every > 0 && (pr.launches[variant] % pr.every) == 0;
  pr.launches[variant]++;
  hipEvent_t a = nullptr, b = nullptr;
  if (timed) {
    for (hipEvent_t* ev : {&a, &b}) {
      if (!pr.pool.empty()) {
        *ev = pr.pool.back();
        pr.pool.pop_back();
      } else {
        HIPTRY(hipEventCreate(ev));
      }
    }
  }
  HIPTRY(launch(a, b));
  if (timed) pr.pending.push_back({variant, a, b});
  return OK;
}

Status resolve_probe(Problem* p) {
  Probe& pr = p->probe;
  for (auto& q : pr.pending) {
    HIPTRY(hipEventSynchronize(q.b));
    float ms = 0;
    HIPTRY(hipEventElapsedTime(&ms, q.a, q.b));
    pr.total_ms[q.variant] += ms;
    pr.timed[q.variant]++;
    pr.pool.push_back(q.a);
    pr.pool.push_back(q.b);
  }
  pr.pending.clear();
  return OK;
}

template <typename T>
StepArgs<T> base_args(const Problem* p) {
  const Mesh& m = *p->mesh;
  StepArgs<T> a{};
  a.lmap = p->d_lmap;
  a.geom = (const T*)p->d_geom;
  a.gdet = (const T*)p->d_gdet;
  a.cell_start = p->d_cell_start;
  a.own_start = p->d_own_start;
  a.sh_start = p->d_sh_start;
  a.sh_idx = p->d_sh_idx;
  a.gword = p->d_gword;
  a.gword_off = p->d_gword_off;
  a.glist = p->d_glist;
  a.glist_off = p->d_glist_off;
  a.shp_ptr = p->d_shp_ptr;
  a.shp_slot = p->d_shp_slot;
  a.ref_slots = p->d_ref_slots;
  a.n_cells = m.n_cells;
  a.n_own = m.n_own_total;
  a.n_dofs = m.n_dofs;
  a.nbl_max = m.max_nbl;
  a.slot_stride = m.slot_stride;
  a.glist_max = m.max_glist;
  a.c2 = (const T*)p->d_c2;
  a.c2_ref = (const T*)p->d_c2_ref;
  a.gamma = (const T*)p->d_gamma;
  a.gamma_ref = (const T*)p->d_gamma_ref;
  a.beta = (const T*)p->d_beta;
  a.beta_ref = (const T*)p->d_beta_ref;
  a.damp_patch = p->d_damp_patch;
  a.amp_scale = T(1);
  a.n_shots = p->nshot;
  a.ss_level = p->ls;
  a.ss_dof = m.n_dofs;
  a.ss_ref = p->rs;
  a.ss_trace = p->nt * p->rec.npts;
  return a;
}

// Parities of one launch: the level finished in it (cur) and the one before it
// (prev), and the step whose partial sums it reads (prev) and writes (cur).
struct Par {
  int lvl_prev, lvl_cur, step_prev, step_cur;
};

template <typename T>
Status step(Problem* p, Sweep& S, bool grad, bool prev, const T* u_in, const T* u_prev, T* u_out, Par q,
            const PointTables* inj, const T* amp, int amp_stride, int64_t amp_shot_stride, T scale,
            const T* uf, T* trace_row, hipStream_t s) {
  const Mesh& m = *p->mesh;
  StepArgs<T> a = base_args<T>(p);
  a.mode = 0;
  a.prev = prev ? 1 : 0;
  a.pair_prev = grad && p->grad_every == 1 ? 1 : 0;
  a.u_in = u_in;
  a.u_in_sh = const_cast<T*>(u_in);
  a.u_prev = u_prev ? u_prev : u_in;  // never dereferenced as a previous level when !prev
  a.u_out = u_out;
  a.du = (T*)S.d;
  a.dsh_prev = (const T*)S.dsh[q.lvl_prev];
  a.dsh_cur = (T*)S.dsh[q.lvl_cur];
  a.part_prev = (const T*)S.part[q.step_prev];
  a.part_cur = (T*)S.part[q.step_cur];
  if (inj && inj->pp_ptr) {
    a.inj_ptr = inj->pp_ptr;
    a.inj_cell = inj->pp_cell;
    a.inj_pt = inj->pp_pt;
    a.inj_w = (const T*)inj->pp_w;
    a.amp = amp;
    a.amp_stride = amp_stride;
    a.amp_scale = scale;
    a.ss_inj = inj->shot_stride;
    a.ss_amp = amp_shot_stride;
  }
  if (trace_row) {
    a.rec_ptr = p->rec.pp_ptr;
    a.rec_cell = p->rec.pp_cell;
    a.rec_pt = p->rec.pp_pt;
    a.rec_w = (const T*)p->rec.pp_w;
    a.trace_row = trace_row;
  }
  if (grad) {
    a.uf = uf;
    a.partr_prev = (const T*)S.partr[q.step_prev];
    a.partr_cur = (T*)S.partr[q.step_cur];
    a.gacc = p->d_gacc;
  }
  if (!p->pml())
    return probed(p, grad ? 1 : 0, s, [&](hipEvent_t e0, hipEvent_t e1) {
      return launch_step<T>(m.dim, m.nd, grad, a, (int)m.n_patches, p->block, s, e0, e1);
    });
  // PML: the patches touching the layer in the PML instance, then the others in
  // the plain one (the two sets are disjoint and neither reads what the other
  // writes in this step; sweep 0 forward, 1 reverse).  A single launch of the PML
  // instance over every patch measured slower: its LDS leaves one workgroup per CU.
  const int sw = &S == &p->adj ? 1 : 0;
  StepArgs<T> a0 = a;
  a.patch_list = p->d_list[1];
  a.pml_b = (const T*)p->d_pml_b;
  a.sig = (const T*)p->d_sig;
  a.sig_ref = (const T*)p->d_sig_ref;
  a.pp_in = (const T*)p->d_pp[sw][q.lvl_cur];
  a.pp_in_sh = (T*)p->d_pp[sw][q.lvl_cur];
  a.pp_io = (T*)p->d_pp[sw][q.lvl_prev];
  a.pt_prev = (const T*)p->d_pt[sw][q.step_prev];
  a.pt_cur = (T*)p->d_pt[sw][q.step_cur];
  a.pml_ls = p->ls;
  a.pml_rs = p->rs;
  a.ss_pml = 2 * p->ls;
  a.ss_pt = 2 * p->rs;
  a.pml_dt = (T)p->dt;
  a.inv_dt = (T)(1.0 / p->dt);
  a.pml_trans = sw;  // the reverse sweep, also its launches without the pairing
  HIPTRY(launch_step<T>(m.dim, m.nd, grad, a, p->n_list[1], p->block, s, nullptr, nullptr, true));
  a0.patch_list = p->d_list[0];
  if (p->n_list[0] > 0)
    STTRY(probed(p, grad ? 1 : 0, s, [&](hipEvent_t e0, hipEvent_t e1) {
      return launch_step<T>(m.dim, m.nd, grad, a0, p->n_list[0], p->block, s, e0, e1);
    }));
  return OK;
}

// Zero the PML's auxiliary levels and partial sums of one sweep (0 forward, 1 adjoint).
template <typename T>
Status zero_pml(Problem* p, int sw, hipStream_t s) {
  if (!p->pml()) return OK;
  for (int k = 0; k < 2; ++k) {
    HIPTRY(launch_fill<T>((T*)p->d_pp[sw][k], T(0), 2 * p->ls * p->nshot, s));
    HIPTRY(launch_fill<T>((T*)p->d_pt[sw][k], T(0), 2 * p->rs * p->nshot, s));
  }
  return OK;
}

// Finish the shared DOFs of one level (u_cur, S.dsh[q.lvl_cur]) from the partials
// of the step that produced it.
template <typename T>
Status finish(Problem* p, Sweep& S, bool grad, const T* u_prev, T* u_cur, Par q, hipStream_t s) {
  const Mesh& m = *p->mesh;
  FinishArgs<T> f{};
  f.n_own = m.n_own_total;
  f.n_shared = m.n_shared;
  f.n_dofs = m.n_dofs;
  f.shp_ptr = p->d_shp_ptr;
  f.shp_slot = p->d_shp_slot;
  f.mode = 0;
  f.part_prev = (const T*)S.part[q.step_prev];
  f.u_prev = u_prev;
  f.u_cur = u_cur;
  f.dsh_prev = (const T*)S.dsh[q.lvl_prev];
  f.dsh_cur = (T*)S.dsh[q.lvl_cur];
  f.gamma = (const T*)p->d_gamma;
  f.beta = (const T*)p->d_beta;
  if (grad) {
    f.partr_prev = (const T*)S.partr[q.step_prev];
    f.gacc = p->d_gacc;
  }
  f.n_shots = p->nshot;
  f.ss_level = p->ls;
  f.ss_dof = m.n_dofs;
  f.ss_ref = p->rs;
  return probed(p, grad ? 3 : 2, s,
                [&](hipEvent_t e0, hipEvent_t e1) { return launch_finish<T>(grad, f, s, e0, e1); });
}

// Gradient subsampling: the pairing partials of the shared DOFs written by
// adjoint launch m (parities q), added to their accumulators right away.
template <typename T>
Status pair_finish(Problem* p, Par q, hipStream_t s) {
  const Mesh& m = *p->mesh;
  FinishArgs<T> f{};
  f.n_own = m.n_own_total;
  f.n_shared = m.n_shared;
  f.n_dofs = m.n_dofs;
  f.shp_ptr = p->d_shp_ptr;
  f.shp_slot = p->d_shp_slot;
  f.mode = 2;
  f.partr_prev = (const T*)p->adj.partr[q.step_cur];
  f.gacc = p->d_gacc;
  f.n_shots = p->nshot;
  f.ss_level = p->ls;
  f.ss_dof = m.n_dofs;
  f.ss_ref = p->rs;
  return probed(p, 3, s, [&](hipEvent_t e0, hipEvent_t e1) { return launch_finish<T>(true, f, s, e0, e1); });
}

Par fwd_par(int64_t n) { return Par{(int)((n + 1) & 1), (int)(n & 1), (int)((n + 1) & 1), (int)(n & 1)}; }
// adjoint launch m finishes level m+1 from level m+2 and the partials of launch m+1
Par adj_par(int64_t m) { return Par{(int)(m & 1), (int)((m + 1) & 1), (int)((m + 1) & 1), (int)(m & 1)}; }

template <typename T>
T* slot_ptr(Problem* p, int64_t k) {
  return (T*)p->d_slots + k * p->ls * p->nshot;
}

Status ensure_slots(Problem* p, int64_t n) {
  if (p->n_slots >= n) return OK;
  STTRY(alloc(&p->d_slots, (size_t)n * p->ls * p->nshot * p->ts));
  p->n_slots = n;
  return OK;
}

template <typename T>
Status zero_level(Problem* p, Sweep& S, T* u, int lvl_par, hipStream_t s) {
  const Mesh& m = *p->mesh;
  HIPTRY(launch_fill<T>(u, T(0), p->ls * p->nshot, s));
  HIPTRY(launch_fill<T>((T*)S.d, T(0), m.n_dofs * p->nshot, s));
  HIPTRY(launch_fill<T>((T*)S.dsh[lvl_par], T(0), p->rs * p->nshot, s));
  return OK;
}

// Non-finite sentinel: every kCheckEvery-th level of each sweep (and the last) is
// scanned for NaN or infinity; an unstable step grows without bound, so a scan of
// every 128th level finds it long before the end of a typical window.
constexpr int64_t kCheckEvery = 128;

template <typename T>
Status check_level(Problem* p, const T* lvl, hipStream_t s) {
  HIPTRY(launch_check_finite<T>(lvl, p->mesh->n_dofs, p->ls, p->nshot, p->d_flag, s));
  return OK;
}

Status clear_flag(Problem* p, hipStream_t s) {
  HIPTRY(launch_fill_i32(p->d_flag, 0, 1, s));
  return OK;
}

// The sentinel tripped (or J is not finite): classify by the step bound of eq.
// spectral for the solve's wave speed (sqrt of the c^2 the kernels used).
template <typename T>
Status classify_nonfinite(Problem* p, hipStream_t s) {
  const Mesh& m = *p->mesh;
  std::vector<T> c2(m.n_dofs);
  HIPTRY(hipMemcpyAsync(c2.data(), p->d_c2, m.n_dofs * sizeof(T), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  std::vector<double> c(m.n_dofs);
  for (int64_t i = 0; i < m.n_dofs; ++i) c[i] = std::sqrt((double)c2[i]);
  const double rho = gershgorin_rho(m, c.data());
  const double dtg = 2.0 / std::sqrt(rho);
  if (p->dt > dtg)
    return Status{KMV_ECFL, "the solve left the floating-point range and dt = " + std::to_string(p->dt) +
                                " s exceeds the Gershgorin step bound " + std::to_string(dtg) +
                                " s of this wave speed (eq. spectral)"};
  return Status{KMV_ENUMERIC, "the solve produced a non-finite value (dt is within the Gershgorin step "
                              "bound; check the wave speed, damping and source inputs)"};
}

// Forward launches n0..n1-1 from a complete level n0 (u in slot_of(n0), owned
// increments in fwd.d, shared increments in fwd.dsh[n0&1]); ends with level n1
// complete.  traces: rows n-1 = d^n.  save_ck: checkpoints at multiples of seg.
// ub: boundary records, row n = u^n at the boundary DOFs (level n is complete
// once launch n has run, level n1 after the final finish).
template <typename T, typename F>
Status run_forward(Problem* p, int64_t n0, int64_t n1, F slot_of, T* traces, bool save_ck, hipStream_t s,
                   T* ub = nullptr) {
  auto record = [&](int64_t n) -> Status {
    HIPTRY(launch_gather_boundary<T>(slot_of(n), p->ls, p->nshot, p->nbd, p->d_bnd_dof, ub + n * p->nbd,
                                     (p->nt + 1) * p->nbd, s));
    return OK;
  };
  const Mesh& m = *p->mesh;
  Sweep& S = p->fwd;
  const int64_t ns = p->nshot;
  const size_t lb = (size_t)(p->ls * ns) * sizeof(T);
  const size_t ob = (size_t)(m.n_dofs * ns) * sizeof(T), shb = (size_t)(p->rs * ns) * sizeof(T);
  bool fresh = true;
  for (int64_t n = n0; n < n1; ++n) {
    if (save_ck && n % p->seg == 0) {
      if (!fresh) STTRY(finish<T>(p, S, false, slot_of(n - 1), slot_of(n), fwd_par(n), s));
      const int64_t k = n / p->seg;
      T* cu = (T*)p->d_ck_u + k * p->ls * ns;
      T* cd = (T*)p->d_ck_du + k * (m.n_dofs + p->rs) * ns;
      HIPTRY(hipMemcpyAsync(cu, slot_of(n), lb, hipMemcpyDeviceToDevice, s));
      HIPTRY(hipMemcpyAsync(cd, S.d, ob, hipMemcpyDeviceToDevice, s));
      HIPTRY(hipMemcpyAsync(cd + m.n_dofs * ns, S.dsh[n & 1], shb, hipMemcpyDeviceToDevice, s));
      fresh = true;
    }
    T* row = (traces && n >= 1) ? traces + (n - 1) * p->rec.npts : nullptr;
    STTRY(step<T>(p, S, false, !fresh, slot_of(n), n > n0 ? slot_of(n - 1) : nullptr, slot_of(n + 1),
                  fwd_par(n), &p->src, (const T*)p->d_wavelet + n, 0, p->wavelet_per_shot ? p->nt : 0, T(1),
                  nullptr, row, s));
    fresh = false;
    if (ub) STTRY(record(n));
    if (n % kCheckEvery == 0) STTRY(check_level<T>(p, slot_of(n), s));  // level n is complete
  }
  if (n1 > n0) STTRY(finish<T>(p, S, false, slot_of(n1 - 1), slot_of(n1), fwd_par(n1), s));
  if (n1 > n0) STTRY(check_level<T>(p, slot_of(n1), s));
  if (ub && n1 > n0) STTRY(record(n1));
  if (traces && n1 >= 1) {
    for (int64_t sh = 0; sh < ns; ++sh) {
      T* un = slot_of(n1) + sh * p->ls;
      T* out = traces + sh * p->nt * p->rec.npts + (n1 - 1) * p->rec.npts;
      STTRY(probed(p, 4, s, [&](hipEvent_t e0, hipEvent_t e1) {
        return launch_sample<T>(un, p->rec.s_dof, (const T*)p->rec.s_w, p->rec.npts, m.nd, out, s, e0, e1);
      }));
    }
  }
  return OK;
}

// c^2 at the DOFs and its copies per shared ref.
template <typename T>
Status set_c2(Problem* p, const double* c, hipStream_t s) {
  const Mesh& m = *p->mesh;
  HIPTRY(launch_square<T>(c, (T*)p->d_c2, m.n_dofs, s));
  HIPTRY(launch_gather<T>((const T*)p->d_c2, p->d_sh_idx, (T*)p->d_c2_ref, p->nref, s));
  if (p->absorb)
    HIPTRY(launch_absorb_coef<T>(c, p->nbd, p->d_bnd_dof, p->d_bnd_coef, (T*)p->d_beta, (T*)p->d_gamma, p->nbr,
                                 p->d_bnd_ref, (T*)p->d_beta_ref, (T*)p->d_gamma_ref, s));
  return OK;
}

// PML on tetrahedra: defined after the stiffness apply they use.
template <typename T>
Status pml3_forward(Problem* p, const double* c, T* traces, bool keep, hipStream_t s);
template <typename T>
Status pml3_reverse(Problem* p, const T* adj_rows, bool grad, T* lambda_out, T* src_trace, hipStream_t s);

// The forward sweep with its two level buffers at base (level n in buffer n & 1).
template <typename T>
Status forward_run(Problem* p, const double* c, T* traces, T* base, hipStream_t s) {
  const int64_t lvl = p->ls * p->nshot;
  STTRY(clear_flag(p, s));
  STTRY(set_c2<T>(p, c, s));
  STTRY(zero_level<T>(p, p->fwd, base, 0, s));
  STTRY(zero_pml<T>(p, 0, s));
  return run_forward<T>(p, 0, p->nt, [base, lvl](int64_t n) { return base + (n & 1) * lvl; }, traces, false,
                        s);
}

template <typename T>
Status forward_t(Problem* p, const double* c, T* traces, hipStream_t s) {
  if (p->pml3) return pml3_forward<T>(p, c, traces, false, s);
  STTRY(ensure_slots(p, 2));
  return forward_run<T>(p, c, traces, slot_ptr<T>(p, 0), s);
}

// Workspace of the allocation-free forward (kmv_forward_noalloc): its two level
// buffers.  Each device holds its own copy for the life of the process; host code
// uses the address from hipGetSymbolAddress, taken once per device at set-up.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The step kernels' dynamic-LDS limit is an attribute of the kernel function, shared
// by every problem on the device: it is only raised (a problem with a smaller footprint
// must not lower it under the launches of another), one caller at a time, and not set
// again once it covers the request.  The device must be current.
std::mutex g_lds_mu;
std::map<std::tuple<int, int, int, int, bool, bool>, size_t> g_lds_limit;

hipError_t raise_lds_limit(int device, int prec, int dim, int nd, bool adjoint, size_t bytes, bool pml) {
  std::lock_guard<std::mutex> lk(g_lds_mu);
  size_t& cur = g_lds_limit[std::make_tuple(device, prec, dim, nd, adjoint, pml)];
  if (bytes <= cur) return hipSuccess;
  const hipError_t e = prec == KMV_FP64 ? set_step_lds_limit<double>(dim, nd, adjoint, (int)bytes, pml)
                                        : set_step_lds_limit<float>(dim, nd, adjoint, (int)bytes, pml);
  if (e == hipSuccess) cur = bytes;
  return e;
}

// Address of this device's workspace (the device must be current).
Status scratch_ptr(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return Status{KMV_EDEVICE, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return Status{KMV_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return OK;
}

Status plan_storage(Problem* p) {
  const Mesh& m = *p->mesh;
  const size_t vb = (size_t)p->ls * p->nshot * p->ts;
  const size_t all = (size_t)(p->nt + 1) * vb;
  p->store_sub = false;
  if (p->grad_every > 1 && p->ckpt_every == 0) {  // keep every r-th state only
    const int64_t nsub = p->nt / p->grad_every + 1;
    if ((size_t)(2 + nsub) * vb <= p->budget) {
      p->store_all = false;
      p->store_sub = true;
      p->seg = p->nt;
      p->n_ck = 0;
      return ensure_slots(p, 2 + nsub);
    }
  }
  if (p->ckpt_every == 0 && all <= p->budget) {
    p->store_all = true;
    p->seg = p->nt;
    p->n_ck = 0;
    return ensure_slots(p, p->nt + 1);
  }
  p->store_all = false;
  int64_t seg = p->ckpt_every > 0 ? p->ckpt_every
                                   : std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt(2.0 * p->nt)));
  seg = std::min(seg, p->nt);
  const int64_t nck = (p->nt + seg - 1) / seg;
  const size_t need = (size_t)(seg + 1) * vb + 2 * (size_t)nck * vb;
  if (need > p->budget && p->ckpt_every <= 0)
    return Status{KMV_ENOMEM, "checkpoint storage (" + std::to_string(need) + " B) exceeds mem_budget"};
  if (p->seg != seg || p->n_ck != nck || !p->d_ck_u) {
    STTRY(alloc(&p->d_ck_u, (size_t)nck * vb));
    STTRY(alloc(&p->d_ck_du, (size_t)nck * (m.n_dofs + p->rs) * p->nshot * p->ts));
  }
  p->seg = seg;
  p->n_ck = nck;
  return ensure_slots(p, seg + 1);
}

// Adjoint level lvl's vector: the two buffers by parity, or slot lvl % lam_k of the ring.
template <typename T>
T* lam_ptr(Problem* p, int64_t lvl) {
  if (p->lam_k > 2) return (T*)p->d_lam_ring + (lvl % p->lam_k) * p->ls * p->nshot;
  return (T*)p->d_lam[lvl & 1];
}

// One reverse launch m (lambda^{m+1} -> lambda^m, finishing level m+1 from level m+2);
// uf = u^m when grad.
template <typename T>
Status adjoint_launch(Problem* p, int64_t m, bool grad, const T* adj_rows, const T* uf, hipStream_t s) {
  const double inv_dt2 = 1.0 / (p->dt * p->dt);
  return step<T>(p, p->adj, grad, m != p->nt, lam_ptr<T>(p, m + 1), lam_ptr<T>(p, m + 2), lam_ptr<T>(p, m),
                 adj_par(m), &p->rec, adj_rows + (m - 1) * p->rec.npts, 1, p->nt * p->rec.npts, (T)inv_dt2, uf,
                 nullptr, s);
}

template <typename T>
Status adjoint_start(Problem* p, hipStream_t s) {
  STTRY(zero_pml<T>(p, 1, s));
  STTRY(zero_level<T>(p, p->adj, lam_ptr<T>(p, p->nt + 1), (int)((p->nt + 1) & 1), s));
  HIPTRY(launch_fill<T>(lam_ptr<T>(p, p->nt), T(0), p->ls * p->nshot, s));
  if (p->lam_k > 2) HIPTRY(launch_fill<T>(lam_ptr<T>(p, p->nt + 2), T(0), p->ls * p->nshot, s));
  return OK;
}

// After launch 1: finish lambda^1 (level 1) from level 2 and launch 1's partials.
template <typename T>
Status adjoint_end(Problem* p, bool grad, hipStream_t s) {
  return finish<T>(p, p->adj, grad, lam_ptr<T>(p, 2), lam_ptr<T>(p, 1), adj_par(0), s);
}

template <typename T>
Status misfit_gradient_t(Problem* p, const double* c, const T* obs, double* J, double* grad, T* traces_out,
                         hipStream_t s, bool accumulate) {
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  if (p->pml3) {  // tetrahedra: every level of u and omega kept, then the reverse sweep
    const size_t need = (size_t)(p->nt + 1) * ((size_t)p->ls + (size_t)N) * p->ts;
    if (need > p->budget)
      return Status{KMV_ENOMEM, "with the PML on tetrahedra every forward level of u and omega is kept: " +
                                    std::to_string(need) + " B exceed mem_budget"};
    T* traces = traces_out ? traces_out : (T*)p->d_traces_tmp;
    STTRY(pml3_forward<T>(p, c, traces, true, s));
    HIPTRY(launch_misfit<T>(traces, obs, (T*)p->d_resid, p->nt * p->rec.npts, p->d_red, p->red_blocks,
                            p->d_red + p->red_blocks, s));
    STTRY(pml3_reverse<T>(p, (const T*)p->d_resid, true, nullptr, nullptr, s));
    HIPTRY(launch_finalize_grad(c, p->d_gacc, 1, 2.0 * p->dt * p->dt * (double)p->grad_every, grad, N, s,
                                accumulate));
    double hJ = 0;
    int flag = 0;
    HIPTRY(hipMemcpyAsync(&hJ, p->d_red + p->red_blocks, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPTRY(hipMemcpyAsync(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    *J = accumulate ? *J + hJ : hJ;
    if (flag || !std::isfinite(hJ)) return classify_nonfinite<T>(p, s);
    return OK;
  }
  STTRY(plan_storage(p));
  if (p->pml() && !p->store_all && !p->store_sub)
    return Status{KMV_ENOMEM, "with the PML the forward states must be kept (all of them, or every r-th with "
                              "gradient_every = r): they do not fit mem_budget, and recomputing from "
                              "checkpoints does not carry the auxiliary fields"};
  T* traces = traces_out ? traces_out : (T*)p->d_traces_tmp;
  STTRY(clear_flag(p, s));
  STTRY(set_c2<T>(p, c, s));
  STTRY(zero_pml<T>(p, 0, s));
  const int64_t r = p->grad_every;
  auto sub_slot = [p, r](int64_t n) { return n % r == 0 ? slot_ptr<T>(p, 2 + n / r) : slot_ptr<T>(p, n & 1); };
  STTRY(zero_level<T>(p, p->fwd, p->store_sub ? sub_slot(0) : slot_ptr<T>(p, 0), 0, s));
  // absorbing boundary: u^n and lambda^n at the boundary DOFs, every level
  T *ub = nullptr, *lb = nullptr;
  if (p->absorb && p->nbd > 0) {
    const size_t rec = (size_t)p->nshot * (p->nt + 1) * p->nbd * sizeof(T);
    if (p->bnd_rec_bytes != rec || !p->d_ub) {
      STTRY(alloc(&p->d_ub, rec));
      STTRY(alloc(&p->d_lb, rec));
      p->bnd_rec_bytes = rec;
    }
    ub = (T*)p->d_ub;
    lb = (T*)p->d_lb;
  }
  if (p->store_all) {  // every level stays in its slot: one gather for all of them
    STTRY(run_forward<T>(p, 0, p->nt, [p](int64_t n) { return slot_ptr<T>(p, n); }, traces, false, s));
    if (ub)
      HIPTRY(launch_gather_levels<T>(slot_ptr<T>(p, 0), p->ls * p->nshot, p->ls, p->nshot, p->nt + 1, p->nbd,
                                     p->d_bnd_dof, ub, s));
  } else if (p->store_sub) {
    STTRY(run_forward<T>(p, 0, p->nt, sub_slot, traces, false, s, ub));
  } else {
    STTRY(run_forward<T>(p, 0, p->nt, [p](int64_t n) { return slot_ptr<T>(p, n & 1); }, traces, true, s, ub));
  }
  // lambda^lvl is complete once reverse launch lvl-1 has run (lambda^1 after the end).
  // The ring keeps lam_k levels, so complete levels lo..top are recorded in one launch
  // just before the oldest of them would be overwritten.
  if (lb && p->lam_k != kLamRing) {
    STTRY(alloc(&p->d_lam_ring, (size_t)kLamRing * p->ls * p->nshot * sizeof(T)));
    p->lam_k = kLamRing;
  }
  int64_t lam_top = p->nt;  // highest level not yet recorded
  auto record_lam = [&](int64_t lo) -> Status {  // levels lo..lam_top are complete
    if (!lb || lo > lam_top) return OK;
    HIPTRY(launch_gather_ring<T>(lam_ptr<T>(p, 0), p->lam_k, p->ls * p->nshot, p->ls, p->nshot, lo,
                                 (int)(lam_top - lo + 1), p->nbd, p->d_bnd_dof, lb, (p->nt + 1) * p->nbd, s));
    lam_top = lo - 1;
    return OK;
  };
  HIPTRY(launch_misfit<T>(traces, obs, (T*)p->d_resid, p->nt * p->rec.npts * p->nshot, p->d_red,
                          p->red_blocks, p->d_red + p->red_blocks, s));
  STTRY(adjoint_start<T>(p, s));
  HIPTRY(launch_fill_f64(p->d_gacc, 0.0, N * p->nshot, s));
  const T* resid = (const T*)p->d_resid;
  // reverse launch mm pairs lambda^{mm+1} with u^mm when mm % r == 0 (every launch
  // for r = 1); with r > 1 the shared DOFs' pairing partials are finished at once
  auto reverse = [&](int64_t mm, const T* uf) -> Status {
    const bool g = mm % r == 0;
    STTRY(adjoint_launch<T>(p, mm, g, resid, g ? uf : nullptr, s));
    if (g && r > 1) STTRY(pair_finish<T>(p, adj_par(mm), s));
    if ((mm + 1) % kCheckEvery == 0) STTRY(check_level<T>(p, lam_ptr<T>(p, mm + 1), s));  // complete now
    // the next launch overwrites level mm + lam_k - 1
    if (lb && (lam_top >= mm + kLamRing - 1 || mm == 1)) STTRY(record_lam(mm + 1));
    return OK;
  };
  if (p->store_all) {
    for (int64_t mm = p->nt; mm >= 1; --mm) STTRY(reverse(mm, slot_ptr<T>(p, mm)));
  } else if (p->store_sub) {
    for (int64_t mm = p->nt; mm >= 1; --mm) STTRY(reverse(mm, sub_slot(mm)));
  } else {
    const int64_t ns = p->nshot;
    const size_t lb = (size_t)(p->ls * ns) * sizeof(T);
    const size_t ob = (size_t)(m.n_dofs * ns) * sizeof(T), shb = (size_t)(p->rs * ns) * sizeof(T);
    for (int64_t k = p->n_ck - 1; k >= 0; --k) {
      const int64_t s0 = k * p->seg, s1 = std::min(s0 + p->seg, p->nt);
      const T* cd = (const T*)p->d_ck_du + k * (m.n_dofs + p->rs) * ns;
      HIPTRY(hipMemcpyAsync(slot_ptr<T>(p, 0), (T*)p->d_ck_u + k * p->ls * ns, lb, hipMemcpyDeviceToDevice, s));
      HIPTRY(hipMemcpyAsync(p->fwd.d, cd, ob, hipMemcpyDeviceToDevice, s));
      HIPTRY(hipMemcpyAsync(p->fwd.dsh[s0 & 1], cd + m.n_dofs * ns, shb, hipMemcpyDeviceToDevice, s));
      STTRY(run_forward<T>(p, s0, s1, [p, s0](int64_t n) { return slot_ptr<T>(p, n - s0); }, (T*)nullptr,
                           false, s));
      for (int64_t mm = s1; mm > s0; --mm) STTRY(reverse(mm, slot_ptr<T>(p, mm - s0)));
    }
  }
  STTRY(adjoint_end<T>(p, r == 1, s));
  STTRY(check_level<T>(p, lam_ptr<T>(p, 1), s));
  STTRY(record_lam(1));
  HIPTRY(launch_finalize_grad(c, p->d_gacc, p->nshot, 2.0 * p->dt * p->dt * (double)r, grad, N, s, accumulate));
  if (lb) {
    const int chunks = (int)std::min<int64_t>(kBndChunks, p->nt);
    if (!p->d_bnd_part) STTRY(alloc((void**)&p->d_bnd_part, (size_t)kBndChunks * p->nbd * sizeof(double)));
    HIPTRY(launch_absorb_grad<T>(ub, lb, p->nt, p->nbd, p->nshot, p->d_bnd_dof, p->d_bnd_hb, p->d_bnd_part,
                                 chunks, grad, s));
  }
  double hJ = 0;
  int flag = 0;
  HIPTRY(hipMemcpyAsync(&hJ, p->d_red + p->red_blocks, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(hipMemcpyAsync(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  *J = accumulate ? *J + hJ : hJ;
  if (flag || !std::isfinite(hJ)) return classify_nonfinite<T>(p, s);
  return OK;
}

// The forward sweep and the float64 misfit only (no stored states, no adjoint).
template <typename T>
Status misfit_t(Problem* p, const double* c, const T* obs, double* J, T* traces_out, hipStream_t s) {
  T* traces = traces_out ? traces_out : (T*)p->d_traces_tmp;
  STTRY(forward_t<T>(p, c, traces, s));
  HIPTRY(launch_misfit<T>(traces, obs, (T*)p->d_resid, p->nt * p->rec.npts * p->nshot, p->d_red,
                          p->red_blocks, p->d_red + p->red_blocks, s));
  double hJ = 0;
  int flag = 0;
  HIPTRY(hipMemcpyAsync(&hJ, p->d_red + p->red_blocks, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(hipMemcpyAsync(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  *J = hJ;
  if (flag || !std::isfinite(hJ)) return classify_nonfinite<T>(p, s);
  return OK;
}

template <typename T>
Status adjoint_t(Problem* p, const double* c, const T* adj, T* lambda_out, T* src_trace, hipStream_t s) {
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  const size_t vb = (size_t)N * sizeof(T);
  STTRY(clear_flag(p, s));
  STTRY(set_c2<T>(p, c, s));
  if (p->pml3) return pml3_reverse<T>(p, adj, false, lambda_out, src_trace, s);
  STTRY(adjoint_start<T>(p, s));
  if (lambda_out) HIPTRY(launch_fill<T>(lambda_out + p->nt * N, T(0), N, s));
  // shot sh samples its own sources: points [sh*nps, (sh+1)*nps) of the table
  const int nps = p->src.npts / p->nshot;
  auto record = [&](int64_t lvl) -> Status {  // level lvl is complete: row lvl-1
    const T* lam = lam_ptr<T>(p, lvl);
    if (lambda_out) HIPTRY(hipMemcpyAsync(lambda_out + (lvl - 1) * N, lam, vb, hipMemcpyDeviceToDevice, s));
    if (src_trace)
      for (int sh = 0; sh < p->nshot; ++sh) {
        const size_t o = (size_t)sh * nps * m.nd;
        STTRY(probed(p, 4, s, [&](hipEvent_t e0, hipEvent_t e1) {
          return launch_sample<T>(lam + sh * p->ls, p->src.s_dof + o, (const T*)p->src.s_w + o, nps, m.nd,
                                  src_trace + (sh * p->nt + lvl - 1) * nps, s, e0, e1);
        }));
      }
    return OK;
  };
  for (int64_t mm = p->nt; mm >= 1; --mm) {
    STTRY(adjoint_launch<T>(p, mm, false, adj, nullptr, s));
    if (mm + 1 <= p->nt) STTRY(record(mm + 1));
    if ((mm + 1) % kCheckEvery == 0) STTRY(check_level<T>(p, lam_ptr<T>(p, mm + 1), s));
  }
  STTRY(adjoint_end<T>(p, false, s));
  STTRY(check_level<T>(p, lam_ptr<T>(p, 1), s));
  return record(1);
}

template <typename T>
Status apply_t(Problem* p, const double* c, const T* u, T* y, hipStream_t s) {
  const Mesh& m = *p->mesh;
  if (c) STTRY(set_c2<T>(p, c, s));
  StepArgs<T> a = base_args<T>(p);
  a.mode = 1;
  a.prev = 0;
  a.n_shots = 1;  // one vector
  a.u_in = u;
  a.y_out = y;
  // loaded (not used) by the branch-free prologue: any valid buffers
  a.du = y;
  a.u_prev = (const T*)p->d_lam[0];  // any level vector: the apply input has no ref copies
  a.dsh_prev = (const T*)p->fwd.dsh[0];
  a.part_prev = (const T*)p->fwd.part[1];
  a.part_cur = (T*)p->fwd.part[0];
  STTRY(probed(p, 0, s, [&](hipEvent_t e0, hipEvent_t e1) {
    return launch_step<T>(m.dim, m.nd, false, a, (int)m.n_patches, p->block, s, e0, e1);
  }));
  FinishArgs<T> f{};
  f.n_own = m.n_own_total;
  f.n_shared = m.n_shared;
  f.n_dofs = m.n_dofs;
  f.shp_ptr = p->d_shp_ptr;
  f.shp_slot = p->d_shp_slot;
  f.mode = 1;
  f.n_shots = 1;
  f.part_prev = (const T*)p->fwd.part[0];
  f.y_out = y;
  return probed(p, 2, s,
                [&](hipEvent_t e0, hipEvent_t e1) { return launch_finish<T>(false, f, s, e0, e1); });
}

// ---- PML on tetrahedra (section on the PML: p_x, p_y, p_z and omega; the
// transposed scheme of the adjoint; the gradient's PML terms).  The layer's terms
// run beside the stiffness apply (pml3d.hip): per step the apply K u, the per-cell
// pass, the per-DOF update rows and the receivers' samples.  Every level is complete
// at the end of its step (no lagged finishing).

// The source's nodal load vector and the transposed receiver rows (DOF -> receiver,
// weight), rebuilt after the sources or receivers change.
Status pml3_points(Problem* p) {
  if (!p->p3_points_dirty) return OK;
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  const int nd = m.nd;
  std::vector<double> sv(N, 0.0);
  for (size_t k = 0; k < p->src.h_dof.size(); ++k) sv[p->src.h_dof[k]] += p->src.h_w[k];
  const int nr = p->rec.npts;
  std::vector<int32_t> ptr(N + 1, 0), idx((size_t)nr * nd);
  std::vector<double> w((size_t)nr * nd);
  for (int j = 0; j < nr; ++j)
    for (int a = 0; a < nd; ++a) ptr[p->rec.h_dof[(size_t)j * nd + a] + 1]++;
  for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int j = 0; j < nr; ++j)  // per DOF, receivers in ascending order
    for (int a = 0; a < nd; ++a) {
      const int32_t i = p->rec.h_dof[(size_t)j * nd + a];
      idx[fill[i]] = j;
      w[fill[i]++] = p->rec.h_w[(size_t)j * nd + a];
    }
  STTRY(upload_real(&p->d_svec, sv, p->prec));
  STTRY(upload_i(&p->d_rptr, ptr));
  STTRY(upload_i(&p->d_ridx, idx.empty() ? std::vector<int32_t>{0} : idx));
  STTRY(upload_real(&p->d_rw, w.empty() ? std::vector<double>{0.0} : w, p->prec));
  p->p3_points_dirty = false;
  return OK;
}

template <typename T>
Pml3CellArgs<T> pml3_cell_args(Problem* p) {
  const Mesh& m = *p->mesh;
  Pml3CellArgs<T> a;
  a.n_cells = m.n_cells;
  a.n_dofs = m.n_dofs;
  a.cdof = p->d_cdof;
  a.cpos = p->d_cpos;
  a.b3 = (const T*)p->d_b3;
  a.geom = (const T*)p->d_geom;
  a.c2 = (const T*)p->d_c2;
  a.sig = (const T*)p->d_sig;
  a.out = (T*)p->d_cellout;
  return a;
}

template <typename T>
Pml3UpdateArgs<T> pml3_update_args(Problem* p) {
  const Mesh& m = *p->mesh;
  Pml3UpdateArgs<T> a;
  a.n_dofs = m.n_dofs;
  a.n_slots = m.n_cells * m.nd;
  a.csr_ptr = p->d_csr_ptr;
  a.cell_out = (const T*)p->d_cellout;
  a.sig = (const T*)p->d_sig;
  a.mass = (const T*)p->d_mass;
  a.c2 = (const T*)p->d_c2;
  a.dt = (T)p->dt;
  a.ku = (const T*)p->d_ku;
  return a;
}

// Forward levels n = 0..N_t from zero (u^{-1} = u^0 = 0, p and omega zero): keep =
// every level of u (slot n) and omega stays, else two of each.  traces: row n-1 =
// P u^n.
template <typename T>
Status pml3_forward(Problem* p, const double* c, T* traces, bool keep, hipStream_t s) {
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  STTRY(pml3_points(p));
  const int64_t nl = keep ? p->nt + 1 : 2;
  STTRY(ensure_slots(p, nl));
  if (p->n_y3 < nl) {
    STTRY(alloc(&p->d_y3, (size_t)nl * N * p->ts));
    p->n_y3 = nl;
  }
  auto U = [&](int64_t n) { return slot_ptr<T>(p, keep ? n : (n & 1)); };
  auto Y = [&](int64_t n) { return (T*)p->d_y3 + (keep ? n : (n & 1)) * N; };
  STTRY(clear_flag(p, s));
  STTRY(set_c2<T>(p, c, s));
  HIPTRY(launch_fill<T>(U(0), T(0), N, s));
  HIPTRY(launch_fill<T>(Y(0), T(0), N, s));
  for (int k = 0; k < 2; ++k) HIPTRY(launch_fill<T>((T*)p->d_p3[k], T(0), 3 * N, s));
  Pml3CellArgs<T> ca = pml3_cell_args<T>(p);
  Pml3UpdateArgs<T> ua = pml3_update_args<T>(p);
  ua.svec = (const T*)p->d_svec;
  for (int64_t n = 0; n < p->nt; ++n) {
    STTRY(apply_t<T>(p, nullptr, U(n), (T*)p->d_ku, s));
    ca.u = U(n);
    ca.y = Y(n);
    ca.p = (const T*)p->d_p3[n & 1];  // p^n; p^{n-1} in the other buffer
    HIPTRY(launch_pml3_cell<T>(m.nd, false, ca, s));
    ua.u = U(n);
    ua.u_prev = n > 0 ? U(n - 1) : nullptr;
    ua.y = Y(n);
    ua.u_out = U(n + 1);
    ua.y_out = Y(n + 1);
    ua.p_io = (T*)p->d_p3[(n + 1) & 1];  // p^{n-1} in, p^{n+1} out
    ua.amp = (const T*)p->d_wavelet + n;
    HIPTRY(launch_pml3_update<T>(false, ua, s));
    if (traces)
      STTRY(probed(p, 4, s, [&](hipEvent_t e0, hipEvent_t e1) {
        return launch_sample<T>(U(n + 1), p->rec.s_dof, (const T*)p->rec.s_w, p->rec.npts, m.nd,
                                traces + n * p->rec.npts, s, e0, e1);
      }));
    if ((n + 1) % kCheckEvery == 0 || n + 1 == p->nt) STTRY(check_level<T>(p, U(n + 1), s));
  }
  return OK;
}

// Reverse levels m = N_t..1 from lambda^{N_t+1} = lambda^{N_t+2} = 0 (mu, nu zero)
// with adjoint data adj_rows (row m-1 = y^m per receiver).  grad: the float64
// accumulator gains the pairing of lambda^{m+1} with u^m and the PML terms at the
// steps m % r == 0 (u^m, omega^m from the kept forward levels).  lambda_out (row
// m-1 = lambda^m, row N_t = 0) and src_trace (row m-1 = lambda^m at the sources)
// are optional.
template <typename T>
Status pml3_reverse(Problem* p, const T* adj_rows, bool grad, T* lambda_out, T* src_trace, hipStream_t s) {
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  const size_t vb = (size_t)N * sizeof(T);
  STTRY(pml3_points(p));
  auto L = [&](int64_t lvl) { return (T*)p->d_lam[lvl & 1]; };
  for (int k = 0; k < 2; ++k) {
    HIPTRY(launch_fill<T>((T*)p->d_lam[k], T(0), N, s));
    HIPTRY(launch_fill<T>((T*)p->d_p3[k], T(0), 3 * N, s));
    HIPTRY(launch_fill<T>((T*)p->d_nu3[k], T(0), N, s));
  }
  if (grad) HIPTRY(launch_fill_f64(p->d_gacc, 0.0, N, s));
  if (lambda_out) HIPTRY(launch_fill<T>(lambda_out + p->nt * N, T(0), N, s));
  Pml3CellArgs<T> ca = pml3_cell_args<T>(p);
  Pml3UpdateArgs<T> ua = pml3_update_args<T>(p);
  ua.rec_ptr = p->d_rptr;
  ua.rec_idx = p->d_ridx;
  ua.rec_w = (const T*)p->d_rw;
  const int64_t r = p->grad_every;
  for (int64_t mm = p->nt; mm >= 1; --mm) {
    const bool pair = grad && mm % r == 0;
    STTRY(apply_t<T>(p, nullptr, L(mm + 1), (T*)p->d_ku, s));
    ca.u = L(mm + 1);
    ca.p = (const T*)p->d_p3[(mm + 1) & 1];  // mu^{m+1}
    ca.uf = pair ? slot_ptr<T>(p, mm) : nullptr;
    ca.yf = pair ? (const T*)p->d_y3 + mm * N : nullptr;
    HIPTRY(launch_pml3_cell<T>(m.nd, true, ca, s));
    ua.u = L(mm + 1);
    ua.u_prev = L(mm);  // lambda^{m+2} in, lambda^m out: the same buffer
    ua.u_out = L(mm);
    ua.y = (const T*)p->d_nu3[(mm + 1) & 1];
    ua.y_out = (T*)p->d_nu3[mm & 1];
    ua.p_in = (const T*)p->d_p3[(mm + 1) & 1];
    ua.p_io = (T*)p->d_p3[mm & 1];  // mu^{m+2} in, mu^m out
    ua.resid_row = adj_rows + (mm - 1) * p->rec.npts;
    ua.gacc = pair ? p->d_gacc : nullptr;
    HIPTRY(launch_pml3_update<T>(true, ua, s));
    if (lambda_out) HIPTRY(hipMemcpyAsync(lambda_out + (mm - 1) * N, L(mm), vb, hipMemcpyDeviceToDevice, s));
    if (src_trace)
      STTRY(probed(p, 4, s, [&](hipEvent_t e0, hipEvent_t e1) {
        return launch_sample<T>(L(mm), p->src.s_dof, (const T*)p->src.s_w, p->src.npts, m.nd,
                                src_trace + (mm - 1) * p->src.npts, s, e0, e1);
      }));
    if (mm % kCheckEvery == 0 || mm == 1) STTRY(check_level<T>(p, L(mm), s));
  }
  return OK;
}

// SplitMix64 (Steele, Lea and Flood, 2014): one step of the generator's output map.
uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

template <typename T>
Status spectral_t(Problem* p, const double* c, int iters, uint64_t seed, double* rho, hipStream_t s) {
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  // Start vector: a standard normal per DOF drawn from a counter-based hash of the
  // seed and the DOF's coordinates, so the iteration does not depend on the
  // library's internal DOF numbering.
  std::vector<T> v0(N);
  std::vector<double> tmp(N);
  double nrm = 0;
  for (int64_t i = 0; i < N; ++i) {
    uint64_t h = splitmix64(seed);
    for (int r = 0; r < m.dim; ++r)
      h = splitmix64(h ^ (uint64_t)std::llround(m.dof_coords[i * m.dim + r] * 1073741824.0));
    const uint64_t h2 = splitmix64(h);
    const double u1 = ((double)(h >> 11) + 0.5) * 0x1.0p-53, u2 = (double)(h2 >> 11) * 0x1.0p-53;
    tmp[i] = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    nrm += tmp[i] * tmp[i];
  }
  for (int64_t i = 0; i < N; ++i) v0[i] = (T)(tmp[i] / std::sqrt(nrm));
  void *v = nullptr, *w = nullptr, *y = nullptr;
  auto cleanup = [&]() {
    dfree(v);
    dfree(w);
    dfree(y);
  };
  Status st = upload(&v, v0.data(), N);
  if (st.code == KMV_OK) st = alloc(&w, N * sizeof(T));
  if (st.code == KMV_OK) st = alloc(&y, N * sizeof(T));
  if (st.code != KMV_OK) {
    cleanup();
    return st;
  }
  STTRY(set_c2<T>(p, c, s));
  const T* ms = (const T*)p->d_minv_sqrt;
  double* dots = p->d_red + p->red_blocks + 1;  // [2]
  for (int it = 0; it < iters; ++it) {
    HIPTRY(launch_scale<T>((const T*)v, ms, (T*)w, N, s));
    STTRY(apply_t<T>(p, nullptr, (const T*)w, (T*)y, s));
    HIPTRY(launch_scale<T>((const T*)y, ms, (T*)w, N, s));
    HIPTRY(launch_dot<T>((const T*)v, (const T*)w, N, p->d_red, p->red_blocks, dots, s));
    HIPTRY(launch_dot<T>((const T*)w, (const T*)w, N, p->d_red, p->red_blocks, dots + 1, s));
    HIPTRY(launch_normalize<T>((T*)v, (const T*)w, dots + 1, N, s));
  }
  double h = 0;
  HIPTRY(hipMemcpyAsync(&h, dots, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  cleanup();
  *rho = h;
  return OK;
}

void free_sweep(Sweep& S) {
  for (void* q : {S.d, S.dsh[0], S.dsh[1], S.part[0], S.part[1], S.partr[0], S.partr[1]}) dfree(q);
  S = Sweep();
}

Status alloc_sweep(Sweep& S, const Mesh& m, size_t ts, bool with_r, int nshot) {
  const size_t rb = std::max<size_t>(1, m.n_shared_refs) * nshot * ts;
  STTRY(alloc(&S.d, (size_t)m.n_dofs * nshot * ts));
  for (int i = 0; i < 2; ++i) {
    STTRY(alloc(&S.dsh[i], rb));
    STTRY(alloc(&S.part[i], rb));
    if (with_r) STTRY(alloc(&S.partr[i], rb));
  }
  return OK;
}

}  // namespace

Problem::~Problem() {
  for (void* q : {(void*)d_lmap, d_geom, (void*)d_cell_start, (void*)d_own_start, (void*)d_sh_start,
                  (void*)d_sh_idx, (void*)d_shp_ptr, (void*)d_shp_slot, (void*)d_ref_slots, (void*)d_gword,
                  (void*)d_glist, (void*)d_gword_off, (void*)d_glist_off, (void*)d_damp_patch, d_gamma, d_gdet, d_beta, d_c2, d_c2_ref, d_gamma_ref, d_beta_ref, d_minv_sqrt, d_lam[0], d_lam[1], d_lam_ring, (void*)d_gacc, (void*)d_red, (void*)d_flag, d_slots,
                  d_ck_u, d_ck_du, d_resid, d_traces_tmp, d_wavelet, (void*)d_bnd_dof, (void*)d_bnd_ref,
                  (void*)d_bnd_coef, (void*)d_bnd_hb, d_ub, d_lb, (void*)d_bnd_part, d_sig, d_sig_ref, d_pml_b,
                  (void*)d_list[0], (void*)d_list[1], d_pp[0][0], d_pp[0][1], d_pp[1][0], d_pp[1][1], d_pt[0][0],
                  d_pt[0][1], d_pt[1][0], d_pt[1][1], (void*)d_cdof, d_b3, (void*)d_csr_ptr, (void*)d_cpos,
                  d_mass, d_cellout, d_ku, d_p3[0], d_p3[1], d_nu3[0], d_nu3[1], d_y3, d_svec, (void*)d_rptr,
                  (void*)d_ridx, d_rw})
    dfree(q);
  free_sweep(fwd);
  free_sweep(adj);
  free_points(src);
  free_points(rec);
  for (auto& q : probe.pending) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (hipEvent_t e : probe.pool) (void)hipEventDestroy(e);
}

Status profile_enable(Problem* p, int every) {
  DeviceGuard dg(p->device);
  if (every < 0) return Status{KMV_EINVAL, "every must be >= 0"};
  STTRY(resolve_probe(p));
  Probe& pr = p->probe;
  pr.every = every;
  for (int v = 0; v < Probe::kVariants; ++v) {
    pr.launches[v] = 0;
    pr.timed[v] = 0;
    pr.total_ms[v] = 0;
  }
  return OK;
}

Status profile_read(Problem* p, int variant, int64_t* launches, int64_t* timed, double* mean_ms) {
  DeviceGuard dg(p->device);
  if (variant < 0 || variant >= Probe::kVariants) return Status{KMV_EINVAL, "variant out of range"};
  STTRY(resolve_probe(p));
  const Probe& pr = p->probe;
  if (launches) *launches = pr.launches[variant];
  if (timed) *timed = pr.timed[variant];
  if (mean_ms) *mean_ms = pr.timed[variant] ? pr.total_ms[variant] / pr.timed[variant] : 0.0;
  return OK;
}

Status problem_create(Mesh* m, int prec, double dt, int64_t nt, int64_t ckpt_every, size_t budget,
                      int n_shots, int64_t grad_every, Problem** out) {
  if (prec != KMV_FP64 && prec != KMV_FP32) return Status{KMV_EINVAL, "precision must be KMV_FP64 or KMV_FP32"};
  if (!(dt > 0) || nt <= 0) return Status{KMV_EINVAL, "dt and n_steps must be positive"};
  if (n_shots < 1 || n_shots > 1024 || (int64_t)n_shots * m->n_patches > INT32_MAX)
    return Status{KMV_EINVAL, "n_shots must be in 1..1024"};
  if (grad_every < 1) return Status{KMV_EINVAL, "gradient_every must be >= 1"};
  if (m->max_patch_cells > 256) return Status{KMV_EINVAL, "patches larger than 256 cells"};
  auto p = new Problem();
  std::unique_ptr<Problem> guard(p);
  p->mesh = m;
  p->prec = prec;
  p->ts = prec == KMV_FP64 ? 8 : 4;
  p->dt = dt;
  p->nt = nt;
  p->ckpt_every = ckpt_every;
  p->budget = budget ? budget : ((size_t)8 << 30);
  HIPTRY(hipGetDevice(&p->device));
  p->block = step_block(m->max_patch_cells);
  p->nref = m->n_shared_refs;
  p->rs = std::max<int64_t>(1, p->nref);
  // a level vector: its DOFs, then a copy per shared ref; at least one such place, so
  // that the step kernel's clamped ref loads (index 0 when the mesh has a single
  // patch and no refs) stay inside every level buffer
  p->ls = m->n_dofs + p->rs;
  p->nshot = n_shots;
  p->grad_every = grad_every;
  for (bool adjv : {false, true}) {
    const size_t bytes = step_lds_bytes(m->dim, m->nd, m->max_nbl, m->slot_stride, m->nb, m->max_glist, adjv, p->ts);
    if (bytes > 160 * 1024)
      return Status{KMV_EINVAL, "patch LDS footprint of " + std::to_string((bytes + 1023) / 1024) +
                                    " KiB above the 160 KiB of a CU; use smaller patches (patch_cells)"};
    if (bytes > 64 * 1024) HIPTRY(raise_lds_limit(p->device, prec, m->dim, m->nd, adjv, bytes, false));
  }
  {
    // local indices of node pairs (2q, 2q+1) of a cell packed in one 32-bit word, SoA
    const int nb2 = (m->nb + 1) / 2;
    std::vector<uint32_t> lm2((size_t)std::max(nb2, 1) * m->n_cells, 0);
    for (int q = 0; q < nb2; ++q)
      for (int64_t e = 0; e < m->n_cells; ++e) {
        const uint32_t lo = m->lmap[(size_t)(2 * q) * m->n_cells + e];
        const uint32_t hi = 2 * q + 1 < m->nb ? m->lmap[(size_t)(2 * q + 1) * m->n_cells + e] : 0u;
        lm2[(size_t)q * m->n_cells + e] = lo | (hi << 16);
      }
    STTRY(upload_i(&p->d_lmap, lm2));
  }
  {
    std::vector<double> g((size_t)m->ng * m->n_cells);  // SoA
    for (int64_t e = 0; e < m->n_cells; ++e)
      for (int k = 0; k < m->ng; ++k) g[(size_t)k * m->n_cells + e] = m->geom[e * m->ng + k];
    STTRY(upload_real(&p->d_geom, g, prec));
  }
  STTRY(upload_i(&p->d_cell_start, m->patch_cell_start));
  STTRY(upload_i(&p->d_own_start, m->patch_own_start));
  STTRY(upload_i(&p->d_sh_start, m->patch_sh_start));
  // ref and list arrays carry padding so that clamped indices of idle lanes stay
  // in bounds (the kernels load them without branching)
  {
    std::vector<int32_t> v(m->sh_idx);
    v.push_back(0);
    STTRY(upload_i(&p->d_sh_idx, v));
    std::vector<int32_t> r(m->ref_slots);
    r.push_back(0);
    r.push_back(0);
    STTRY(upload_i(&p->d_ref_slots, r));
    std::vector<uint16_t> gl(m->glist);
    gl.resize(gl.size() + 8, 0);
    STTRY(upload_i(&p->d_glist, gl));
  }
  STTRY(upload_i(&p->d_gword, m->gword));
  STTRY(upload_i(&p->d_gword_off, m->gword_off));
  STTRY(upload_i(&p->d_glist_off, m->glist_off));
  STTRY(upload_i(&p->d_shp_ptr, m->shp_ptr));
  STTRY(upload_i(&p->d_shp_slot, m->shp_slot));
  STTRY(upload_coefficients(p));
  {
    std::vector<double> ms(m->n_dofs);
    for (int64_t i = 0; i < m->n_dofs; ++i) ms[i] = 1.0 / std::sqrt(m->mass[i]);
    STTRY(upload_real(&p->d_minv_sqrt, ms, prec));
  }
  const size_t vb = (size_t)m->n_dofs * p->ts;
  STTRY(alloc(&p->d_c2, vb));
  STTRY(alloc(&p->d_c2_ref, std::max<size_t>(1, m->n_shared_refs) * p->ts));
  STTRY(alloc_sweep(p->fwd, *m, p->ts, false, n_shots));
  STTRY(alloc_sweep(p->adj, *m, p->ts, true, n_shots));
  STTRY(alloc(&p->d_lam[0], (size_t)p->ls * n_shots * p->ts));
  STTRY(alloc(&p->d_lam[1], (size_t)p->ls * n_shots * p->ts));
  STTRY(alloc((void**)&p->d_gacc, (size_t)m->n_dofs * n_shots * 8));
  STTRY(alloc((void**)&p->d_red, (size_t)(p->red_blocks + 8) * 8));
  STTRY(alloc((void**)&p->d_flag, 256));
  HIPTRY(launch_fill_i32(p->d_flag, 0, 1, nullptr));
  {
    // set-up of the allocation-free forward's workspace address on this device; a
    // failure is reported by kmv_forward_noalloc, which asks again
    void* ws = nullptr;
    (void)scratch_ptr(p->device, &ws);
    (void)hipGetLastError();
  }
  *out = guard.release();
  return OK;
}

Status set_absorbing_boundary(Problem* p, bool on) {
  DeviceGuard dg(p->device);
  if (on && p->pml3) return Status{KMV_ESTATE, "the absorbing boundary term does not combine with the PML on tetrahedra"};
  if (on && p->bnd_dof.empty()) {
    const std::vector<int32_t>* d;
    const std::vector<double>* b;
    boundary_of(*p->mesh, &d, &b);
    p->bnd_dof = *d;
    p->bnd_b = *b;
    p->nbd = (int)p->bnd_dof.size();
    STTRY(upload_i(&p->d_bnd_dof, p->bnd_dof.empty() ? std::vector<int32_t>{0} : p->bnd_dof));
    dfree(p->d_bnd_part);
    p->d_bnd_part = nullptr;
  }
  p->absorb = on;
  if (!on) {  // the records are kept only while the term is on
    dfree(p->d_ub);
    dfree(p->d_lb);
    p->d_ub = p->d_lb = nullptr;
    p->bnd_rec_bytes = 0;
  }
  return upload_coefficients(p);
}

Status set_damping(Problem* p, const double* eta) {
  DeviceGuard dg(p->device);
  if (p->pml()) return Status{KMV_ESTATE, "the PML's damping takes the place of eta; turn the PML off first"};
  if (eta) {
    for (int64_t i = 0; i < p->mesh->n_dofs; ++i)
      if (!(eta[i] >= 0) || !std::isfinite(eta[i])) return Status{KMV_EINVAL, "damping must be finite and >= 0"};
    p->eta.assign(eta, eta + p->mesh->n_dofs);
  } else {
    p->eta.clear();
  }
  return upload_coefficients(p);
}

// PML on tetrahedra: sigma [n_dofs*3] (sigma_x, sigma_y, sigma_z per DOF).  One
// shot per problem; not with the absorbing boundary term.
Status set_pml3(Problem* p, const double* sigma) {
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs, ne = m.n_cells;
  const int nd = m.nd;
  if (p->nshot != 1) return Status{KMV_EINVAL, "the PML on tetrahedra takes one shot per problem"};
  if (p->absorb) return Status{KMV_ESTATE, "turn the absorbing boundary term off before the PML on tetrahedra"};
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!(sigma[i] >= 0) || !std::isfinite(sigma[i]))
      return Status{KMV_EINVAL, "PML damping functions must be finite and >= 0"};
  if (ne * nd > INT32_MAX) return Status{KMV_EINVAL, "mesh too large for the PML's cell-node slots"};
  std::vector<double> sc(3 * N);
  for (int64_t i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) sc[k * N + i] = sigma[3 * i + k];
  std::vector<int32_t> cdof((size_t)ne * nd), ptr(N + 1, 0), cpos((size_t)ne * nd);
  for (size_t k = 0; k < cdof.size(); ++k) {
    cdof[k] = (int32_t)m.cell_dofs[k];
    ptr[cdof[k] + 1]++;
  }
  for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
  {
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t k = 0; k < cdof.size(); ++k)  // ascending (cell, node) within each DOF's range
      cpos[(k % nd) * ne + k / nd] = fill[cdof[k]]++;
  }
  std::vector<double> b(9 * (size_t)ne);  // B_e = |det J| J^-T, entry (k, r) at 3k + r
  for (int64_t e = 0; e < ne; ++e)
    for (int k = 0; k < 3; ++k)
      for (int r = 0; r < 3; ++r) b[(size_t)(3 * k + r) * ne + e] = m.absdet[e] * m.jinv[e * 9 + r * 3 + k];
  STTRY(upload_real(&p->d_sig, sc, p->prec));
  {
    std::vector<int32_t> cm(cdof.size());  // node-major for the per-cell pass
    for (size_t k = 0; k < cdof.size(); ++k) cm[(k % nd) * ne + k / nd] = cdof[k];
    STTRY(upload_i(&p->d_cdof, cm));
  }
  STTRY(upload_i(&p->d_csr_ptr, ptr));
  STTRY(upload_i(&p->d_cpos, cpos));
  STTRY(upload_real(&p->d_b3, b, p->prec));
  STTRY(upload_real(&p->d_mass, m.mass, p->prec));
  STTRY(alloc(&p->d_cellout, (size_t)12 * ne * nd * p->ts));
  STTRY(alloc(&p->d_ku, (size_t)N * p->ts));
  for (int k = 0; k < 2; ++k) {
    STTRY(alloc(&p->d_p3[k], (size_t)3 * N * p->ts));
    STTRY(alloc(&p->d_nu3[k], (size_t)N * p->ts));
  }
  p->sigma = sc;
  p->pml3 = true;
  p->p3_points_dirty = true;
  return OK;
}

Status set_pml(Problem* p, const double* sigma) {
  DeviceGuard dg(p->device);
  const Mesh& m = *p->mesh;
  const int64_t N = m.n_dofs;
  if (!sigma) {
    p->sigma.clear();
    p->eta.clear();
    for (void* q : {p->d_sig, p->d_sig_ref, p->d_pml_b, (void*)p->d_list[0], (void*)p->d_list[1]}) dfree(q);
    for (int w = 0; w < 2; ++w)
      for (int k = 0; k < 2; ++k) {
        dfree(p->d_pp[w][k]);
        dfree(p->d_pt[w][k]);
        p->d_pp[w][k] = p->d_pt[w][k] = nullptr;
      }
    p->d_sig = p->d_sig_ref = p->d_pml_b = nullptr;
    p->d_list[0] = p->d_list[1] = nullptr;
    p->n_list[0] = p->n_list[1] = 0;
    for (void** q : {(void**)&p->d_cdof, &p->d_b3, (void**)&p->d_csr_ptr, (void**)&p->d_cpos, &p->d_mass,
                     &p->d_cellout, &p->d_ku, &p->d_p3[0], &p->d_p3[1], &p->d_nu3[0], &p->d_nu3[1], &p->d_y3}) {
      dfree(*q);
      *q = nullptr;
    }
    p->n_y3 = 0;
    p->pml3 = false;
    return upload_coefficients(p);
  }
  if (m.dim == 3) return set_pml3(p, sigma);
  for (int64_t i = 0; i < 2 * N; ++i)
    if (!(sigma[i] >= 0) || !std::isfinite(sigma[i]))
      return Status{KMV_EINVAL, "PML damping functions must be finite and >= 0"};
  for (bool adjv : {false, true}) {
    const size_t bytes =
        step_lds_bytes(m.dim, m.nd, m.max_nbl, m.slot_stride, m.nb, m.max_glist, adjv, p->ts, true);
    if (bytes > 160 * 1024)
      return Status{KMV_EINVAL, "PML patch LDS footprint of " + std::to_string((bytes + 1023) / 1024) +
                                    " KiB above the 160 KiB of a CU; use smaller patches (patch_cells)"};
    if (bytes > 64 * 1024) HIPTRY(raise_lds_limit(p->device, p->prec, m.dim, m.nd, adjv, bytes, true));
  }
  std::vector<double> sc(2 * N), eta(N), sr(2 * p->rs, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    sc[i] = sigma[2 * i];
    sc[N + i] = sigma[2 * i + 1];
    eta[i] = sc[i] + sc[N + i];  // tr Psi_1
  }
  p->sigma = sc;
  for (int64_t r = 0; r < m.n_shared_refs; ++r) {
    sr[r] = sc[m.sh_idx[r]];
    sr[p->rs + r] = sc[N + m.sh_idx[r]];
  }
  p->eta = eta;
  STTRY(upload_real(&p->d_sig, sc, p->prec));
  STTRY(upload_real(&p->d_sig_ref, sr, p->prec));
  {
    std::vector<double> b(4 * (size_t)m.n_cells);  // B_e = |det J| J^-T, entry (k, r) at (2k + r)
    for (int64_t e = 0; e < m.n_cells; ++e)
      for (int k = 0; k < 2; ++k)
        for (int r = 0; r < 2; ++r) b[(size_t)(2 * k + r) * m.n_cells + e] = m.absdet[e] * m.jinv[e * 4 + r * 2 + k];
    STTRY(upload_real(&p->d_pml_b, b, p->prec));
  }
  // patches with a DOF in the layer run the PML instance
  std::vector<int32_t> list[2];
  for (int64_t q = 0; q < m.n_patches; ++q) {
    bool in = false;
    for (int32_t i = m.patch_own_start[q]; i < m.patch_own_start[q + 1] && !in; ++i) in = eta[i] != 0.0;
    for (int32_t r = m.patch_sh_start[q]; r < m.patch_sh_start[q + 1] && !in; ++r) in = eta[m.sh_idx[r]] != 0.0;
    list[in ? 1 : 0].push_back((int32_t)q);
  }
  for (int k = 0; k < 2; ++k) {
    p->n_list[k] = (int)list[k].size();
    if (list[k].empty()) list[k].push_back(0);
    STTRY(upload_i(&p->d_list[k], list[k]));
  }
  for (int w = 0; w < 2; ++w)
    for (int k = 0; k < 2; ++k) {
      STTRY(alloc(&p->d_pp[w][k], 2 * (size_t)p->ls * p->nshot * p->ts));
      STTRY(alloc(&p->d_pt[w][k], 2 * (size_t)p->rs * p->nshot * p->ts));
    }
  return upload_coefficients(p);
}

Status set_wavelet(Problem* p, const double* w) {
  DeviceGuard dg(p->device);
  p->wavelet.assign(w, w + p->nt);
  p->wavelet_per_shot = false;
  return upload_real(&p->d_wavelet, p->wavelet, p->prec);
}

// One wavelet per shot, shot-major [n_shots][nt]: the forward launch offsets the
// amplitude pointer by shot * nt, as it offsets the other per-shot buffers.
Status set_wavelets(Problem* p, const double* w) {
  DeviceGuard dg(p->device);
  p->wavelet.assign(w, w + p->nt * p->nshot);
  p->wavelet_per_shot = true;
  return upload_real(&p->d_wavelet, p->wavelet, p->prec);
}

Status set_sources(Problem* p, const double* xs, int nsrc, double f0, double t0, double amp) {
  DeviceGuard dg(p->device);
  if (nsrc <= 0 || !xs) return Status{KMV_EINVAL, "need at least one source"};
  if (nsrc % p->nshot != 0) return Status{KMV_EINVAL, "n_src must be a multiple of n_shots (shot-major)"};
  free_points(p->src);
  STTRY(build_points(p, xs, nsrc, p->nshot, p->src));
  std::vector<double> w(p->nt);
  const double pi = 3.14159265358979323846;
  for (int64_t n = 0; n < p->nt; ++n) {
    const double t = n * p->dt - t0;
    const double arg = pi * pi * f0 * f0 * t * t;
    w[n] = amp * (1.0 - 2.0 * arg) * std::exp(-arg);
  }
  p->has_src = true;
  return set_wavelet(p, w.data());
}

Status set_receivers(Problem* p, const double* xr, int nrec) {
  DeviceGuard dg(p->device);
  if (nrec <= 0 || !xr) return Status{KMV_EINVAL, "need at least one receiver"};
  free_points(p->rec);
  STTRY(build_points(p, xr, nrec, 1, p->rec));
  const size_t tb = (size_t)p->nt * nrec * p->nshot * p->ts;
  STTRY(alloc(&p->d_resid, tb));
  STTRY(alloc(&p->d_traces_tmp, tb));
  return OK;
}

Status forward_noalloc(Problem* p, const double* c, void* traces, hipStream_t s) {
  DeviceGuard dg(p->device);
  if (p->pml3) return Status{KMV_ESTATE, "the allocation-free forward does not take the PML on tetrahedra"};
  if (!p->has_src || p->rec.npts == 0) return Status{KMV_ESTATE, "sources and receivers must be set first"};
  if (!c || !traces) return Status{KMV_EINVAL, "null device pointer"};
  const size_t need = 2 * (size_t)p->ls * p->nshot * p->ts;
  if (need > kScratchBytes)
    return Status{KMV_EINVAL, "the allocation-free forward needs " + std::to_string(need) +
                                  " bytes of workspace; the static workspace holds " +
                                  std::to_string(kScratchBytes) + " (use kmv_forward)"};
  void* base = nullptr;
  STTRY(scratch_ptr(p->device, &base));
  // no timing events either: the launches are counted but not timed
  const int every = p->probe.every;
  p->probe.every = 0;
  const Status st = p->prec == KMV_FP64 ? forward_run<double>(p, c, (double*)traces, (double*)base, s)
                                        : forward_run<float>(p, c, (float*)traces, (float*)base, s);
  p->probe.every = every;
  return st;
}

Status forward(Problem* p, const double* c, void* traces, hipStream_t s) {
  DeviceGuard dg(p->device);
  if (!p->has_src || p->rec.npts == 0) return Status{KMV_ESTATE, "sources and receivers must be set first"};
  if (!c || !traces) return Status{KMV_EINVAL, "null device pointer"};
  return p->prec == KMV_FP64 ? forward_t<double>(p, c, (double*)traces, s) : forward_t<float>(p, c, (float*)traces, s);
}

Status misfit_gradient(Problem* p, const double* c, const void* obs, double* J, double* grad, void* traces,
                       hipStream_t s, bool accumulate) {
  DeviceGuard dg(p->device);
  if (!p->has_src || p->rec.npts == 0) return Status{KMV_ESTATE, "sources and receivers must be set first"};
  if (!c || !obs || !J || !grad) return Status{KMV_EINVAL, "null pointer"};
  return p->prec == KMV_FP64
             ? misfit_gradient_t<double>(p, c, (const double*)obs, J, grad, (double*)traces, s, accumulate)
             : misfit_gradient_t<float>(p, c, (const float*)obs, J, grad, (float*)traces, s, accumulate);
}

Status misfit(Problem* p, const double* c, const void* obs, double* J, void* traces, hipStream_t s) {
  DeviceGuard dg(p->device);
  if (!p->has_src || p->rec.npts == 0) return Status{KMV_ESTATE, "sources and receivers must be set first"};
  if (!c || !obs || !J) return Status{KMV_EINVAL, "null pointer"};
  return p->prec == KMV_FP64 ? misfit_t<double>(p, c, (const double*)obs, J, (double*)traces, s)
                             : misfit_t<float>(p, c, (const float*)obs, J, (float*)traces, s);
}

Status solve_status(Problem* p, hipStream_t s) {
  DeviceGuard dg(p->device);
  int flag = 0;
  HIPTRY(hipMemcpyAsync(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  if (!flag) return OK;
  return p->prec == KMV_FP64 ? classify_nonfinite<double>(p, s) : classify_nonfinite<float>(p, s);
}

Status adjoint(Problem* p, const double* c, const void* adj, void* lambda_out, void* src_trace, hipStream_t s) {
  DeviceGuard dg(p->device);
  if (p->rec.npts == 0) return Status{KMV_ESTATE, "receivers must be set first"};
  if (src_trace && !p->has_src) return Status{KMV_ESTATE, "sources must be set to record at them"};
  if (lambda_out && p->nshot != 1) return Status{KMV_EINVAL, "lambda_out needs a one-shot problem"};
  if (!c || !adj) return Status{KMV_EINVAL, "null device pointer"};
  return p->prec == KMV_FP64
             ? adjoint_t<double>(p, c, (const double*)adj, (double*)lambda_out, (double*)src_trace, s)
             : adjoint_t<float>(p, c, (const float*)adj, (float*)lambda_out, (float*)src_trace, s);
}

Status stiffness_apply(Problem* p, const double* c, const void* u, void* y, hipStream_t s) {
  DeviceGuard dg(p->device);
  if (!c || !u || !y) return Status{KMV_EINVAL, "null device pointer"};
  return p->prec == KMV_FP64 ? apply_t<double>(p, c, (const double*)u, (double*)y, s)
                             : apply_t<float>(p, c, (const float*)u, (float*)y, s);
}

Status spectral_radius(Problem* p, const double* c, int iters, uint64_t seed, double* rho, hipStream_t s) {
  DeviceGuard dg(p->device);
  if (!c || !rho || iters <= 0) return Status{KMV_EINVAL, "bad argument"};
  return p->prec == KMV_FP64 ? spectral_t<double>(p, c, iters, seed, rho, s)
                             : spectral_t<float>(p, c, iters, seed, rho, s);
}

}  // namespace kmv
