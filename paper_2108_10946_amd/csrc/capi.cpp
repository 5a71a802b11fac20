// extern "C" boundary: argument checks, status codes, thread-local error text.
// No C++ exception crosses this file.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/kmvwave.h"
#include "element.hpp"
#include "kernels.hpp"
#include "mesh.hpp"
#include "problem.hpp"
#include "server.hpp"

struct kmv_mesh_s {
  kmv::Mesh* m;
};
struct kmv_problem_s {
  kmv::Problem* p;
};
struct kmv_server_s {
  kmv::Server* s;
};

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int done(const kmv::Status& s) {
  if (s.code != KMV_OK) g_err = s.msg;
  return s.code;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const kmv::MeshError& e) {
    return fail(KMV_EMESH, e.what);
  } catch (const std::bad_alloc&) {
    return fail(KMV_ENOMEM, "host allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(KMV_EINVAL, e.what());
  } catch (const std::exception& e) {
    return fail(KMV_EINVAL, e.what());
  } catch (...) {
    return fail(KMV_EINVAL, "unknown error");
  }
}
}  // namespace

extern "C" {

const char* kmv_last_error(void) { return g_err.c_str(); }

int kmv_element_tables(int dim, int degree, int* n_nodes, double* nodes, double* weights, double* grads) {
  return guarded([&]() {
    if (!kmv::element_supported(dim, degree))
      return fail(KMV_EDEGREE, "unsupported (dim, degree): tri 1..5, tet 1..3");
    const kmv::Element& el = kmv::element(dim, degree);
    if (n_nodes) *n_nodes = el.n;
    if (nodes) std::memcpy(nodes, el.nodes.data(), el.nodes.size() * sizeof(double));
    if (weights) std::memcpy(weights, el.weights.data(), el.weights.size() * sizeof(double));
    if (grads) std::memcpy(grads, el.grads.data(), el.grads.size() * sizeof(double));
    return (int)KMV_OK;
  });
}

int kmv_mesh_create(int dim, int degree, const double* coords, int64_t n_vertices, const int32_t* cells,
                    int64_t n_cells, int patch_cells, kmv_mesh* out) {
  return guarded([&]() {
    if (!out) return fail(KMV_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(KMV_EINVAL, "dim must be 2 or 3");
    if (!kmv::element_supported(dim, degree))
      return fail(KMV_EDEGREE, "unsupported (dim, degree): tri 1..5, tet 1..3");
    if (!coords || !cells || n_vertices <= 0 || n_cells <= 0) return fail(KMV_EINVAL, "empty mesh");
    if (patch_cells < 0 || patch_cells > 256) return fail(KMV_EINVAL, "patch_cells must be in 0..256");
    kmv::Mesh* m = kmv::build_mesh(dim, degree, coords, n_vertices, cells, n_cells, patch_cells);
    *out = new kmv_mesh_s{m};
    return (int)KMV_OK;
  });
}

int kmv_mesh_info(kmv_mesh h, int64_t* n_dofs, int64_t* n_cells, int* n_nodes, int64_t* n_patches,
                  int64_t* n_shared_dofs) {
  if (!h) return fail(KMV_EINVAL, "mesh is NULL");
  const kmv::Mesh& m = *h->m;
  if (n_dofs) *n_dofs = m.n_dofs;
  if (n_cells) *n_cells = m.n_cells;
  if (n_nodes) *n_nodes = m.nd;
  if (n_patches) *n_patches = m.n_patches;
  if (n_shared_dofs) *n_shared_dofs = m.n_shared;
  return KMV_OK;
}

int kmv_mesh_dof_coords(kmv_mesh h, double* out) {
  if (!h || !out) return fail(KMV_EINVAL, "NULL argument");
  std::memcpy(out, h->m->dof_coords.data(), h->m->dof_coords.size() * sizeof(double));
  return KMV_OK;
}

int kmv_mesh_lumped_mass(kmv_mesh h, double* out) {
  if (!h || !out) return fail(KMV_EINVAL, "NULL argument");
  std::memcpy(out, h->m->mass.data(), h->m->mass.size() * sizeof(double));
  return KMV_OK;
}

int kmv_mesh_boundary_mass(kmv_mesh h, double* out) {
  return guarded([&]() {
    if (!h || !out) return fail(KMV_EINVAL, "NULL argument");
    const std::vector<int32_t>* d;
    const std::vector<double>* b;
    kmv::boundary_of(*h->m, &d, &b);
    std::memset(out, 0, h->m->n_dofs * sizeof(double));
    for (size_t t = 0; t < d->size(); ++t) out[(*d)[t]] = (*b)[t];
    return (int)KMV_OK;
  });
}

int kmv_mesh_cell_dofs(kmv_mesh h, int64_t* out) {
  if (!h || !out) return fail(KMV_EINVAL, "NULL argument");
  const kmv::Mesh& m = *h->m;
  for (int64_t i = 0; i < m.n_cells; ++i)
    std::memcpy(out + m.cell_input[i] * m.nd, &m.cell_dofs[i * m.nd], m.nd * sizeof(int64_t));
  return KMV_OK;
}

int kmv_mesh_destroy(kmv_mesh h) {
  if (!h) return KMV_OK;
  delete h->m;
  delete h;
  return KMV_OK;
}

int kmv_problem_create(kmv_mesh m, const kmv_options* opt, kmv_problem* out) {
  return guarded([&]() {
    if (!m || !opt || !out) return fail(KMV_EINVAL, "NULL argument");
    *out = nullptr;
    kmv::Problem* p = nullptr;
    kmv::Status s = kmv::problem_create(m->m, opt->precision, opt->dt, opt->n_steps, opt->checkpoint_every,
                                        opt->mem_budget, opt->n_shots == 0 ? 1 : opt->n_shots,
                                        opt->gradient_every == 0 ? 1 : opt->gradient_every, &p);
    if (s.code != KMV_OK) return done(s);
    *out = new kmv_problem_s{p};
    return (int)KMV_OK;
  });
}

int kmv_problem_info(kmv_problem h, int64_t* n_dofs, int64_t* n_steps, int* n_rec, int* precision,
                     int64_t* checkpoint_every) {
  if (!h) return fail(KMV_EINVAL, "problem is NULL");
  const kmv::Problem& p = *h->p;
  if (n_dofs) *n_dofs = p.mesh->n_dofs;
  if (n_steps) *n_steps = p.nt;
  if (n_rec) *n_rec = p.rec.npts;
  if (precision) *precision = p.prec;
  if (checkpoint_every) *checkpoint_every = p.store_all || p.store_sub ? 0 : p.seg;
  return KMV_OK;
}

int kmv_problem_num_shots(kmv_problem h, int* n_shots) {
  if (!h || !n_shots) return fail(KMV_EINVAL, "NULL argument");
  *n_shots = h->p->nshot;
  return KMV_OK;
}

int kmv_cfl_dt(kmv_mesh h, const double* c_host, double* dt_max) {
  return guarded([&]() {
    if (!h || !c_host || !dt_max) return fail(KMV_EINVAL, "NULL argument");
    const double rho = kmv::gershgorin_rho(*h->m, c_host);
    if (!(rho > 0) || !std::isfinite(rho)) return fail(KMV_EINVAL, "wavespeed gives no positive spectral bound");
    *dt_max = 2.0 / std::sqrt(rho);
    return (int)KMV_OK;
  });
}

int kmv_mesh_validate(kmv_mesh h) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "mesh is NULL");
    std::string why;
    if (!kmv::validate_mesh(*h->m, why)) return fail(KMV_EMESH, why);
    return (int)KMV_OK;
  });
}

int kmv_mesh_patch_stats(kmv_mesh h, int adjoint, int64_t* max_patch_cells, int64_t* max_shared_refs,
                         int64_t* first_batch_refs) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "mesh is NULL");
    const kmv::Mesh& m = *h->m;
    int64_t most = 0;
    for (int64_t q = 0; q < m.n_patches; ++q)
      most = std::max<int64_t>(most, m.patch_sh_start[q + 1] - m.patch_sh_start[q]);
    if (max_patch_cells) *max_patch_cells = m.max_patch_cells;
    if (max_shared_refs) *max_shared_refs = most;
    if (first_batch_refs)
      *first_batch_refs = kmv::step_first_batch_refs(m.dim, m.nd, adjoint != 0, kmv::step_block(m.max_patch_cells));
    return (int)KMV_OK;
  });
}

int kmv_spectral_radius(kmv_problem h, const void* c_dev, int iters, uint64_t seed, double* rho,
                        void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::spectral_radius(h->p, (const double*)c_dev, iters, seed, rho, (hipStream_t)stream));
  });
}

int kmv_set_pml(kmv_problem h, const double* sigma) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::set_pml(h->p, sigma));
  });
}

int kmv_set_damping(kmv_problem h, const double* eta) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::set_damping(h->p, eta));
  });
}

int kmv_set_absorbing_boundary(kmv_problem h, int enable) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    if (enable != 0 && enable != 1) return fail(KMV_EINVAL, "enable must be 0 or 1");
    return done(kmv::set_absorbing_boundary(h->p, enable == 1));
  });
}

int kmv_set_sources(kmv_problem h, const double* xs, int n_src, double f0, double t0, double amp) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::set_sources(h->p, xs, n_src, f0, t0, amp));
  });
}

int kmv_set_source_wavelets(kmv_problem h, const double* w) {
  return guarded([&]() {
    if (!h || !w) return fail(KMV_EINVAL, "NULL argument");
    if (!h->p->has_src) return fail(KMV_ESTATE, "set the source points first");
    return done(kmv::set_wavelets(h->p, w));
  });
}

int kmv_set_source_wavelet(kmv_problem h, const double* w) {
  return guarded([&]() {
    if (!h || !w) return fail(KMV_EINVAL, "NULL argument");
    if (!h->p->has_src) return fail(KMV_ESTATE, "set the source points first");
    return done(kmv::set_wavelet(h->p, w));
  });
}

int kmv_set_receivers(kmv_problem h, const double* xr, int n_rec) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::set_receivers(h->p, xr, n_rec));
  });
}

int kmv_forward(kmv_problem h, const void* c_dev, void* traces_dev, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::forward(h->p, (const double*)c_dev, traces_dev, (hipStream_t)stream));
  });
}

int kmv_forward_noalloc(kmv_problem h, const void* c_dev, void* traces_dev, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::forward_noalloc(h->p, (const double*)c_dev, traces_dev, (hipStream_t)stream));
  });
}

int kmv_misfit_gradient(kmv_problem h, const void* c_dev, const void* observed_dev, double* J_out,
                        double* grad_dev, void* traces_dev, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::misfit_gradient(h->p, (const double*)c_dev, observed_dev, J_out, grad_dev, traces_dev,
                                     (hipStream_t)stream));
  });
}

int kmv_misfit_gradient_accumulate(kmv_problem h, const void* c_dev, const void* observed_dev, double* J_acc,
                                   double* grad_acc, void* traces_dev, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::misfit_gradient(h->p, (const double*)c_dev, observed_dev, J_acc, grad_acc, traces_dev,
                                     (hipStream_t)stream, true));
  });
}

int kmv_misfit(kmv_problem h, const void* c_dev, const void* observed_dev, double* J_out, void* traces_dev,
               void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::misfit(h->p, (const double*)c_dev, observed_dev, J_out, traces_dev, (hipStream_t)stream));
  });
}

int kmv_problem_status(kmv_problem h, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::solve_status(h->p, (hipStream_t)stream));
  });
}

int kmv_adjoint(kmv_problem h, const void* c_dev, const void* adj_src_dev, void* lambda_out_dev,
                void* src_trace_dev, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::adjoint(h->p, (const double*)c_dev, adj_src_dev, lambda_out_dev, src_trace_dev,
                             (hipStream_t)stream));
  });
}

int kmv_stiffness_apply(kmv_problem h, const void* c_dev, const void* u_dev, void* y_dev, void* stream) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::stiffness_apply(h->p, (const double*)c_dev, u_dev, y_dev, (hipStream_t)stream));
  });
}

int kmv_profile_enable(kmv_problem h, int every) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::profile_enable(h->p, every));
  });
}

int kmv_profile_read(kmv_problem h, int variant, int64_t* n_launches, int64_t* n_timed, double* mean_ms) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "problem is NULL");
    return done(kmv::profile_read(h->p, variant, n_launches, n_timed, mean_ms));
  });
}

int kmv_problem_destroy(kmv_problem h) {
  if (!h) return KMV_OK;
  delete h->p;
  delete h;
  return KMV_OK;
}

// ------------------------------------------------------------------- serving

int kmv_server_create(size_t mem_budget, int max_slots, kmv_server* out) {
  return guarded([&]() -> int {
    if (!out) return fail(KMV_EINVAL, "out is NULL");
    kmv::Server* s = nullptr;
    const int rc = done(kmv::server_create(mem_budget, max_slots, &s));
    if (rc != KMV_OK) return rc;
    *out = new kmv_server_s{s};
    return KMV_OK;
  });
}

int kmv_server_submit(kmv_server h, const kmv_request* req, uint64_t* ticket) {
  return guarded([&]() {
    if (!h || !req || !req->mesh) return fail(KMV_EINVAL, "server, request or mesh is NULL");
    return done(kmv::server_submit(h->s, req->mesh->m, req, ticket));
  });
}

namespace {
int result_status(int rc, const kmv_result* out, const std::string& msg) {
  if (rc == KMV_OK && out && out->status != KMV_OK) g_err = msg;
  return rc;
}
}  // namespace

int kmv_server_poll(kmv_server h, uint64_t ticket, kmv_result* out) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "server is NULL");
    std::string msg;
    const int rc = done(kmv::server_poll(h->s, ticket, out, &msg));
    return result_status(rc, out, msg);
  });
}

int kmv_server_wait(kmv_server h, uint64_t ticket, double timeout_s, kmv_result* out) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "server is NULL");
    std::string msg;
    const int rc = done(kmv::server_wait(h->s, ticket, timeout_s, out, &msg));
    return result_status(rc, out, msg);
  });
}

int kmv_server_release(kmv_server h, uint64_t ticket) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "server is NULL");
    return done(kmv::server_release(h->s, ticket));
  });
}

int kmv_server_stats(kmv_server h, int* running, int* queued, size_t* bytes_in_use) {
  return guarded([&]() {
    if (!h) return fail(KMV_EINVAL, "server is NULL");
    return done(kmv::server_stats(h->s, running, queued, bytes_in_use));
  });
}

int kmv_server_destroy(kmv_server h) {
  if (!h) return KMV_OK;
  kmv::server_destroy(h->s);
  delete h;
  return KMV_OK;
}

}  // extern "C"
