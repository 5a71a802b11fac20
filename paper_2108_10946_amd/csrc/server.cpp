// Shot server.  Requests (one or several shots: mesh, wave speed, damping,
// sources, receivers, time window, observed data) are copied on submission and
// queued in arrival order.  The shots of one request run as one multi-shot
// problem.  Each of `slots` worker threads owns a HIP stream; a free worker
// admits the request at the head of the queue as soon as its device memory fits
// in what the running requests leave of the budget, solves it on its stream
// (forward, or misfit + adjoint + gradient) and stores the results on the host.
// Requests admitted together run concurrently on the GPU; since every kernel of a
// solve is deterministic and a solve shares no buffers with another, each result
// is bitwise the one the request gets alone.
#include "server.hpp"

#include "boundary.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace kmv {
namespace {

const Status OK{KMV_OK, ""};

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Runs one job on stream st (worker thread).  Device memory comes from the
// stream-ordered allocator, so setting up and tearing down a solve does not wait
// for the other workers' kernels.
Status run_job(Server* S, Job* j, hipStream_t st) {
  AllocStreamScope scope(st);
  const Mesh& m = *j->mesh;
  const size_t ts = j->prec == KMV_FP64 ? 8 : 4;
  const size_t N = (size_t)m.n_dofs, rows = (size_t)j->nt * j->nrec * j->nshot;
  Problem* p = nullptr;
  Status s = problem_create(j->mesh, j->prec, j->dt, j->nt, 0, S->per_job_budget, j->nshot, 1, &p);
  if (s.code != KMV_OK) return s;
  std::unique_ptr<Problem> guard(p);
  void *c_dev = nullptr, *obs = nullptr, *tr = nullptr, *g = nullptr;
  auto fail = [&](hipError_t e, const char* what) {
    return Status{KMV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
  };
  auto cleanup = [&]() {
    for (void* q : {c_dev, obs, tr, g})
      if (q) (void)hipFreeAsync(q, st);
  };
  auto run = [&]() -> Status {
    if (!j->eta.empty()) {
      Status r = set_damping(p, j->eta.data());
      if (r.code != KMV_OK) return r;
    }
    if (j->absorbing) {
      Status r = set_absorbing_boundary(p, true);
      if (r.code != KMV_OK) return r;
    }
    Status r = set_sources(p, j->xs.data(), j->nsrc, j->f0, j->t0, j->amp);
    if (r.code != KMV_OK) return r;
    if (!j->wavelets.empty()) {
      r = set_wavelets(p, j->wavelets.data());
      if (r.code != KMV_OK) return r;
    }
    r = set_receivers(p, j->xr.data(), j->nrec);
    if (r.code != KMV_OK) return r;
    hipError_t e;
    if ((e = hipMallocAsync(&c_dev, N * 8, st)) != hipSuccess) return fail(e, "hipMallocAsync");
    if ((e = hipMallocAsync(&tr, rows * ts, st)) != hipSuccess) return fail(e, "hipMallocAsync");
    if ((e = hipMemcpyAsync(c_dev, j->c.data(), N * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
      return fail(e, "hipMemcpyAsync");
    if (!j->forward_only) {
      if ((e = hipMallocAsync(&obs, rows * ts, st)) != hipSuccess) return fail(e, "hipMallocAsync");
      if ((e = hipMallocAsync(&g, N * 8, st)) != hipSuccess) return fail(e, "hipMallocAsync");
      if ((e = hipMemcpyAsync(obs, j->observed.data(), rows * ts, hipMemcpyHostToDevice, st)) != hipSuccess)
        return fail(e, "hipMemcpyAsync");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e, "hipStreamSynchronize");
    j->traces.resize(rows * ts);
    if (j->forward_only) {
      r = forward(p, (const double*)c_dev, tr, st);
      if (r.code != KMV_OK) return r;
    } else {
      j->grad.resize(N);
      r = misfit_gradient(p, (const double*)c_dev, obs, &j->J, (double*)g, tr, st);
      if (r.code != KMV_OK) return r;
      if ((e = hipMemcpyAsync(j->grad.data(), g, N * 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return fail(e, "hipMemcpyAsync");
    }
    if ((e = hipMemcpyAsync(j->traces.data(), tr, rows * ts, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e, "hipStreamSynchronize");
    return OK;
  };
  Status r = run();
  cleanup();
  guard.reset();  // frees the problem's buffers on st
  const hipError_t e = hipStreamSynchronize(st);
  if (r.code == KMV_OK && e != hipSuccess) r = fail(e, "hipStreamSynchronize");
  return r;
}

void worker(Server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[slot];
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&]() {
        return S->stop || (!S->queue.empty() && S->queue.front()->need <= S->budget - S->used);
      });
      if (S->stop) return;
      j = S->queue.front();
      S->queue.pop_front();
      S->used += j->need;
      S->running++;
      j->t_admit = S->now();
    }
    // the head changed: another worker may admit the next request
    S->cv_work.notify_all();
    Status r;
    try {
      r = run_job(S, j, st);
    } catch (const std::exception& ex) {
      r = Status{KMV_ENOMEM, ex.what()};
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->used -= j->need;
      S->running--;
      j->status = r.code;
      j->msg = r.msg;
      j->t_done = S->now();
      j->done = true;
      if (r.code != KMV_OK) {
        j->traces.clear();
        j->grad.clear();
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

}  // namespace

double Server::now() const { return seconds_since(epoch); }

size_t job_device_bytes(const Mesh& m, int prec, int64_t nt, int nrec, size_t budget, int nshot, int64_t n_bnd) {
  const size_t ts = prec == KMV_FP64 ? 8 : 4;
  const size_t N = (size_t)m.n_dofs, ne = (size_t)m.n_cells, np = (size_t)m.n_patches;
  size_t b = 0;
  // mesh tables
  b += (size_t)((m.nb + 1) / 2) * ne * 4 + (size_t)(m.ng + 1) * ne * ts + 4 * (np + 1) * 4;
  b += (size_t)(m.n_shared_refs + 1) * 12 + (size_t)(m.n_shared + 1) * 4 + m.gword.size() * 4 +
       (m.glist.size() + 8) * 2 + (np + 1) * 8;
  // coefficient vectors (and per-ref copies), sweeps, adjoint levels, gradient accumulator
  const size_t refs = std::max<size_t>(1, (size_t)m.n_shared_refs);
  // (the per-shot ones n_shot times)
  const size_t S = (size_t)std::max(1, nshot);
  b += 4 * N * ts + 3 * refs * ts + S * (2 * (N + 6 * refs) * ts + 6 * refs * ts + 2 * (N + refs) * ts + N * 8) +
       4096;
  // state storage (the plan the problem will take under `budget`): level vectors
  // hold a copy per shared ref after the DOFs, one per shot
  const size_t vb = (N + refs) * ts * S;
  if ((size_t)(nt + 1) * vb <= budget) {
    b += (size_t)(nt + 1) * vb;
  } else {
    const int64_t seg = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt(2.0 * nt)));
    const int64_t nck = (nt + seg - 1) / seg;
    b += (size_t)(seg + 1) * vb + 2 * (size_t)nck * vb;
  }
  // traces, residual, wavelet, point tables; request buffers
  const size_t rows = (size_t)nt * nrec * S;
  b += 2 * rows * ts + (size_t)nt * S * ts + (size_t)(nrec + 8 * S) * m.nd * 16 + S * (np + 1) * 4;
  b += 2 * N * 8 + 2 * rows * ts;
  // absorbing boundary (n_bnd >= 0): coefficient tables, u and lambda records, partial sums
  // and the ring of adjoint levels those records are taken from
  if (n_bnd >= 0)
    b += (size_t)n_bnd * (2 * S * (nt + 1) * ts + 4 * 8 + 4 + kBndChunks * 8) + 2 * N * ts +
         (size_t)kLamRing * (N + refs) * ts * S + 4096;
  // allocation granularity
  return b + (b >> 4) + ((size_t)4 << 20);
}

Status server_create(size_t budget, int slots, Server** out) {
  if (slots <= 0 || slots > 64) return Status{KMV_EINVAL, "max_slots must be in 1..64"};
  std::unique_ptr<Server> S(new Server());
  if (hipGetDevice(&S->device) != hipSuccess) return Status{KMV_EDEVICE, "no HIP device"};
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return Status{KMV_EDEVICE, "hipMemGetInfo failed"};
  S->budget = budget ? std::min(budget, free_b) : free_b / 10 * 8;
  S->slots = slots;
  // state storage each request may use before it checkpoints; independent of the
  // slot count, so a request's plan and memory do not depend on how many others
  // may run beside it
  S->per_job_budget = std::min(S->budget / 2, (size_t)32 << 30);
  S->epoch = std::chrono::steady_clock::now();
  // keep freed blocks in the stream-ordered pool instead of returning them
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, S->device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  for (int i = 0; i < slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t q : S->streams) (void)hipStreamDestroy(q);
      return Status{KMV_EDEVICE, "hipStreamCreateWithFlags failed"};
    }
    S->streams.push_back(st);
  }
  Server* raw = S.get();
  for (int i = 0; i < slots; ++i) S->workers.emplace_back(worker, raw, i);
  *out = S.release();
  return OK;
}

Status server_submit(Server* S, Mesh* m, const kmv_request* q, uint64_t* ticket) {
  if (!q || !ticket || !m) return Status{KMV_EINVAL, "null request, mesh or ticket"};
  if (q->precision != KMV_FP64 && q->precision != KMV_FP32) return Status{KMV_EINVAL, "bad precision"};
  if (!(q->dt > 0) || q->n_steps <= 0) return Status{KMV_EINVAL, "dt and n_steps must be positive"};
  if (!q->c || !q->xs || q->n_src <= 0 || !q->xr || q->n_rec <= 0)
    return Status{KMV_EINVAL, "wave speed, sources and receivers are required"};
  if (!q->forward_only && !q->observed) return Status{KMV_EINVAL, "observed data required"};
  const int nshot = q->n_shots == 0 ? 1 : q->n_shots;
  if (nshot < 1 || nshot > 1024) return Status{KMV_EINVAL, "n_shots must be in 1..1024"};
  if (q->n_src % nshot != 0) return Status{KMV_EINVAL, "n_src must be a multiple of n_shots (shot-major)"};
  if (q->absorbing != 0 && q->absorbing != 1) return Status{KMV_EINVAL, "absorbing must be 0 or 1"};
  std::unique_ptr<Job> j(new Job());
  j->mesh = m;
  j->prec = q->precision;
  j->forward_only = q->forward_only ? 1 : 0;
  j->dt = q->dt;
  j->nt = q->n_steps;
  j->nsrc = q->n_src;
  j->nrec = q->n_rec;
  j->nshot = nshot;
  j->absorbing = q->absorbing;
  j->f0 = q->f0;
  j->t0 = q->t0;
  j->amp = q->amp;
  const size_t N = (size_t)m->n_dofs, ts = q->precision == KMV_FP64 ? 8 : 4;
  j->c.assign(q->c, q->c + N);
  if (q->eta) j->eta.assign(q->eta, q->eta + N);
  j->xs.assign(q->xs, q->xs + (size_t)q->n_src * m->dim);
  j->xr.assign(q->xr, q->xr + (size_t)q->n_rec * m->dim);
  if (q->wavelets) j->wavelets.assign(q->wavelets, q->wavelets + (size_t)nshot * q->n_steps);
  if (!j->forward_only) {
    const unsigned char* o = static_cast<const unsigned char*>(q->observed);
    j->observed.assign(o, o + (size_t)q->n_steps * q->n_rec * nshot * ts);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t n_bnd = -1;
  if (j->absorbing) {
    const std::vector<int32_t>* d;
    const std::vector<double>* bw;
    boundary_of(*m, &d, &bw);
    n_bnd = (int64_t)d->size();
  }
  j->need = job_device_bytes(*m, j->prec, j->nt, j->nrec, S->per_job_budget, nshot, n_bnd);
  if (j->need > S->budget)
    return Status{KMV_ENOMEM, "request needs " + std::to_string(j->need) + " device bytes, budget is " +
                                  std::to_string(S->budget)};
  if (S->stop) return Status{KMV_ESTATE, "server is shutting down"};
  j->ticket = S->next_ticket++;
  j->t_submit = S->now();
  *ticket = j->ticket;
  S->queue.push_back(j.get());
  S->jobs.emplace(j->ticket, std::move(j));
  S->cv_work.notify_all();
  return OK;
}

namespace {
void fill_result(const Job& j, kmv_result* out) {
  out->status = j.status;
  out->J = j.J;
  out->traces = j.traces.empty() ? nullptr : j.traces.data();
  out->grad = j.grad.empty() ? nullptr : j.grad.data();
  out->n_steps = j.nt;
  out->n_rec = j.nrec;
  out->n_shots = j.nshot;
  out->n_dofs = j.mesh->n_dofs;
  out->t_submit = j.t_submit;
  out->t_admit = j.t_admit;
  out->t_done = j.t_done;
  out->device_bytes = j.need;
}
}  // namespace

Status server_poll(Server* S, uint64_t ticket, kmv_result* out, std::string* msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return Status{KMV_EINVAL, "unknown ticket"};
  const Job& j = *it->second;
  if (!j.done) return Status{KMV_EBUSY, "pending"};
  if (out) fill_result(j, out);
  if (msg) *msg = j.msg;
  return OK;
}

Status server_wait(Server* S, uint64_t ticket, double timeout_s, kmv_result* out, std::string* msg) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return Status{KMV_EINVAL, "unknown ticket"};
  Job* j = it->second.get();
  auto pred = [&]() { return j->done; };
  if (timeout_s < 0) {
    S->cv_done.wait(lk, pred);
  } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return Status{KMV_EBUSY, "pending"};
  }
  if (out) fill_result(*j, out);
  if (msg) *msg = j->msg;
  return OK;
}

Status server_release(Server* S, uint64_t ticket) {
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return Status{KMV_EINVAL, "unknown ticket"};
  if (!it->second->done) return Status{KMV_EBUSY, "pending"};
  S->jobs.erase(it);
  return OK;
}

Status server_stats(Server* S, int* running, int* queued, size_t* bytes_in_use) {
  std::lock_guard<std::mutex> lk(S->mu);
  if (running) *running = S->running;
  if (queued) *queued = (int)S->queue.size();
  if (bytes_in_use) *bytes_in_use = S->used;
  return OK;
}

void server_destroy(Server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Job* j : S->queue) {  // never admitted: cancelled
      j->done = true;
      j->status = KMV_ESTATE;
      j->msg = "server destroyed before the request was admitted";
    }
    S->queue.clear();
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();  // running solves finish first
  for (hipStream_t q : S->streams) (void)hipStreamDestroy(q);
  delete S;
}

}  // namespace kmv
