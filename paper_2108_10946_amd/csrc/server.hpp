// Shot server: continuous admission of independent shot solves onto one GPU.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/kmvwave.h"
#include "mesh.hpp"
#include "problem.hpp"

namespace kmv {

// One request with its host inputs copied, and its result once done.
struct Job {
  uint64_t ticket = 0;
  // request
  Mesh* mesh = nullptr;
  int prec = 0, forward_only = 0, nsrc = 0, nrec = 0, nshot = 1, absorbing = 0;
  double dt = 0, f0 = 0, t0 = 0, amp = 0;
  int64_t nt = 0;
  std::vector<double> c, eta, xs, xr;
  std::vector<double> wavelets;  // [nshot * nt], or empty: the Ricker of f0, t0, amp
  std::vector<unsigned char> observed;
  size_t need = 0;  // device bytes reserved while it runs
  // result
  bool done = false;
  int status = KMV_EBUSY;
  std::string msg;
  double J = 0;
  std::vector<unsigned char> traces;
  std::vector<double> grad;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Server {
  int device = 0;
  size_t budget = 0, used = 0, per_job_budget = 0;
  int slots = 0, running = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;                                   // FIFO of admitted-to-wait jobs
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;  // every job until released
  uint64_t next_ticket = 1;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point epoch;
  double now() const;
};

Status server_create(size_t budget, int slots, Server** out);
Status server_submit(Server* s, Mesh* m, const kmv_request* req, uint64_t* ticket);
// KMV_EBUSY while pending; then the result (its status in out->status, the
// job's error text in *msg).
Status server_poll(Server* s, uint64_t ticket, kmv_result* out, std::string* msg);
Status server_wait(Server* s, uint64_t ticket, double timeout_s, kmv_result* out, std::string* msg);
Status server_release(Server* s, uint64_t ticket);
Status server_stats(Server* s, int* running, int* queued, size_t* bytes_in_use);
void server_destroy(Server* s);

// Upper bound of the device bytes a problem of this size holds (mesh tables,
// vectors, the state storage plan under `budget`, traces) plus the request's
// own buffers.
size_t job_device_bytes(const Mesh& m, int prec, int64_t nt, int nrec, size_t budget, int nshot = 1,
                        int64_t n_bnd = -1);

}  // namespace kmv
