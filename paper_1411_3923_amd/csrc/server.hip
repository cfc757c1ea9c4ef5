// Serving runtime: many optimisation runs (sessions) share one GPU.
//
// A session is one robust topology-optimisation run on its own mesh: a
// tpcg handle whose factors and coarse space stay resident in device memory
// across design updates, its own HIP stream and a worker thread. Sessions are
// admitted against a device-memory budget and a cap on concurrent sessions;
// a refused open returns TPCG_EAGAIN and leaves nothing allocated, so a
// caller retries when a session closes. A job is one design update of a
// session: the density pipeline of its realisations (Sec. 4.3, Sec. 4.4),
// the preconditioner rebuild decided by the iteration-count rule of Sec. 5.2,
// the batched PCG solve of the realisations warm-started from the previous
// displacements (Sec. 5.2), compliance and sensitivities and their chain
// rule. Jobs of one session run in submission order; the workers of
// different sessions run concurrently, so their kernels overlap on the
// device.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "tpcg_internal.h"

namespace tpcg {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Job {
  int64_t id = 0;
  int64_t session = 0;
  const double* rho = nullptr;
  const double* f = nullptr;
  double* u = nullptr;
  double* c = nullptr;
  double* dc = nullptr;
  tpcg_job_opts o{};
  Clock::time_point submitted;
  tpcg_job_result res{};
  bool done = false;
};

struct Server;

struct Session {
  int64_t id = 0;
  Server* srv = nullptr;
  tpcg_problem prob{};
  int nsys = 0;
  int64_t nel = 0;
  size_t bytes = 0;
  tpcg_handle* h = nullptr;
  hipStream_t stream = nullptr;
  double* rt = nullptr;    // filtered design [n_el]
  double* rb = nullptr;    // physical densities [nsys][n_el]
  double* dcb = nullptr;   // sensitivities to the physical densities [nsys][n_el]
  double* mnd = nullptr;   // non-discreteness of the representative realisation [1]
  std::thread worker;
  std::deque<Job*> queue;
  bool closing = false;
  // rebuild rule state (Sec. 5.2)
  int built = 0;
  int ref_iters = 0;       // lowest count since the last rebuild
  int last_iters = 0;
  int rebuilds = 0;
};

struct Server {
  size_t budget = 0, used = 0;
  int max_active = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;    // a job finished or a queue changed
  std::map<int64_t, Session*> sessions;
  std::map<int64_t, Job*> jobs;
  int64_t next_id = 1;
};

// the job, run by the session's worker thread on the session's stream
void run_job(Session* s, Job* j) {
  const tpcg_job_opts& o = j->o;
  tpcg_job_result& r = j->res;
  const auto t0 = Clock::now();
  r.queue_ms = ms_between(j->submitted, t0);
  tpcg_handle* h = s->h;
  const int ns = s->nsys;
  int rc = TPCG_OK;
  if (o.rmin > 0.0) {
    rc = tpcg_filter_project(h, j->rho, o.rmin, o.beta, o.eta, ns, s->rt, s->rb);
  } else {
    for (int q = 0; q < ns && rc == TPCG_OK; ++q)
      if (hipMemcpyAsync(s->rb + (size_t)q * s->nel, j->rho, sizeof(double) * s->nel,
                         hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        rc = TPCG_EHIP;
  }
  // rebuild: no preconditioner yet, forced, or (rule) the last solve took
  // more than `growth` times the lowest count since the last rebuild
  bool rebuild = !s->built || o.rebuild > 0 ||
                 (o.rebuild == 0 && s->last_iters > o.growth * (double)s->ref_iters);
  const auto t1 = Clock::now();
  bool refactored = false;
  if (rc == TPCG_OK && rebuild) {
    rc = tpcg_build_coarse_basis(h, s->rb, ns, o.rep);
    if (rc == TPCG_OK) {
      s->built = 1;
      ++s->rebuilds;
    }
  } else if (rc == TPCG_OK && o.refactor) {
    rc = tpcg_refactor(h, s->rb, ns);
    refactored = rc == TPCG_OK;
  }
  const auto t2 = Clock::now();
  tpcg_info info[kMaxSys];
  if (rc == TPCG_OK) {
    const int st = tpcg_pcg_solve(h, s->rb, j->f, j->u, ns, o.rtol, o.maxit, info);
    if (st < 0) rc = st;
  }
  const auto t3 = Clock::now();
  if (rc == TPCG_OK) rc = tpcg_compliance_and_sensitivity(h, s->rb, j->u, j->f, ns, j->c,
                                                          j->dc ? s->dcb : nullptr);
  if (rc == TPCG_OK && j->dc) {
    if (o.rmin > 0.0)
      rc = tpcg_filter_project_adjoint(h, s->rt, o.rmin, o.beta, o.eta, ns, s->dcb, j->dc);
    else if (hipMemcpyAsync(j->dc, s->dcb, sizeof(double) * ns * s->nel, hipMemcpyDeviceToDevice,
                            s->stream) != hipSuccess)
      rc = TPCG_EHIP;
  }
  if (rc == TPCG_OK) rc = tpcg_nondiscreteness(h, s->rb + (size_t)o.rep * s->nel, s->mnd);
  double mnd = 0.0;
  if (rc == TPCG_OK &&
      (hipMemcpyAsync(&mnd, s->mnd, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
       hipStreamSynchronize(s->stream) != hipSuccess))
    rc = TPCG_EHIP;
  const auto t4 = Clock::now();
  int worst = 0;
  for (int q = 0; q < ns; ++q) {
    r.iters[q] = rc == TPCG_OK ? info[q].iters : 0;
    r.status[q] = rc == TPCG_OK ? info[q].status : rc;
    r.relres[q] = rc == TPCG_OK ? info[q].relres : 0.0;
    r.true_relres[q] = rc == TPCG_OK ? info[q].true_relres : 0.0;
    if (r.iters[q] > worst) worst = r.iters[q];
  }
  r.status_all = rc;
  r.rebuilt = rebuild && rc == TPCG_OK ? 1 : 0;
  r.refactored = refactored ? 1 : 0;
  r.rebuilds = s->rebuilds;
  r.build_ms = ms_between(t1, t2);
  r.solve_ms = ms_between(t2, t3);
  r.total_ms = ms_between(t0, t4);
  r.m_nd = mnd;
  if (rc == TPCG_OK) {
    // reference count of the rule: the count right after a rebuild, then the
    // lowest one since (warm starts lower the count after a rebuild)
    if (r.rebuilt || worst < s->ref_iters) s->ref_iters = worst;
    s->last_iters = worst;
  }
}

void worker_loop(Session* s) {
  Server* srv = s->srv;
  hipSetDevice(srv->device);
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] { return s->closing || !s->queue.empty(); });
      if (s->queue.empty()) return;   // closing and drained
      j = s->queue.front();
    }
    run_job(s, j);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      s->queue.pop_front();
      j->done = true;
    }
    srv->cv.notify_all();
  }
}

size_t session_bytes(const tpcg_problem& pr, int nsys) {
  const size_t ws = tpcg_workspace_bytes(&pr, nsys);
  if (!ws) return 0;
  const int64_t nel = (int64_t)pr.nel[0] * pr.nel[1] * (pr.dim == 3 ? pr.nel[2] : 1);
  return ws + sizeof(double) * ((size_t)nel * (1 + 2 * (size_t)nsys) + 1);
}

void free_session(Session* s) {
  if (s->h) tpcg_destroy(s->h);
  for (double* p : {s->rt, s->rb, s->dcb, s->mnd})
    if (p) hipFree(p);
  if (s->stream) hipStreamDestroy(s->stream);
  (void)hipGetLastError();
}

Server* S(tpcg_server* p) { return reinterpret_cast<Server*>(p); }

}  // namespace
}  // namespace tpcg

using namespace tpcg;

extern "C" {

int tpcg_server_create(size_t budget_bytes, int32_t max_active, tpcg_server** out) {
  if (!out || budget_bytes == 0 || max_active < 1) return TPCG_EINVAL;
  *out = nullptr;
  Server* s = new (std::nothrow) Server();
  if (!s) return TPCG_ENOMEM;
  s->budget = budget_bytes;
  s->max_active = max_active;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return TPCG_EHIP;
  }
  *out = reinterpret_cast<tpcg_server*>(s);
  return TPCG_OK;
}

size_t tpcg_server_session_bytes(const tpcg_problem* prob, int32_t nsys) {
  return prob ? session_bytes(*prob, nsys) : 0;
}

int tpcg_server_open(tpcg_server* sv, const tpcg_problem* prob, const uint8_t* fixed_mask,
                     int32_t nsys, int64_t* session) {
  Server* srv = S(sv);
  if (!srv || !prob || !fixed_mask || !session) return TPCG_EINVAL;
  if (nsys < 1 || nsys > prob->nsys_max) return TPCG_EINVAL;
  const size_t bytes = session_bytes(*prob, nsys);
  if (!bytes) return TPCG_EINVAL;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (bytes > srv->budget) return TPCG_EINVAL;    // could never be admitted
    if (srv->used + bytes > srv->budget || (int)srv->sessions.size() >= srv->max_active)
      return TPCG_EAGAIN;
    srv->used += bytes;                             // reserved while the session is set up
  }
  Session* s = new (std::nothrow) Session();
  int rc = s ? TPCG_OK : TPCG_ENOMEM;
  if (rc == TPCG_OK) {
    s->srv = srv;
    s->prob = *prob;
    s->nsys = nsys;
    s->bytes = bytes;
    s->nel = (int64_t)prob->nel[0] * prob->nel[1] * (prob->dim == 3 ? prob->nel[2] : 1);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) rc = TPCG_EHIP;
  }
  if (rc == TPCG_OK) rc = tpcg_build_partition(prob, fixed_mask, s->stream, &s->h);
  // a session solves many times: its handle tunes its launches (bitwise neutral)
  if (rc == TPCG_OK) tpcg_set_autotune(s->h, 1);
  if (rc == TPCG_OK) {
    void* p[4] = {nullptr, nullptr, nullptr, nullptr};
    const size_t n[4] = {(size_t)s->nel, (size_t)nsys * s->nel, (size_t)nsys * s->nel, 1};
    for (int i = 0; i < 4 && rc == TPCG_OK; ++i)
      if (!device_alloc(&p[i], sizeof(double) * n[i])) rc = TPCG_ENOMEM;
    s->rt = static_cast<double*>(p[0]);
    s->rb = static_cast<double*>(p[1]);
    s->dcb = static_cast<double*>(p[2]);
    s->mnd = static_cast<double*>(p[3]);
  }
  if (rc != TPCG_OK) {
    if (s) {
      free_session(s);
      delete s;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->used -= bytes;
    return rc;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    s->id = srv->next_id++;
    srv->sessions[s->id] = s;
    *session = s->id;
  }
  s->worker = std::thread(worker_loop, s);
  return TPCG_OK;
}

int tpcg_server_submit(tpcg_server* sv, int64_t session, const double* rho, const double* f,
                       double* u, double* c, double* dc, const tpcg_job_opts* opts, int64_t* job) {
  Server* srv = S(sv);
  if (!srv || !rho || !f || !u || !c || !opts || !job) return TPCG_EINVAL;
  if (!(opts->rtol > 0.0) || opts->maxit < 0 || !(opts->growth >= 1.0)) return TPCG_EINVAL;
  Job* j = new (std::nothrow) Job();
  if (!j) return TPCG_ENOMEM;
  j->rho = rho;
  j->f = f;
  j->u = u;
  j->c = c;
  j->dc = dc;
  j->o = *opts;
  j->session = session;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end() || it->second->closing) {
      delete j;
      return TPCG_EINVAL;
    }
    if (opts->rep < 0 || opts->rep >= it->second->nsys) {
      delete j;
      return TPCG_EINVAL;
    }
    j->id = srv->next_id++;
    j->submitted = Clock::now();
    srv->jobs[j->id] = j;
    it->second->queue.push_back(j);
    *job = j->id;
  }
  srv->cv.notify_all();
  return TPCG_OK;
}

int tpcg_server_wait(tpcg_server* sv, int64_t job, tpcg_job_result* out) {
  Server* srv = S(sv);
  if (!srv || !out) return TPCG_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(job);
  if (it == srv->jobs.end()) return TPCG_EINVAL;
  Job* j = it->second;
  srv->cv.wait(lk, [&] { return j->done; });
  *out = j->res;
  srv->jobs.erase(it);
  delete j;
  return TPCG_OK;
}

int tpcg_server_test(tpcg_server* sv, int64_t job, tpcg_job_result* out) {
  Server* srv = S(sv);
  if (!srv || !out) return TPCG_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(job);
  if (it == srv->jobs.end()) return TPCG_EINVAL;
  if (!it->second->done) return TPCG_EAGAIN;
  *out = it->second->res;
  delete it->second;
  srv->jobs.erase(it);
  return TPCG_OK;
}

int tpcg_server_close(tpcg_server* sv, int64_t session) {
  Server* srv = S(sv);
  if (!srv) return TPCG_EINVAL;
  Session* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end() || it->second->closing) return TPCG_EINVAL;
    s = it->second;
    s->closing = true;
  }
  srv->cv.notify_all();
  s->worker.join();   // its queued jobs run first
  free_session(s);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->used -= s->bytes;
    srv->sessions.erase(session);
  }
  delete s;
  srv->cv.notify_all();
  return TPCG_OK;
}

size_t tpcg_server_free_bytes(const tpcg_server* sv) {
  Server* srv = S(const_cast<tpcg_server*>(sv));
  if (!srv) return 0;
  std::lock_guard<std::mutex> lk(srv->mu);
  return srv->budget - srv->used;
}

void tpcg_server_destroy(tpcg_server* sv) {
  Server* srv = S(sv);
  if (!srv) return;
  std::vector<int64_t> ids;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto& kv : srv->sessions) ids.push_back(kv.first);
  }
  for (int64_t id : ids) tpcg_server_close(sv, id);
  for (auto& kv : srv->jobs) delete kv.second;
  delete srv;
}

}  // extern "C"
