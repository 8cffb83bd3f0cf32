// Serving front end of the TJM library: independent jobs (one whole run
// each, Sec. "Algorithm") submitted as they arrive and executed on one GPU.
//
// Trajectories of a job are independent of other jobs, so jobs share the
// device freely: each admitted job runs on a stream of its own through the
// same begin/advance/end path as tjm_run.  Admission is first come, first
// served: the oldest waiting job starts as soon as an executor is free and
// its device-memory footprint fits in what the budget has left; a younger
// job never overtakes it.  A job larger than the whole budget is refused at
// submission.  See include/tjm.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "tjm.h"
#include "tjm_internal.h"

namespace {

typedef std::chrono::steady_clock Clock;

// executors: concurrent jobs, one HIP stream each (the hardware queues a
// process gets by default)
constexpr int kExecutors = 4;

struct Job {
  uint64_t id = 0;
  tjm_model* model = nullptr;          // the server's own copy
  int n_traj = 0, chi_max = 0, n_obs = 0;
  int n_out = 0;                       // output columns: n_obs site observables + the model's MPO observables
  double dt = 0, T = 0;
  uint64_t seed = 0;
  std::vector<int> obs_site;
  std::vector<double> obs_op;
  tjm_options opt{};
  size_t bytes = 0;
  int n_steps = 0;
  int done = 0;
  int waited = 0;                      // a tjm_wait call has claimed the job
  tjm_status status = TJM_OK;
  std::string err;
  std::vector<double> mean, sem;
  tjm_stats stats{};
  Clock::time_point t_submit, t_start, t_done;
};

thread_local std::string t_err;

tjm_status sfail(tjm_status st, const std::string& msg) {
  t_err = msg;
  return st;
}

}  // namespace

struct tjm_server {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> queue;              // waiting, oldest first
  std::map<uint64_t, Job*> jobs;       // every job not yet collected by tjm_wait
  size_t active_bytes = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> exec;
};

static void run_job(Job* j) {
  const long entries = (long)(j->n_steps + 1) * j->n_out;
  j->mean.assign(std::max<long>(entries, 1), 0.0);
  j->sem.assign(std::max<long>(entries, 1), 0.0);
  j->status = tjm_run(j->model, j->n_traj, j->dt, j->T, j->chi_max, j->n_obs,
                      j->obs_site.empty() ? nullptr : j->obs_site.data(),
                      j->obs_op.empty() ? nullptr : j->obs_op.data(), j->seed, &j->opt,
                      j->mean.data(), j->sem.data());
  if (j->status != TJM_OK) j->err = tjm_last_error(j->model);
  tjm_get_stats(j->model, &j->stats);
}

static void executor(tjm_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv.wait(lk, [s] {
      return s->stop || (!s->queue.empty() && s->active_bytes + s->queue.front()->bytes <= s->budget);
    });
    if (s->stop) return;
    Job* j = s->queue.front();
    s->queue.pop_front();
    s->active_bytes += j->bytes;
    j->t_start = Clock::now();
    lk.unlock();
    run_job(j);
    lk.lock();
    j->t_done = Clock::now();
    j->done = 1;
    s->active_bytes -= j->bytes;
    s->cv.notify_all();
  }
}

extern "C" tjm_status tjm_server_create(tjm_server** out, int device, size_t hbm_budget_bytes) {
  if (!out) return sfail(TJM_E_INVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return sfail(TJM_E_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return sfail(TJM_E_INVAL, "device ordinal out of range");
  int prev = 0;
  (void)hipGetDevice(&prev);
  size_t freeb = 0, totalb = 0;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMemGetInfo(&freeb, &totalb);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return sfail(TJM_E_DEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
  tjm_server* s = new (std::nothrow) tjm_server();
  if (!s) return sfail(TJM_E_NOMEM, "host allocation failed");
  s->device = device;
  s->budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : (size_t)(0.85 * (double)freeb);
  try {
    for (int i = 0; i < kExecutors; ++i) s->exec.emplace_back(executor, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    for (auto& t : s->exec) t.join();
    delete s;
    return sfail(TJM_E_NOMEM, "could not start executor threads");
  }
  *out = s;
  return TJM_OK;
}

extern "C" tjm_status tjm_submit(tjm_server* s, const tjm_model* m, const tjm_run_args* a, uint64_t* job) {
  if (!s || !m || !a || !job) return sfail(TJM_E_INVAL, "NULL argument");
  *job = 0;
  if (a->n_obs < 0 || (a->n_obs > 0 && (!a->obs_site || !a->obs_op)))
    return sfail(TJM_E_INVAL, "bad observables");
  Job* j = new (std::nothrow) Job();
  if (!j) return sfail(TJM_E_NOMEM, "host allocation failed");
  j->model = tjm_model_copy(m);
  if (!j->model) {
    delete j;
    return sfail(TJM_E_NOMEM, "host allocation failed");
  }
  const int d = tjm_model_d(m);
  j->n_traj = a->n_traj; j->dt = a->dt; j->T = a->T; j->chi_max = a->chi_max; j->n_obs = a->n_obs;
  j->n_out = a->n_obs + tjm_model_n_mpo_obs(j->model);
  j->seed = a->seed;
  try {
    if (a->n_obs > 0) {
      j->obs_site.assign(a->obs_site, a->obs_site + a->n_obs);
      j->obs_op.assign(a->obs_op, a->obs_op + 2L * a->n_obs * d * d);
    }
  } catch (...) {
    tjm_destroy(j->model);
    delete j;
    return sfail(TJM_E_NOMEM, "host allocation failed");
  }
  tjm_default_options(&j->opt);
  if (a->opt) j->opt = *a->opt;
  j->opt.device = s->device;
  // size the job with the checks of a run; the caller's current device is kept
  int prev = 0;
  (void)hipGetDevice(&prev);
  int workers = 1;
  tjm_status st = tjm_run_footprint(j->model, j->n_traj, j->dt, j->T, j->chi_max, j->n_obs,
                                    j->obs_site.empty() ? nullptr : j->obs_site.data(),
                                    j->obs_op.empty() ? nullptr : j->obs_op.data(), &j->opt, &j->bytes,
                                    &workers);
  (void)hipSetDevice(prev);
  if (st != TJM_OK) {
    std::string msg = tjm_last_error(j->model);
    tjm_destroy(j->model);
    delete j;
    return sfail(st, msg);
  }
  if (j->bytes > s->budget) {
    tjm_destroy(j->model);
    delete j;
    return sfail(TJM_E_NOMEM, "job needs more device memory than the server's budget");
  }
  j->opt.workers = workers;      // the footprint above assumed at most this many
  j->n_steps = (int)std::lround(j->T / j->dt);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) {
      tjm_destroy(j->model);
      delete j;
      return sfail(TJM_E_BUSY, "server is shutting down");
    }
    j->id = s->next_id++;
    j->t_submit = Clock::now();
    s->jobs[j->id] = j;
    s->queue.push_back(j);
    *job = j->id;
  }
  s->cv.notify_all();
  return TJM_OK;
}

extern "C" tjm_status tjm_poll(tjm_server* s, uint64_t job, int* done) {
  if (!s || !done) return sfail(TJM_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return sfail(TJM_E_INVAL, "unknown job");
  *done = it->second->done;
  return TJM_OK;
}

extern "C" tjm_status tjm_wait(tjm_server* s, uint64_t job, double* mean, double* sem, tjm_job_report* rep) {
  if (!s) return sfail(TJM_E_INVAL, "server is NULL");
  Job* j = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job);
    if (it == s->jobs.end()) return sfail(TJM_E_INVAL, "unknown job");
    j = it->second;
    if (j->waited) return sfail(TJM_E_BUSY, "another call is already waiting for this job");
    j->waited = 1;
    s->cv.wait(lk, [j] { return j->done != 0; });
    s->jobs.erase(j->id);
  }
  const long entries = (long)(j->n_steps + 1) * j->n_out;
  if (j->status == TJM_OK) {
    if (mean) std::copy(j->mean.begin(), j->mean.begin() + entries, mean);
    if (sem) std::copy(j->sem.begin(), j->sem.begin() + entries, sem);
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    auto sec = [](Clock::duration x) { return std::chrono::duration<double>(x).count(); };
    rep->latency_s = sec(j->t_done - j->t_submit);
    rep->queue_s = sec(j->t_start - j->t_submit);
    rep->run_s = sec(j->t_done - j->t_start);
    rep->start_s = sec(j->t_start.time_since_epoch());
    rep->end_s = sec(j->t_done.time_since_epoch());
    rep->n_traj = j->n_traj;
    rep->n_steps = j->n_steps;
    rep->device_bytes = j->bytes;
    rep->stats = j->stats;
  }
  const tjm_status st = j->status;
  if (st != TJM_OK) t_err = j->err;
  tjm_destroy(j->model);
  delete j;
  return st;
}

extern "C" const char* tjm_server_last_error(void) { return t_err.c_str(); }

extern "C" void tjm_server_destroy(tjm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->exec) t.join();
  for (auto& kv : s->jobs) {
    tjm_destroy(kv.second->model);
    delete kv.second;
  }
  delete s;
}
