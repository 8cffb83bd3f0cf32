// Serving front end of the TJM library: independent jobs (one whole run
// each, Sec. "Algorithm") submitted as they arrive and executed on one GPU
// with continuous batching at the level of trajectories.
//
// Trajectories are independent of each other and of other jobs (Eq.
// TJMExpVal averages within a job), so the server keeps one resident work
// queue per contraction precision: a persistent kernel (tjm_serve_kernel)
// whose workgroups take (job, trajectory) items in arrival order and run
// each trajectory whole, F_0 to F_n.  Jobs of any chain length, bond
// dimension and model share that queue: the trajectories of a job admitted
// while others run are taken as soon as workgroups free up, next to the
// rest.  Each workgroup's scratch is a slot of its queue's pool.  A job too
// large for the current pool of its precision waits until that queue has
// drained; the idle queue is released and a new one opens with a pool
// shaped for every waiting job of the precision that the budget allows, so
// that a stream of mixed shapes reshapes the pool rarely and never runs two
// resident kernels of one precision against each other.
//
// A dispatcher thread admits jobs first come, first served (the oldest
// waiting job is admitted once its buffers, and any new pool it needs, fit
// in what the budget has left; a younger job never overtakes it), appends
// their items, (re)launches the resident kernel whenever items are pending
// and it has exited (it exits by itself when idle), and finishes a job
// (reduction, copies, release) once all of its items are marked done.
// Results are bit-identical to tjm_run with the same arguments: each
// trajectory runs the same device code on the same data.  See include/tjm.h
// for the contract.
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

constexpr int kMaxJobs = 256;          // parameter slots per pool (jobs in flight)
constexpr int kCap = 1 << 20;          // ring of work items per pool
// sleeps (about 3.4 us each) an idle workgroup waits for new items before it
// exits: long enough that the workgroups of a resident kernel stay for the
// next request of a stream, short enough that an idle kernel soon frees
// the device
constexpr int kIdleSpins = 150000;

struct Pool;

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
  size_t bytes = 0;                    // the job's own device buffers (scratch is the pool's)
  long stride = 0;                     // scratch one of its workgroups needs
  int L = 0;
  int n_steps = 0;
  int done = 0;
  int waited = 0;                      // a tjm_wait call has claimed the job
  tjm_status status = TJM_OK;
  std::string err;
  std::vector<double> mean, sem;
  tjm_stats stats{};
  Clock::time_point t_submit, t_start, t_done;
  // while admitted
  Pool* pool = nullptr;
  void* run = nullptr;
  int slot = -1;
  unsigned first = 0;                  // its items are first .. first + n_traj - 1
  int seen = 0;                        // items known done
  size_t pool_bytes = 0;
};

// The resident queue of one contraction precision.
struct Pool {
  int mixed = 0;
  char* scratch = nullptr;
  long stride = 0;
  int workers = 0;
  int L_max = 0;
  size_t bytes = 0;                    // scratch bytes held
  hipStream_t stream = nullptr;
  TjmParams* d_params = nullptr;       // [kMaxJobs]
  unsigned* d_head = nullptr;
  ServeShared* sh = nullptr;           // host-coherent
  ServeItem* items = nullptr;          // host-coherent [kCap]
  int* done = nullptr;                 // host-coherent [kCap]
  unsigned long long* steps = nullptr; // host-coherent [kMaxJobs]: step functions finished per slot
  int* d_count = nullptr;              // [kMaxJobs] trajectories finished per slot (device)
  unsigned pushed = 0;
  int active = 0;                      // admitted jobs not yet finished
  bool retired = false;                // takes no new job; released once drained
  std::vector<int> free_slots;
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
  int n_cu = 0;
  std::mutex mu;
  std::condition_variable cv;          // job state changes (waiters)
  std::condition_variable wake;        // new work for the dispatcher
  std::deque<Job*> queue;              // waiting, oldest first
  std::vector<Job*> active;            // admitted, not finished
  std::map<uint64_t, Job*> jobs;       // every job not yet collected by tjm_wait
  size_t active_bytes = 0;             // admitted jobs' buffers plus the pools
  uint64_t next_id = 1;
  bool stop = false;
  std::vector<Pool*> pools[2];         // FP64, mixed: queues, the newest last
  long floor_stride[2] = {0, 0};       // tjm_server_reserve: least pool shape per precision
  int floor_L[2] = {0, 0};
  // finished jobs whose buffers await release: freeing device memory waits
  // for the whole device, so it happens only while no resident kernel runs
  // (the bytes stay counted in active_bytes until then)
  std::vector<std::pair<void*, size_t>> graveyard;
  // streams of the server's lifetime, each put to use once at creation,
  // before any resident kernel runs: the resident kernels' (one per
  // precision; a queue's successor opens only after it has been released)
  // and the one that carries every job's uploads
  hipStream_t kstream[2] = {nullptr, nullptr};
  hipStream_t up_stream = nullptr;
  char* d_touch = nullptr;             // target of those first copies (freed with the server)
  std::thread dispatcher;
};

// A resident kernel's stream carries only that kernel, which occupies the
// stream's hardware queue until it exits.  Ordinary streams share the
// process's few hardware queues, so a job's uploads on a stream that landed
// on the same queue would wait for the kernel; a stream created with a CU
// mask (here all compute units) gets a hardware queue of its own.  The
// server issues nothing on the null stream, which would wait for this one.
static hipError_t stream_create(hipStream_t* st, int n_cu, bool own_queue, char* d_touch) {
  hipError_t e = hipErrorUnknown;
  if (own_queue) {
    std::vector<uint32_t> mask((size_t)(n_cu + 31) / 32, 0xffffffffu);
    e = hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data());
    if (e != hipSuccess) (void)hipGetLastError();
  }
  if (e != hipSuccess) e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  // first use: a small copy, so that whatever the runtime sets up for the
  // stream happens now, not behind a running resident kernel
  static const char zero[64] = {};
  e = hipMemcpyAsync(d_touch, zero, sizeof zero, hipMemcpyHostToDevice, *st);
  if (e == hipSuccess) e = hipStreamSynchronize(*st);
  return e;
}

static hipError_t pool_init(Pool& p, int mixed, hipStream_t stream) {
  p.mixed = mixed;
  p.stream = stream;                   // the server's, for this precision
  hipError_t e = hipMalloc((void**)&p.d_params, sizeof(TjmParams) * kMaxJobs);
  if (e == hipSuccess) e = hipMalloc((void**)&p.d_head, 256);
  if (e == hipSuccess) e = hipMalloc((void**)&p.d_count, sizeof(int) * kMaxJobs);
  // zeroed by copies (no fill kernel: another queue's resident kernel may
  // hold every compute unit)
  std::vector<char> zero(std::max<size_t>(256, sizeof(int) * kMaxJobs), 0);
  if (e == hipSuccess) e = hipMemcpyAsync(p.d_head, zero.data(), 256, hipMemcpyHostToDevice, p.stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p.d_count, zero.data(), sizeof(int) * kMaxJobs, hipMemcpyHostToDevice, p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p.sh, sizeof(ServeShared), hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p.items, sizeof(ServeItem) * (size_t)kCap, hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p.done, sizeof(int) * (size_t)kCap, hipHostMallocCoherent);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&p.steps, sizeof(unsigned long long) * kMaxJobs, hipHostMallocCoherent);
  if (e != hipSuccess) return e;
  std::memset(p.steps, 0, sizeof(unsigned long long) * kMaxJobs);
  std::memset(p.sh, 0, sizeof(ServeShared));
  std::memset(p.done, 0, sizeof(int) * (size_t)kCap);
  for (int i = kMaxJobs - 1; i >= 0; --i) p.free_slots.push_back(i);
  return hipSuccess;
}

static void pool_free(Pool& p) {
  if (p.stream) (void)hipStreamSynchronize(p.stream);
  if (p.scratch) (void)hipFree(p.scratch);
  if (p.d_params) (void)hipFree(p.d_params);
  if (p.d_head) (void)hipFree(p.d_head);
  if (p.d_count) (void)hipFree(p.d_count);
  if (p.sh) (void)hipHostFree(p.sh);
  if (p.items) (void)hipHostFree(p.items);
  if (p.done) (void)hipHostFree(p.done);
  if (p.steps) (void)hipHostFree(p.steps);
  p = Pool();
}

static bool pool_running(Pool& p) { return hipStreamQuery(p.stream) == hipErrorNotReady; }

// Workgroups of the resident kernel for chains up to L: what the compute
// units hold, less one per 32 compute units (one per XCD on MI355X), so
// that copies the runtime runs as small kernels (from pageable memory, for
// one: the zeroed counters of a queue that opens while the other
// precision's kernel runs) find room instead of waiting for it to exit.
static int pool_workers(tjm_server* s, int mixed, int L) {
  int bpc = 1;
  if (tjm_blocks_per_cu(mixed, L, &bpc) != hipSuccess || bpc < 1) bpc = 1;
  return std::max(1, bpc * s->n_cu - std::max(1, s->n_cu / 32));
}

// The shape of a pool that serves the current pool's jobs and j.
static void pool_shape(const Pool* cur, const Job* j, long* stride, int* L) {
  *stride = cur ? std::max(cur->stride, j->stride) : j->stride;
  *L = cur ? std::max(cur->L_max, j->L) : j->L;
}

static size_t pool_bytes_for(tjm_server* s, int mixed, long stride, int L) {
  return (size_t)pool_workers(s, mixed, L) * (size_t)stride;
}

// A new queue with a scratch pool of the given shape; the caller holds the
// lock and has checked the budget.
static hipError_t pool_open(tjm_server* s, int mixed, long stride, int L, Pool** out) {
  Pool* p = new (std::nothrow) Pool();
  if (!p) return hipErrorOutOfMemory;
  hipError_t e = pool_init(*p, mixed, s->kstream[mixed]);
  const int w = pool_workers(s, mixed, L);
  if (e == hipSuccess) e = hipMalloc((void**)&p->scratch, (size_t)w * (size_t)stride);
  if (e != hipSuccess) {
    pool_free(*p);
    delete p;
    return e;
  }
  p->stride = stride;
  p->L_max = L;
  p->workers = w;
  p->bytes = (size_t)w * (size_t)stride;
  s->active_bytes += p->bytes;
  for (Pool* o : s->pools[mixed]) o->retired = true;
  s->pools[mixed].push_back(p);
  *out = p;
  return hipSuccess;
}

// the queue new jobs of a precision go to, or null
static Pool* current_pool(tjm_server* s, int q) {
  if (s->pools[q].empty() || s->pools[q].back()->retired) return nullptr;
  return s->pools[q].back();
}

// the job's slot is free again; its buffers go to the graveyard
static void release_slot(tjm_server* s, Job* j, void* run) {
  j->pool->free_slots.push_back(j->slot);
  j->pool->active--;
  if (run) s->graveyard.emplace_back(run, j->bytes);
  else s->active_bytes -= j->bytes;
}

static bool any_running(tjm_server* s) {
  for (int q = 0; q < 2; ++q)
    for (Pool* p : s->pools[q])
      if (pool_running(*p)) return true;
  return false;
}

static void mark_done(tjm_server* s, Job* j) {
  j->t_done = Clock::now();
  j->done = 1;
  s->cv.notify_all();
}

static void finish_job(tjm_server* s, Job* j, std::unique_lock<std::mutex>& lk) {
  const long entries = (long)(j->n_steps + 1) * j->n_out;
  j->mean.assign(std::max<long>(entries, 1), 0.0);
  j->sem.assign(std::max<long>(entries, 1), 0.0);
  void* run = j->run;
  lk.unlock();
  const tjm_status st = tjm_pool_finish(j->model, run, j->mean.data(), j->sem.data(), &j->stats);
  lk.lock();
  j->status = st;
  if (st != TJM_OK) j->err = tjm_last_error(j->model);
  j->run = nullptr;
  release_slot(s, j, run);
  mark_done(s, j);
}

// Whether n more items fit in the pool's ring: the new indices must not
// reach the oldest item whose completion has not been observed yet.
static bool ring_has_room(tjm_server* s, const Pool& p, int n) {
  unsigned in_flight = 0;              // items from the oldest unobserved one on (wrap-safe differences)
  for (const Job* j : s->active)
    if (j->pool == &p) in_flight = std::max(in_flight, p.pushed - (j->first + (unsigned)j->seen));
  return (unsigned long long)in_flight + (unsigned)n <= (unsigned long long)kCap;
}

// Admits the oldest waiting job if it fits; returns false if it must wait.
static bool admit_front(tjm_server* s, std::unique_lock<std::mutex>& lk) {
  Job* j = s->queue.front();
  const int q = j->opt.precision == TJM_PREC_MIXED ? 1 : 0;
  Pool* cur = current_pool(s, q);
  // One resident queue per precision at a time (two persistent kernels that
  // each fill the device would take compute units from each other in no
  // useful order).  A job larger than the current pool waits until that
  // queue has drained; the idle queue is then released, and the next pool
  // is shaped for every waiting job of the precision that the budget allows.
  const bool fits = cur && j->stride <= cur->stride && j->L <= cur->L_max;
  if (cur && !fits) {
    if (cur->active == 0) cur->retired = true;
    return false;
  }
  if (!cur)
    for (Pool* o : s->pools[q])
      if (o->retired) return false;                             // still being released
  if (fits && (cur->free_slots.empty() || !ring_has_room(s, *cur, j->n_traj))) return false;
  long stride = 0;
  int Lp = 0;
  if (!fits) {
    pool_shape(nullptr, j, &stride, &Lp);
    for (const Job* w : s->queue) {                             // the front job first
      if ((w->opt.precision == TJM_PREC_MIXED ? 1 : 0) != q) continue;
      const long ws = std::max(stride, w->stride);
      const int wl = std::max(Lp, w->L);
      if (s->active_bytes + j->bytes + pool_bytes_for(s, q, ws, wl) > s->budget) break;
      stride = ws;
      Lp = wl;
    }
    // the reserved shape too, where the budget allows it
    const long fs = std::max(stride, s->floor_stride[q]);
    const int fl = std::max(Lp, s->floor_L[q]);
    if (s->active_bytes + j->bytes + pool_bytes_for(s, q, fs, fl) <= s->budget) {
      stride = fs;
      Lp = fl;
    }
  }
  const size_t extra = fits ? 0 : pool_bytes_for(s, q, stride, Lp);
  if (s->active_bytes + j->bytes + extra > s->budget) {
    // no room: idle queues of either precision give up their pools (they are
    // released once their kernels have exited), and the job waits
    if (!fits)
      for (int r = 0; r < 2; ++r)
        for (Pool* o : s->pools[r])
          if (o->active == 0) o->retired = true;
    return false;
  }
  s->queue.pop_front();
  j->t_start = Clock::now();
  if (!fits) {
    const hipError_t e = pool_open(s, q, stride, Lp, &cur);
    if (e != hipSuccess) {
      j->status = e == hipErrorOutOfMemory ? TJM_E_NOMEM : TJM_E_DEVICE;
      j->err = std::string("scratch pool: ") + hipGetErrorString(e);
      mark_done(s, j);
      return true;
    }
  }
  Pool& p = *cur;
  j->pool = &p;
  j->slot = p.free_slots.back();
  p.free_slots.pop_back();
  p.active++;
  s->active_bytes += j->bytes;
  j->pool_bytes = p.bytes;
  char* scratch = p.scratch;
  const long pstride = p.stride;
  const int workers = p.workers;
  lk.unlock();
  void* run = nullptr;
  TjmParams P;
  std::string err;
  tjm_status st = tjm_pool_prepare(j->model, j->n_traj, j->dt, j->T, j->chi_max, j->n_obs,
                                   j->obs_site.empty() ? nullptr : j->obs_site.data(),
                                   j->obs_op.empty() ? nullptr : j->obs_op.data(), j->seed, &j->opt, scratch,
                                   pstride, workers, p.d_params + j->slot, s->up_stream, &run, &P);
  if (st != TJM_OK) err = tjm_last_error(j->model);
  lk.lock();
  if (st != TJM_OK) {
    j->status = st;
    j->err = err;
    release_slot(s, j, run);             // run is null if nothing was allocated
    mark_done(s, j);
    return true;
  }
  j->run = run;
  __atomic_store_n(&p.steps[j->slot], 0ull, __ATOMIC_RELAXED);
  // append the job's trajectories to the ring, then publish them
  j->first = p.pushed;
  for (int t = 0; t < j->n_traj; ++t) {
    const unsigned idx = p.pushed + (unsigned)t;
    p.done[idx % kCap] = 0;
    p.items[idx % kCap] = ServeItem{j->slot, t};
  }
  p.pushed += (unsigned)j->n_traj;
  __atomic_store_n(&p.sh->tail, p.pushed, __ATOMIC_RELEASE);
  s->active.push_back(j);
  return true;
}

// Launches the resident kernel of a pool whose admitted jobs have items
// left and whose previous kernel has exited; on a launch error every job
// of the pool fails.
static void keep_resident(tjm_server* s, Pool& p, std::unique_lock<std::mutex>& lk) {
  if (!p.stream || p.active == 0 || pool_running(p)) return;
  bool pending = false;
  for (Job* j : s->active)
    if (j->pool == &p && j->seen < j->n_traj) { pending = true; break; }
  if (!pending) return;
  ServeDev S;
  S.params = p.d_params; S.items = p.items; S.done = p.done; S.steps = p.steps; S.count = p.d_count; S.sh = p.sh; S.head = p.d_head;
  S.cap = kCap; S.idle_spins = kIdleSpins;
  const hipError_t e = p.mixed ? tjm_launch_serve_float(S, p.workers, p.L_max, p.stream)
                               : tjm_launch_serve_double(S, p.workers, p.L_max, p.stream);
  if (e == hipSuccess) return;
  for (size_t i = 0; i < s->active.size();) {
    Job* j = s->active[i];
    if (j->pool != &p) { ++i; continue; }
    s->active.erase(s->active.begin() + (long)i);
    void* run = j->run;
    j->run = nullptr;
    j->status = TJM_E_DEVICE;
    j->err = std::string("serve kernel launch: ") + hipGetErrorString(e);
    release_slot(s, j, run);
    mark_done(s, j);
  }
}

static void dispatcher(tjm_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admission, first come first served
    while (!s->queue.empty() && !s->stop)
      if (!admit_front(s, lk)) break;
    // finished jobs: every item of the job marked done by the kernel
    for (size_t i = 0; i < s->active.size();) {
      Job* j = s->active[i];
      const Pool& p = *j->pool;
      while (j->seen < j->n_traj &&
             __atomic_load_n(&p.done[(j->first + (unsigned)j->seen) % kCap], __ATOMIC_ACQUIRE))
        ++j->seen;
      if (j->seen == j->n_traj) {
        s->active.erase(s->active.begin() + (long)i);
        finish_job(s, j, lk);
      } else {
        ++i;
      }
    }
    // a resident kernel wherever items are pending (it exits when idle);
    // retired queues are stopped once drained
    for (int q = 0; q < 2; ++q)
      for (Pool* p : s->pools[q]) {
        keep_resident(s, *p, lk);
        if (p->retired && p->active == 0) __atomic_store_n(&p->sh->stop, 1, __ATOMIC_RELEASE);
      }
    // releases that wait for the whole device: only while no resident
    // kernel runs (finished jobs' buffers, drained retired queues)
    if (!any_running(s)) {
      for (auto& g : s->graveyard) {
        tjm_pool_release(g.first);
        s->active_bytes -= g.second;
      }
      s->graveyard.clear();
      for (int q = 0; q < 2; ++q)
        for (size_t i = 0; i < s->pools[q].size();) {
          Pool* p = s->pools[q][i];
          if (p->retired && p->active == 0) {
            s->active_bytes -= p->bytes;
            pool_free(*p);
            delete p;
            s->pools[q].erase(s->pools[q].begin() + (long)i);
            continue;
          }
          ++i;
        }
    }
    if (s->stop && s->active.empty()) break;
    s->wake.wait_for(lk, std::chrono::microseconds(500));
  }
  lk.unlock();
  for (int q = 0; q < 2; ++q)
    for (Pool* p : s->pools[q]) {
      __atomic_store_n(&p->sh->stop, 1, __ATOMIC_RELEASE);
      (void)hipStreamSynchronize(p->stream);
    }
  for (auto& g : s->graveyard) tjm_pool_release(g.first);
  s->graveyard.clear();
}

static void server_streams_destroy(tjm_server* s) {
  for (hipStream_t* st : {&s->kstream[0], &s->kstream[1], &s->up_stream})
    if (*st) {
      (void)hipStreamSynchronize(*st);
      (void)hipStreamDestroy(*st);
      *st = nullptr;
    }
  if (s->d_touch) (void)hipFree(s->d_touch);
  s->d_touch = nullptr;
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
  hipDeviceProp_t prop;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMemGetInfo(&freeb, &totalb);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
  tjm_server* s = nullptr;
  if (e == hipSuccess) {
    s = new (std::nothrow) tjm_server();
    if (!s) e = hipErrorOutOfMemory;
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    delete s;
    return sfail(e == hipErrorOutOfMemory ? TJM_E_NOMEM : TJM_E_DEVICE,
                 std::string("server set-up: ") + hipGetErrorString(e));
  }
  s->device = device;
  s->n_cu = prop.multiProcessorCount;
  if ((e = hipSetDevice(device)) == hipSuccess) {
    e = hipMalloc((void**)&s->d_touch, 64);
    for (int q = 0; q < 2 && e == hipSuccess; ++q) e = stream_create(&s->kstream[q], s->n_cu, true, s->d_touch);
    if (e == hipSuccess) e = stream_create(&s->up_stream, s->n_cu, false, s->d_touch);
    (void)hipSetDevice(prev);
  }
  if (e != hipSuccess) {
    server_streams_destroy(s);
    delete s;
    return sfail(TJM_E_DEVICE, std::string("server streams: ") + hipGetErrorString(e));
  }
  s->budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : (size_t)(0.85 * (double)freeb);
  try {
    s->dispatcher = std::thread(dispatcher, s);
  } catch (...) {
    delete s;
    return sfail(TJM_E_NOMEM, "could not start the dispatcher thread");
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
  j->L = tjm_model_L(j->model);
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
  j->opt.workers = 0;
  // validate and size the job with the checks of a run (no device call)
  tjm_status st = tjm_pool_plan(j->model, j->n_traj, j->dt, j->T, j->chi_max, j->n_obs,
                                j->obs_site.empty() ? nullptr : j->obs_site.data(),
                                j->obs_op.empty() ? nullptr : j->obs_op.data(), &j->opt, &j->stride, &j->bytes);
  if (st != TJM_OK) {
    std::string msg = tjm_last_error(j->model);
    tjm_destroy(j->model);
    delete j;
    return sfail(st, msg);
  }
  j->n_steps = (int)std::lround(j->T / j->dt);
  if (j->n_traj > kCap) {
    tjm_destroy(j->model);
    delete j;
    return sfail(TJM_E_UNSUPPORTED, "more trajectories than the server's work ring holds (1048576)");
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    // a job that could not run even alone next to the other precision's pool
    const int q = j->opt.precision == TJM_PREC_MIXED ? 1 : 0;
    if (j->bytes + pool_bytes_for(s, q, j->stride, j->L) > s->budget) {
      tjm_destroy(j->model);
      delete j;
      return sfail(TJM_E_NOMEM, "job needs more device memory than the server's budget");
    }
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
  s->wake.notify_all();
  return TJM_OK;
}

extern "C" tjm_status tjm_server_reserve(tjm_server* s, const tjm_model* m, const tjm_run_args* a) {
  if (!s || !m || !a) return sfail(TJM_E_INVAL, "NULL argument");
  if (a->n_obs < 0 || (a->n_obs > 0 && (!a->obs_site || !a->obs_op)))
    return sfail(TJM_E_INVAL, "bad observables");
  tjm_model* c = tjm_model_copy(m);
  if (!c) return sfail(TJM_E_NOMEM, "host allocation failed");
  tjm_options opt;
  tjm_default_options(&opt);
  if (a->opt) opt = *a->opt;
  opt.device = s->device;
  opt.workers = 0;
  long stride = 0;
  size_t bytes = 0;
  const tjm_status st = tjm_pool_plan(c, a->n_traj, a->dt, a->T, a->chi_max, a->n_obs, a->obs_site, a->obs_op,
                                      &opt, &stride, &bytes);
  const int L = tjm_model_L(c);
  std::string msg = st != TJM_OK ? tjm_last_error(c) : "";
  tjm_destroy(c);
  if (st != TJM_OK) return sfail(st, msg);
  const int q = opt.precision == TJM_PREC_MIXED ? 1 : 0;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (bytes + pool_bytes_for(s, q, std::max(stride, s->floor_stride[q]), std::max(L, s->floor_L[q])) > s->budget)
      return sfail(TJM_E_NOMEM, "the reserved shape needs more device memory than the server's budget");
    s->floor_stride[q] = std::max(stride, s->floor_stride[q]);
    s->floor_L[q] = std::max(L, s->floor_L[q]);
  }
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

extern "C" tjm_status tjm_job_progress(tjm_server* s, uint64_t job, int* traj_done, unsigned long long* steps_done) {
  if (!s || !traj_done || !steps_done) return sfail(TJM_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return sfail(TJM_E_INVAL, "unknown job");
  const Job* j = it->second;
  *traj_done = j->done ? j->n_traj : j->seen;
  if (j->done) *steps_done = j->status == TJM_OK ? (unsigned long long)j->n_traj * j->n_steps : 0ull;
  else if (j->pool) *steps_done = __atomic_load_n(&j->pool->steps[j->slot], __ATOMIC_RELAXED);
  else *steps_done = 0ull;
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
    rep->pool_bytes = j->pool_bytes;
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
    s->queue.clear();                  // never admitted: released with the server below
  }
  s->wake.notify_all();
  if (s->dispatcher.joinable()) s->dispatcher.join();   // admitted jobs finish first
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (int q = 0; q < 2; ++q)
    for (Pool* p : s->pools[q]) {
      pool_free(*p);
      delete p;
    }
  server_streams_destroy(s);
  (void)hipSetDevice(prev);
  for (auto& kv : s->jobs) {
    tjm_destroy(kv.second->model);
    delete kv.second;
  }
  delete s;
}
