// Serving layer: many LocalPower jobs on one GPU (host code only).
//
// One worker thread owns all GPU work.  Jobs wait in a FIFO until their
// device footprint fits the budget and a slot is free (admission); an
// admitted job gets a slot (a stream for its allocations and a pinned change
// cell), a range of the server's device arena for its workspace and buffers,
// and an lp_problem with its own stream.  The worker keeps one round in
// flight per job: a round, the change sin theta(Z_r, Z_{r-1}) into pinned
// memory and an event; it polls the events, applies the per-job stop rule,
// halves p on a stall, and enqueues the next round.  Rounds of different jobs
// therefore overlap on the GPU, and a finished job's slot is refilled at once
// from the queue (continuous batching).
#include <algorithm>
#include <cstddef>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "arena.h"
#include "lp_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Job {
  uint64_t id = 0;
  lp_job spec;                 // copied at submit, zero-extended for shorter structs
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  size_t a_bytes = 0;          // generated A inside the footprint (0: the caller's A)
  std::vector<int64_t> offsets;
  std::vector<double> y0;
  size_t ws_bytes = 0, footprint = 0;
  Clock::time_point t_submit, t_admit;
  // set at admission
  int slot = -1;
  char* mem = nullptr;
  size_t arena_off = 0, arena_bytes = 0;   // the job's range of the server's arena
  lp_problem* P = nullptr;
  double* y0_dev = nullptr;
  double* zprev = nullptr;
  double* change_dev = nullptr;
  // schedule state
  int rounds = 0, iters = 0;
  lp::StopRule rule;
  bool in_flight = false;
};

}  // namespace

struct lp_server {
  int device = 0;
  size_t budget = 0, used = 0;
  int max_active = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::deque<lp_job_result> done;
  uint64_t next_id = 1;
  bool stopping = false;
  // owned by the worker thread
  std::vector<Job*> active;
  std::vector<hipStream_t> slot_stream;
  std::vector<hipEvent_t> slot_event;
  std::vector<int> free_slots;
  double* pinned = nullptr;   // one change cell per slot
  // the jobs' device memory: one arena of the budget, allocated with the server;
  // a job is admitted when a range of its footprint is free (per-job allocations
  // from a stream-ordered pool left the GPU idle for 0.1-1.4 s at some
  // admissions once the pool had grown over many job sizes)
  lp::Arena arena;
  std::thread worker;
};

namespace {

size_t elem(lp_dtype t) { return t == LP_F64 ? 8 : (t == LP_F32 ? 4 : 2); }

// The caller's job zero-extended to the current struct (fields past its
// struct_size read as zero: stream NULL, no generation).
bool widen(const lp_job* j, lp_job* out) {
  if (j == nullptr || j->struct_size < (int32_t)offsetof(lp_job, stream)) return false;
  std::memset(out, 0, sizeof(*out));
  std::memcpy(out, j, std::min<size_t>(sizeof(*out), (size_t)j->struct_size));
  out->struct_size = sizeof(*out);
  return true;
}

lp_status validate(const lp_job* j) {
  if (j->offsets == nullptr || j->Z_out == nullptr)
    return lp::report(LP_EINVAL, "offsets and Z_out are required");
  if (j->A == nullptr) {
    if (j->dtype != LP_F32 && j->dtype != LP_BF16) return lp::report(LP_EINVAL, "generated A is FP32 or BF16");
    if (!lp::truth_shape_ok(j->n, j->d))
      return lp::report(LP_EINVAL, "generated A needs d a power of two in [16, 8192] and n a multiple of d");
    if (!(j->gen_gap >= 1.0) || !(j->gen_decay > 0.0 && j->gen_decay <= 1.0))
      return lp::report(LP_EINVAL, "generated A needs gen_gap >= 1 and 0 < gen_decay <= 1");
  }
  if (j->n < 1 || j->d < 1 || (j->A != nullptr && j->lda < j->d) || j->m < 1)
    return lp::report(LP_EINVAL, "bad n, d, lda or m");
  if (j->k < 1 || j->k > 64 || j->k > j->d) return lp::report(LP_EINVAL, "need 1 <= k <= min(d, 64)");
  if (j->p0 < 1 || j->max_rounds < 1 || !(j->target > 0.0)) return lp::report(LP_EINVAL, "need p0 >= 1, max_rounds >= 1, target > 0");
  if (j->mode != LP_AGG_VANILLA && j->mode != LP_AGG_SIGN && j->mode != LP_AGG_OPT) return lp::report(LP_EINVAL, "unknown mode");
  if (j->offsets[0] != 0 || j->offsets[j->m] != j->n) return lp::report(LP_EINVAL, "offsets must run from 0 to n");
  for (int i = 0; i < j->m; ++i)
    if (j->offsets[i + 1] - j->offsets[i] < j->k) return lp::report(LP_EINVAL, "every partition needs at least k rows");
  return LP_OK;
}

// bytes of the per-job buffers after the workspace: Y0, previous Z, change cell
size_t extra_bytes(const lp_job* j) { return 2 * round_up((size_t)j->d * j->k * 8, 256) + 256; }
// bytes of a generated A (none when the caller passes A)
size_t gen_bytes(const lp_job* j) {
  return j->A == nullptr ? round_up((size_t)j->n * j->d * elem(j->dtype), 256) : 0;
}

void publish(lp_server* S, Job* j, lp_status st) {
  lp_job_result r;
  std::memset(&r, 0, sizeof(r));
  r.id = j->id;
  r.status = st;
  r.rounds = j->rounds;
  r.local_iters = j->iters;
  r.p_final = j->rule.p_run;
  r.change = j->rule.change;
  r.estimate = j->rule.estimate;
  const Clock::time_point now = Clock::now();
  r.ms_queued = ms_between(j->t_submit, j->t_admit);
  r.ms_total = ms_between(j->t_submit, now);
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->used -= j->footprint;
    S->done.push_back(r);
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

// release the job's GPU resources (its stream has been synchronised)
void release(lp_server* S, Job* j) {
  if (j->P != nullptr) (void)lp_destroy(j->P);
  j->P = nullptr;
  if (j->arena_bytes > 0) {
    // the job's range is reused by the next admission: nothing of this job may
    // still run on its slot stream (its problem stream was synchronised)
    if (j->slot >= 0) (void)hipStreamSynchronize(S->slot_stream[j->slot]);
    S->arena.give(j->arena_off, j->arena_bytes);
  }
  j->arena_bytes = 0;
  j->mem = nullptr;
  if (j->ready != nullptr) (void)hipEventDestroy(j->ready);
  j->ready = nullptr;
  if (j->slot >= 0) S->free_slots.push_back(j->slot);
  j->slot = -1;
}

// end the job: copy Z_out, check breakdown flags, free, publish
void finish(lp_server* S, Job* j, lp_status st) {
  if (j->P != nullptr) {
    hipStream_t s = lp::drive_stream(j->P);
    if (hipMemcpyAsync(j->spec.Z_out, lp::drive_z(j->P), (size_t)j->spec.d * j->spec.k * 8,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      st = LP_EDEVICE;
    int breakdowns = 0;
    if (lp::drive_breakdowns(j->P, &breakdowns) != LP_OK) st = LP_EDEVICE;
    else if (breakdowns > 0 && st == LP_OK) st = LP_EBREAKDOWN;
  }
  release(S, j);
  publish(S, j, st);
  delete j;
}

// one round, the change and its copy to the job's pinned cell, then the event
lp_status launch(lp_server* S, Job* j) {
  lp_problem* P = j->P;
  hipStream_t s = lp::drive_stream(P);
  const int64_t dk = j->spec.d * j->spec.k;
  lp_status st = lp::drive_round(P, j->spec.k, j->rule.p, j->spec.mode);
  if (st != LP_OK) return st;
  if (lp::drive_change(P, j->spec.k, j->zprev, j->change_dev) != hipSuccess ||
      hipMemcpyAsync(j->zprev, lp::drive_z(P), dk * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(S->pinned + j->slot, j->change_dev, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipEventRecord(S->slot_event[j->slot], s) != hipSuccess)
    return lp::report(LP_EDEVICE, "serving: enqueue failed");
  j->in_flight = true;
  return LP_OK;
}

// admission work for one job: memory, problem, Z_0 = orth(Y0), first round
lp_status start(lp_server* S, Job* j) {
  if (S->free_slots.empty()) return lp::report(LP_EDEVICE, "serving: no free slot");
  j->slot = S->free_slots.back();
  S->free_slots.pop_back();
  hipStream_t ss = S->slot_stream[j->slot];
  // everything the caller queued on its stream before the submit comes first
  if (hipStreamWaitEvent(ss, j->ready, 0) != hipSuccess)
    return lp::report(LP_EDEVICE, "serving: wait for the caller's stream failed");
  j->mem = S->arena.base + j->arena_off;
  lp_job& sp = j->spec;
  if (j->a_bytes > 0) {
    // the job's own matrix, generated at admission after the buffers it uses
    sp.A = j->mem + j->footprint - j->a_bytes;
    sp.lda = sp.d;
    if (lp::launch_truth_matrix((void*)sp.A, sp.dtype, sp.n, sp.d, sp.lda, sp.k, sp.gen_gap,
                                sp.gen_decay, sp.gen_seed, ss) != hipSuccess)
      return lp::report(LP_EDEVICE, "serving: generating A failed");
  }
  lp_status st = lp_create(&j->P, sp.A, sp.dtype, sp.n, sp.d, sp.lda, j->offsets.data(), sp.m,
                           sp.k, j->mem, j->ws_bytes, ss);
  if (st != LP_OK) {
    j->P = nullptr;
    return st;
  }
  if (sp.dtype == LP_BF16 && (st = lp::drive_split_operands(j->P, sp.single_bf16 == 0)) != LP_OK)
    return st;
  lp::drive_prefer_matrix_cores(j->P, sp.k);
  const size_t dk8 = round_up((size_t)sp.d * sp.k * 8, 256);
  j->y0_dev = (double*)(j->mem + j->ws_bytes);
  j->zprev = (double*)(j->mem + j->ws_bytes + dk8);
  j->change_dev = (double*)(j->mem + j->ws_bytes + 2 * dk8);
  hipStream_t s = lp::drive_stream(j->P);
  const hipError_t ey = j->y0.empty()
                            ? lp::launch_gaussian((int64_t)sp.d * sp.k, sp.gen_seed, j->y0_dev, s)
                            : hipMemcpyAsync(j->y0_dev, j->y0.data(), (size_t)sp.d * sp.k * 8,
                                             hipMemcpyHostToDevice, s);
  if (ey != hipSuccess) return lp::report(LP_EDEVICE, "serving: start copy failed");
  if ((st = lp::drive_begin(j->P, sp.k, j->y0_dev, false)) != LP_OK) return st;
  if (hipMemcpyAsync(j->zprev, lp::drive_z(j->P), (size_t)sp.d * sp.k * 8, hipMemcpyDeviceToDevice,
                     s) != hipSuccess)
    return lp::report(LP_EDEVICE, "serving: start copy failed");
  j->rule.p = sp.p0;
  j->rule.target = sp.target;
  return launch(S, j);
}

// a round of job j has completed: stop rule, stall rule, next round.  Returns
// false when the job has ended (it is then published and deleted).
bool advance(lp_server* S, Job* j) {
  j->in_flight = false;
  const int p = j->rule.p;
  j->rounds++;
  j->iters += p;
  // settled at p = 1: done (settled at p > 1 or a stall halves p inside step)
  if (j->rule.step(S->pinned[j->slot])) {
    finish(S, j, LP_OK);
    return false;
  }
  if (j->rounds >= j->spec.max_rounds) {
    finish(S, j, LP_ENOTCONV);
    return false;
  }
  lp_status st = launch(S, j);
  if (st != LP_OK) {
    finish(S, j, st);
    return false;
  }
  return true;
}

void worker_main(lp_server* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<Job*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stopping) {
        for (Job* j : S->queue) {
          S->used -= j->footprint;
          if (j->ready != nullptr) (void)hipEventDestroy(j->ready);
          delete j;
        }
        S->queue.clear();
        if (S->active.empty()) break;
      }
      // a job is admitted only with a slot reserved for it (slots are taken in
      // start()) and a range of the arena for its footprint (FIFO: the head waits
      // until one is free; with no job active the whole arena is, and every
      // footprint fits the budget)
      while (!S->queue.empty() && admitted.size() < S->free_slots.size()) {
        Job* j = S->queue.front();
        const size_t bytes = round_up(j->footprint, 256);
        if (!S->arena.take(bytes, &j->arena_off)) break;
        j->arena_bytes = bytes;
        S->queue.pop_front();
        S->used += j->footprint;
        admitted.push_back(j);
      }
      if (admitted.empty() && S->active.empty()) {
        S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        continue;
      }
    }
    for (Job* j : admitted) {
      j->t_admit = Clock::now();
      lp_status st = start(S, j);
      if (st != LP_OK) {
        if (j->P != nullptr) (void)hipStreamSynchronize(lp::drive_stream(j->P));
        release(S, j);
        publish(S, j, st);
        delete j;
        continue;
      }
      S->active.push_back(j);
    }
    bool progressed = !admitted.empty();
    for (size_t a = 0; a < S->active.size();) {
      Job* j = S->active[a];
      const hipError_t q = hipEventQuery(S->slot_event[j->slot]);
      if (q == hipErrorNotReady) {
        ++a;
        continue;
      }
      progressed = true;
      bool keep = false;
      if (q != hipSuccess)
        finish(S, j, lp::report(LP_EDEVICE, std::string("serving: ") + hipGetErrorString(q)));
      else
        keep = advance(S, j);
      if (keep)
        ++a;
      else
        S->active.erase(S->active.begin() + a);
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

lp_status lp_server_footprint(const lp_job* job_in, size_t* bytes) {
  if (bytes == nullptr) return lp::report(LP_EINVAL, "bytes is NULL");
  lp_job job;
  if (!widen(job_in, &job)) return lp::report(LP_EINVAL, "job is NULL or struct_size too small");
  lp_status st = validate(&job);
  if (st != LP_OK) return st;
  size_t ws = 0;
  if ((st = lp_workspace_size(job.dtype, job.n, job.d, job.offsets, job.m, job.k, &ws)) != LP_OK)
    return st;
  *bytes = round_up(ws, 256) + extra_bytes(&job) + gen_bytes(&job);
  return LP_OK;
}

lp_status lp_server_create(lp_server** out, size_t hbm_budget_bytes, int32_t max_active) {
  if (out == nullptr || max_active < 1 || max_active > 64 || hbm_budget_bytes == 0)
    return lp::report(LP_EINVAL, "need out != NULL, 1 <= max_active <= 64, budget > 0");
  lp_server* S = new lp_server();
  S->budget = hbm_budget_bytes;
  S->max_active = max_active;
  if (hipGetDevice(&S->device) != hipSuccess ||
      hipHostMalloc((void**)&S->pinned, sizeof(double) * max_active, hipHostMallocDefault) != hipSuccess) {
    delete S;
    return lp::report(LP_EDEVICE, "serving: device or pinned memory unavailable");
  }
  S->arena.size = round_up(hbm_budget_bytes, 256);
  if (hipMalloc((void**)&S->arena.base, S->arena.size) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(S->pinned);
    delete S;
    return lp::report(LP_ENOMEM, "serving: the budget does not fit in free device memory");
  }
  S->arena.free_ranges.emplace(0, S->arena.size);
  S->slot_stream.assign(max_active, nullptr);
  S->slot_event.assign(max_active, nullptr);
  for (int i = 0; i < max_active; ++i) {
    if (hipStreamCreateWithFlags(&S->slot_stream[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->slot_event[i], hipEventDisableTiming) != hipSuccess) {
      for (int t = 0; t <= i; ++t) {
        if (S->slot_stream[t]) (void)hipStreamDestroy(S->slot_stream[t]);
        if (S->slot_event[t]) (void)hipEventDestroy(S->slot_event[t]);
      }
      (void)hipFree(S->arena.base);
      (void)hipHostFree(S->pinned);
      delete S;
      return lp::report(LP_EDEVICE, "serving: stream creation failed");
    }
    S->free_slots.push_back(max_active - 1 - i);
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return LP_OK;
}

lp_status lp_server_submit(lp_server* S, const lp_job* job_in, uint64_t* job_id) {
  if (S == nullptr || job_id == nullptr) return lp::report(LP_EINVAL, "server or job_id is NULL");
  size_t fp = 0;
  lp_status st = lp_server_footprint(job_in, &fp);
  if (st != LP_OK) return st;
  if (fp > S->budget) return lp::report(LP_ENOMEM, "job footprint exceeds the server budget");
  lp_job job;
  widen(job_in, &job);
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ready, (hipStream_t)job.stream) != hipSuccess) {
    if (ready != nullptr) (void)hipEventDestroy(ready);
    return lp::report(LP_EDEVICE, "serving: event on the caller's stream failed");
  }
  Job* j = new Job();
  j->spec = job;
  j->ready = ready;
  j->offsets.assign(job.offsets, job.offsets + job.m + 1);
  j->spec.offsets = nullptr;
  if (job.Y0 != nullptr) j->y0.assign(job.Y0, job.Y0 + (size_t)job.d * job.k);
  j->spec.Y0 = nullptr;
  j->footprint = fp;
  j->a_bytes = gen_bytes(&job);
  j->ws_bytes = fp - extra_bytes(&job) - j->a_bytes;
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopping) {
      (void)hipEventDestroy(j->ready);
      delete j;
      return lp::report(LP_EBUSY, "server is stopping");
    }
    j->id = S->next_id++;
    *job_id = j->id;
    S->queue.push_back(j);
  }
  S->cv_work.notify_all();
  return LP_OK;
}

lp_status lp_server_poll(lp_server* S, lp_job_result* out, int32_t max, int32_t* n_done) {
  if (S == nullptr || n_done == nullptr || (max > 0 && out == nullptr)) return lp::report(LP_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  int n = 0;
  while (n < max && !S->done.empty()) {
    out[n++] = S->done.front();
    S->done.pop_front();
  }
  *n_done = n;
  return LP_OK;
}

lp_status lp_server_wait(lp_server* S, int32_t min_done, double timeout_s) {
  if (S == nullptr) return lp::report(LP_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  const bool ok = S->cv_done.wait_for(lk, std::chrono::duration<double>(std::max(timeout_s, 0.0)),
                                      [&] { return (int)S->done.size() >= min_done; });
  return ok ? LP_OK : lp::report(LP_EBUSY, "timed out waiting for results");
}

lp_status lp_server_destroy(lp_server* S) {
  if (S == nullptr) return LP_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (int i = 0; i < S->max_active; ++i) {
    (void)hipStreamSynchronize(S->slot_stream[i]);
    (void)hipStreamDestroy(S->slot_stream[i]);
    (void)hipEventDestroy(S->slot_event[i]);
  }
  // every slot stream has been synchronised above, and every problem stream when
  // its job ended
  (void)hipFree(S->arena.base);
  (void)hipHostFree(S->pinned);
  delete S;
  return LP_OK;
}

}  // extern "C"
