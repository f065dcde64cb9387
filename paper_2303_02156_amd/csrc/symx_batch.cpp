// Batched PCG for the serving loop.
//
// Every admitted request runs its own Newton loop (assembly, line search and
// the small kernels on its own stream), but the PCG chunks of all requests
// that are solving at the same time go through one PcgBatcher: it gathers the
// waiting chunks, and one SpMV and one update launch per iteration (and per
// precision/contact group) cover all of their meshes, each mesh with its own
// grid and arrays (launch_pcg_batch).  A mesh therefore computes exactly what
// it computes alone; only the number of launches and host synchronisations
// changes.  Kernel boundaries are the only synchronisation between the
// iterations, as in the one-mesh path.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "symx_internal.h"

namespace symxi {

struct PcgBatcher::Job {
  PcgBatchItem item;
  hipEvent_t ready = nullptr;  // recorded on the mesh's stream before the chunk
  double S[2] = {0.0, 0.0};
  int ran = 0;  // iterations the batch ran
  symx_status status = SYMX_OK;
  bool done = false;
};

PcgBatcher::PcgBatcher(int device, int max_meshes, std::function<int()> active)
    : device_(device), active_(std::move(active)) {
  init_status_ = hip_check(hipSetDevice(device), "hipSetDevice");
  if (init_status_ == SYMX_OK)
    init_status_ = hip_check(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking),
                             "hipStreamCreate");
  if (init_status_ == SYMX_OK) init_status_ = pcg_batch_tables_alloc(tables_, max_meshes);
  if (init_status_ == SYMX_OK) {
    void* p = nullptr;
    init_status_ = hip_check(hipHostMalloc(&p, 2 * sizeof(double) * max_meshes), "hipHostMalloc");
    s_host_ = static_cast<double*>(p);
  }
  cap_ = max_meshes;
  if (init_status_ == SYMX_OK) thread_ = std::thread(&PcgBatcher::loop, this);
}

PcgBatcher::~PcgBatcher() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (thread_.joinable()) thread_.join();
  pcg_batch_tables_free(tables_);
  if (s_host_) (void)hipHostFree(s_host_);
  if (stream_) (void)hipStreamDestroy(stream_);
}

symx_status PcgBatcher::run(Mesh& m, int precision, const PcgBuffers& B, int k0, int n,
                            double S_out[2], int* ran) {
  if (init_status_ != SYMX_OK) return init_status_;
  Job job;
  job.item = PcgBatchItem{&m, precision, B, k0, n};
  symx_status st = hip_check(hipEventCreateWithFlags(&job.ready, hipEventDisableTiming),
                             "hipEventCreate");
  if (st != SYMX_OK) return st;
  st = hip_check(hipEventRecord(job.ready, m.stream), "hipEventRecord");
  if (st == SYMX_OK) {
    std::unique_lock<std::mutex> lk(mu_);
    pending_.push_back(&job);
    cv_.notify_all();
    done_cv_.wait(lk, [&] { return job.done; });
    st = job.status;
  }
  (void)hipEventDestroy(job.ready);
  if (st == SYMX_OK) {
    S_out[0] = job.S[0];
    S_out[1] = job.S[1];
    *ran = job.ran;
  }
  return st;
}

void PcgBatcher::loop() {
  (void)hipSetDevice(device_);
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    cv_.wait(lk, [&] { return stop_ || !pending_.empty(); });
    if (stop_ && pending_.empty()) return;
    // gather: wait until every active request has a chunk waiting, or for a
    // short window after the first one arrived (requests in other phases
    // join the next batch)
    const auto t_first = std::chrono::steady_clock::now();
    while (!stop_ && (int)pending_.size() < std::min(cap_, std::max(1, active_())) &&
           std::chrono::steady_clock::now() - t_first < std::chrono::microseconds(kGatherUs))
      cv_.wait_for(lk, std::chrono::microseconds(20));
    std::vector<Job*> jobs;
    while (!pending_.empty() && (int)jobs.size() < cap_) {
      jobs.push_back(pending_.front());
      pending_.pop_front();
    }
    lk.unlock();
    // the batch runs the smallest chunk asked for: no request waits on
    // iterations of a larger one (those ask again)
    int n_run = jobs[0]->item.n;
    for (Job* j : jobs) n_run = std::min(n_run, j->item.n);
    symx_status st = SYMX_OK;
    std::vector<PcgBatchItem> items;
    for (Job* j : jobs) {
      items.push_back(j->item);
      items.back().n = n_run;
      if (st == SYMX_OK) st = hip_check(hipStreamWaitEvent(stream_, j->ready, 0), "hipStreamWaitEvent");
    }
    if (st == SYMX_OK) st = launch_pcg_batch(stream_, tables_, items.data(), (int)items.size());
    for (size_t i = 0; i < jobs.size() && st == SYMX_OK; ++i)
      st = hip_check(hipMemcpyAsync(s_host_ + 2 * i, jobs[i]->item.m->scalars, 2 * sizeof(double),
                                    hipMemcpyDeviceToHost, stream_),
                     "hipMemcpyAsync");
    if (st == SYMX_OK) st = hip_check(hipStreamSynchronize(stream_), "hipStreamSynchronize");
    lk.lock();
    ++batches_;
    chunks_ += (int64_t)jobs.size();
    for (size_t i = 0; i < jobs.size(); ++i) {
      jobs[i]->status = st;
      jobs[i]->S[0] = s_host_[2 * i];
      jobs[i]->S[1] = s_host_[2 * i + 1];
      jobs[i]->ran = n_run;
      jobs[i]->done = true;
    }
    done_cv_.notify_all();
  }
}

int64_t PcgBatcher::batches() {
  std::lock_guard<std::mutex> lk(mu_);
  return batches_;
}

int64_t PcgBatcher::chunks() {
  std::lock_guard<std::mutex> lk(mu_);
  return chunks_;
}

}  // namespace symxi
