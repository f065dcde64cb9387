// Serving loop: many independent time-step requests of differently sized
// scenes on one GPU.
//
// A request carries a full scene description, its state x(t), v(t) and step
// parameters.  Requests wait in a FIFO queue; a request is admitted when one
// of the server's slots is free and its estimated device footprint fits in
// what the memory budget has left.  Each slot owns a worker thread and its own
// HIP stream: it builds the request's mesh (host setup overlaps with other
// slots' GPU work), runs one Newton time step on its stream, copies the result
// back and frees the mesh.  Kernels of different slots run concurrently on the
// device.  Every request's kernels touch only its own buffers and use fixed
// reduction orders, so a result does not depend on what else is running.
//
// Device memory comes from the server's pool (no hipMalloc / hipFree per
// request), and block patterns stay resident in a topology cache: a request
// whose connectivity was seen before skips the pattern build and upload.
// Budget accounting: running requests are charged their estimate; idle cached
// patterns are charged their size and evicted when a request needs the room.
// The pool itself holds at most the budget in chunks (a request that does not
// fit because of fragmentation gets a chunk beyond it).
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "symx_internal.h"

namespace symxi {

symx_status mesh_create(const symx_mesh_desc* d, Mesh** out, DevicePool* pool,
                        TopologyCache* cache);
void mesh_free(Mesh* m);
symx_status newton_step(Mesh& m, double* x, double* v, const symx_step_params& P,
                        symx_step_report* out);

namespace {

using clk = std::chrono::steady_clock;

struct OwnedScene {
  std::vector<double> X;
  std::vector<uint8_t> fixed;
  std::vector<std::vector<int32_t>> conn;
  std::vector<std::vector<double>> young;
  std::vector<symx_energy_desc> energies;
  symx_mesh_desc desc{};
};

struct Request {
  int64_t ticket = 0;
  OwnedScene scene;
  std::vector<double> x, v;
  symx_step_params params{};
  size_t bytes = 0;
  clk::time_point t_submit, t_start, t_setup, t_step, t_end;
  bool done = false;
  symx_status status = SYMX_OK;
  symx_step_report report{};
};

}  // namespace

// Device bytes a mesh and its Newton workspace need (upper bound from sizes).
// project: include the incidence-ordered records of per-element projection.
size_t estimate_request_bytes(const symx_mesh_desc& d, int precision, bool project) {
  const size_t N = (size_t)d.n_nodes;
  size_t pairs = N, inc = 0, elems = 0, rot_elems = 0, conn = 0;
  for (int s = 0; s < d.n_energies; ++s) {
    const int k = kind_nodes(d.energies[s].kind);
    pairs += (size_t)d.energies[s].n_elem * k * (k - 1);
    inc += (size_t)d.energies[s].n_elem * k;
    elems += (size_t)d.energies[s].n_elem;
    conn += (size_t)d.energies[s].n_elem * 4 * (k < 4 ? 4 : k);
    if (k >= 10) conn += (size_t)d.energies[s].n_elem * k * k * 4;  // relabelled incidence nodes
    if (kind_has_rotation(d.energies[s].kind)) rot_elems += (size_t)d.energies[s].n_elem;
  }
  // the solve's values (half storage; refined solves keep float64 and float32)
  const size_t vbytes = precision == SYMX_F64 ? 8 : precision == SYMX_F32 ? 4 : 12;
  const size_t half = (pairs + N) / 2;
  size_t b = 0;
  b += half * 9 * vbytes + (pairs / 2 + N) * 4;  // half values, transposed positions, rows
  b += pairs * (4 + 4 + 2 * 3);                 // col_idx, contribution info/entries
  b += inc * 4 + conn + elems * (2 * 8 * kPrm + 4 * 4);  // incidence codes, conn, params
  b += rot_elems * 9 * (8 + 4);                // lagged rotations
  if (project) b += inc * (kIncRec * vbytes + 4);  // projected records, their positions
  b += N * (3 * 8 + 8 + 1 + 4 * 4);            // X, mass, fixed, row/inc pointers
  b += N * 3 * 8 * 9 + N * 9 * 8 * 2;          // Newton workspace, Dinv (and its float64 copy)
  b += N * 3 * 8 * 5;                          // PCG vectors (double worst case)
  b += (size_t)kMaxPartials * 8 + (1 << 16);   // reductions and slack
  return b;
}

struct Server {
  int device = 0;
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<int64_t, std::unique_ptr<Request>> requests;
  int64_t next_ticket = 1;
  size_t in_use = 0, peak = 0;
  int active = 0, peak_active = 0;
  int64_t completed = 0;
  bool stop = false;
  clk::time_point t0 = clk::now();
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::unique_ptr<DevicePool> pool;
  std::unique_ptr<TopologyCache> cache;
  std::atomic<int> solving{0};               // requests between setup and teardown
  std::unique_ptr<PcgBatcher> batcher;       // batched PCG of the solving requests

  void worker(int slot);
  bool fits(size_t bytes);  // with mu held
};

// Room for a request of `bytes` next to the running requests, evicting idle
// cached patterns if that makes it fit.
bool Server::fits(size_t bytes) {
  const size_t room = budget - in_use;  // in_use <= budget always
  if (bytes > room) return false;
  const size_t idle = cache->idle_bytes();
  if (bytes + idle <= room) return true;
  cache->evict_idle(bytes + idle - room);
  return bytes + cache->idle_bytes() <= room;
}

void Server::worker(int slot) {
  (void)hipSetDevice(device);
  hipStream_t stream = streams[slot];
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    cv_work.wait(lk, [&] { return stop || (!queue.empty() && fits(queue.front()->bytes)); });
    if (stop) return;
    Request* r = queue.front();
    queue.pop_front();
    in_use += r->bytes;
    peak = std::max(peak, in_use);
    ++active;
    peak_active = std::max(peak_active, active);
    r->t_start = clk::now();
    lk.unlock();

    symx_status st = SYMX_OK;
    Mesh* m = nullptr;
    double *dx = nullptr, *dv = nullptr;
    const size_t nb = r->x.size() * sizeof(double);
    r->scene.desc.hip_stream = stream;
    st = mesh_create(&r->scene.desc, &m, pool.get(), cache.get());
    if (st == SYMX_OK) {
      st = dev_alloc(pool.get(), (void**)&dx, nb);
      if (st == SYMX_OK) st = dev_alloc(pool.get(), (void**)&dv, nb);
    }
    if (st == SYMX_OK)
      st = hip_check(hipMemcpyAsync(dx, r->x.data(), nb, hipMemcpyHostToDevice, stream), "copy");
    if (st == SYMX_OK)
      st = hip_check(hipMemcpyAsync(dv, r->v.data(), nb, hipMemcpyHostToDevice, stream), "copy");
    if (st == SYMX_OK) st = hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    r->t_setup = clk::now();
    if (st == SYMX_OK) {
      m->batcher = batcher.get();
      ++solving;
      st = newton_step(*m, dx, dv, r->params, &r->report);
      --solving;
    }
    if (st == SYMX_OK) {
      symx_status s2 = hip_check(hipMemcpyAsync(r->x.data(), dx, nb, hipMemcpyDeviceToHost, stream), "copy");
      if (s2 == SYMX_OK)
        s2 = hip_check(hipMemcpyAsync(r->v.data(), dv, nb, hipMemcpyDeviceToHost, stream), "copy");
      if (s2 == SYMX_OK) s2 = hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
      st = s2;
    }
    (void)hipStreamSynchronize(stream);
    r->t_step = clk::now();
    dev_free(pool.get(), dx);
    dev_free(pool.get(), dv);
    if (m) mesh_free(m);

    lk.lock();
    r->status = st;
    r->report.status = st;
    r->t_end = clk::now();
    r->done = true;
    in_use -= r->bytes;
    --active;
    ++completed;
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

static double ms_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

symx_status server_create(uint64_t budget, int32_t max_slots, Server** out) {
  Server* s = new Server();
  s->budget = budget;
  s->max_slots = max_slots;
  symx_status st = hip_check(hipGetDevice(&s->device), "hipGetDevice");
  if (st != SYMX_OK) {
    delete s;
    return st;
  }
  s->pool = std::make_unique<DevicePool>(s->device, budget);
  s->cache = std::make_unique<TopologyCache>(256);
  s->batcher = std::make_unique<PcgBatcher>(s->device, max_slots,
                                            [s] { return s->solving.load(); });
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t h = nullptr;
    st = hip_check(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), "hipStreamCreate");
    if (st != SYMX_OK) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return st;
    }
    s->streams.push_back(h);
  }
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(&Server::worker, s, i);
  *out = s;
  return SYMX_OK;
}

void server_destroy(Server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // requests still queued are abandoned; running ones finish first
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers) t.join();
  s->batcher.reset();
  for (hipStream_t h : s->streams) (void)hipStreamDestroy(h);
  s->cache.reset();  // cached patterns go back to the pool first
  s->pool.reset();
  delete s;
}

symx_status server_submit(Server* s, const symx_mesh_desc* d, const double* x, const double* v,
                          const symx_step_params* P, int64_t* ticket) {
  if (!d || !x || !v || !P || !ticket || d->n_nodes < 1 || d->n_energies < 1 ||
      d->n_energies > kMaxSets || !d->energies || !d->x_rest) {
    set_error("invalid request");
    return SYMX_ERR_INVALID_ARG;
  }
  if (!step_params_valid(*P)) {
    set_error("invalid step parameters in request");
    return SYMX_ERR_INVALID_ARG;
  }
  auto r = std::make_unique<Request>();
  OwnedScene& sc = r->scene;
  const size_t N = (size_t)d->n_nodes;
  sc.X.assign(d->x_rest, d->x_rest + 3 * N);
  if (d->fixed) sc.fixed.assign(d->fixed, d->fixed + N);
  sc.energies.assign(d->energies, d->energies + d->n_energies);
  sc.conn.resize(d->n_energies);
  sc.young.resize(d->n_energies);
  for (int e = 0; e < d->n_energies; ++e) {
    const symx_energy_desc& ed = d->energies[e];
    const int k = kind_nodes(ed.kind);
    if (ed.n_elem < 0 || (ed.n_elem > 0 && !ed.conn)) {
      set_error("invalid energy set in request");
      return SYMX_ERR_INVALID_ARG;
    }
    sc.conn[e].assign(ed.conn, ed.conn + ed.n_elem * k);
    sc.energies[e].conn = sc.conn[e].data();
    if (ed.young) {
      sc.young[e].assign(ed.young, ed.young + ed.n_elem);
      sc.energies[e].young = sc.young[e].data();
    }
  }
  sc.desc = *d;
  sc.desc.x_rest = sc.X.data();
  sc.desc.fixed = d->fixed ? sc.fixed.data() : nullptr;
  sc.desc.energies = sc.energies.data();
  r->x.assign(x, x + 3 * N);
  r->v.assign(v, v + 3 * N);
  r->params = *P;
  r->bytes = estimate_request_bytes(*d, P->precision, P->project != 0);
  if (r->bytes > s->budget) {
    set_error("request footprint exceeds the server's memory budget");
    return SYMX_ERR_BUDGET;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->ticket = s->next_ticket++;
  r->t_submit = clk::now();
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->requests[r->ticket] = std::move(r);
  s->cv_work.notify_all();
  return SYMX_OK;
}

symx_status server_poll(Server* s, int64_t ticket, int32_t wait, double* x_out, double* v_out,
                        symx_step_report* rep, double* times_ms) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) {
    set_error("unknown ticket");
    return SYMX_ERR_INVALID_ARG;
  }
  Request* r = it->second.get();
  if (wait) s->cv_done.wait(lk, [&] { return r->done; });
  if (!r->done) return SYMX_PENDING;
  if (x_out) std::memcpy(x_out, r->x.data(), r->x.size() * sizeof(double));
  if (v_out) std::memcpy(v_out, r->v.data(), r->v.size() * sizeof(double));
  if (rep) *rep = r->report;
  if (times_ms) {
    times_ms[0] = ms_between(s->t0, r->t_submit);
    times_ms[1] = ms_between(s->t0, r->t_start);
    times_ms[2] = ms_between(s->t0, r->t_setup);
    times_ms[3] = ms_between(s->t0, r->t_step);
    times_ms[4] = ms_between(s->t0, r->t_end);
  }
  const symx_status st = r->status;
  s->requests.erase(it);
  return st;
}

void server_stats(Server* s, symx_server_stats* out) {
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  out->budget_bytes = s->budget;
  out->in_use_bytes = s->in_use;
  out->peak_bytes = s->peak;
  out->pattern_cache_bytes = s->cache->idle_bytes();
  out->pattern_hits = s->cache->hits;
  out->pattern_misses = s->cache->misses;
  out->queued = (int64_t)s->queue.size();
  out->active = s->active;
  out->peak_active = s->peak_active;
  out->completed = s->completed;
  out->max_slots = s->max_slots;
  out->peak_device_bytes = s->pool->peak_live_bytes();
  out->pcg_batches = s->batcher ? s->batcher->batches() : 0;
  out->pcg_chunks = s->batcher ? s->batcher->chunks() : 0;
}

}  // namespace symxi
