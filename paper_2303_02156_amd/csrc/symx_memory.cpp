// Device memory for the serving loop: a caching allocator and a cache of
// device-resident mesh topologies.
//
// A request of the serving loop builds a mesh, runs one time step and frees
// the mesh.  Without a pool every request would call hipMalloc / hipFree some
// forty times, and hipFree may wait for kernels of other requests.  The pool
// carves blocks out of a few large chunks instead (best fit, coalescing).  Requests whose scenes have the same
// connectivity (same node count, energy kinds and element lists) also share
// one Topology: the block pattern, incidence lists and contribution lists stay
// on the device, and only the per-request rest data (positions, materials,
// masses) is rebuilt.
#include <algorithm>
#include <cstring>

#include "symx_internal.h"

namespace symxi {

// ---------------------------------------------------------------------------
// DevicePool
// ---------------------------------------------------------------------------

namespace {
constexpr size_t kAlign = 256;
constexpr size_t kChunk = size_t(256) << 20;  // 256 MiB
size_t align_up(size_t n, size_t a) { return (n + a - 1) / a * a; }
}  // namespace

void DevicePool::add_free(Chunk* c, size_t off, size_t len) {
  c->free_at[off] = len;
  free_by_len_.emplace(len, FreeKey(c, off));
}

void DevicePool::remove_free(Chunk* c, size_t off, size_t len) {
  c->free_at.erase(off);
  auto r = free_by_len_.equal_range(len);
  for (auto it = r.first; it != r.second; ++it)
    if (it->second.first == c && it->second.second == off) {
      free_by_len_.erase(it);
      return;
    }
}

bool DevicePool::add_chunk(size_t min_bytes) {
  size_t size = std::max(kChunk, align_up(min_bytes, size_t(2) << 20));
  if (capacity_ && held_ + size > capacity_ && held_ + min_bytes <= capacity_)
    size = align_up(capacity_ - held_, kAlign);  // last chunk: what the capacity leaves
  // Allocate on the pool's device whatever device the calling thread has
  // current, and leave the caller's current device as it was.
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (prev != device_ && hipSetDevice(device_) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  void* p = nullptr;
  const bool ok = hipMalloc(&p, size) == hipSuccess;
  if (!ok) (void)hipGetLastError();
  if (prev != device_) (void)hipSetDevice(prev);
  if (!ok) return false;
  auto c = std::make_unique<Chunk>();
  c->base = static_cast<char*>(p);
  c->size = size;
  add_free(c.get(), 0, size);
  held_ += size;
  chunks_.push_back(std::move(c));
  return true;
}

void* DevicePool::alloc(size_t bytes) {
  const size_t n = align_up(bytes ? bytes : 1, kAlign);
  std::lock_guard<std::mutex> lk(mu_);
  auto it = free_by_len_.lower_bound(n);  // best fit
  if (it == free_by_len_.end()) {
    if (!add_chunk(n)) return nullptr;
    it = free_by_len_.lower_bound(n);
    if (it == free_by_len_.end()) return nullptr;
  }
  Chunk* c = it->second.first;
  const size_t off = it->second.second, len = it->first;
  remove_free(c, off, len);
  if (len > n) add_free(c, off + n, len - n);
  void* p = c->base + off;
  live_[p] = {c, n};
  live_bytes_ += n;
  peak_live_ = std::max(peak_live_, live_bytes_);
  return p;
}

void DevicePool::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = live_.find(p);
  if (it == live_.end()) return;  // not ours: leave it alone
  Chunk* c = it->second.first;
  size_t off = size_t(static_cast<char*>(p) - c->base), len = it->second.second;
  live_bytes_ -= len;
  live_.erase(it);
  // coalesce with the free neighbours
  auto next = c->free_at.find(off + len);
  if (next != c->free_at.end()) {
    const size_t nl = next->second;
    remove_free(c, off + len, nl);
    len += nl;
  }
  auto prev = c->free_at.lower_bound(off);
  if (prev != c->free_at.begin()) {
    --prev;
    if (prev->first + prev->second == off) {
      const size_t po = prev->first, pl = prev->second;
      remove_free(c, po, pl);
      off = po;
      len += pl;
    }
  }
  add_free(c, off, len);
}

void* DevicePool::alloc_pinned(size_t bytes) {
  const size_t cls = align_up(bytes ? bytes : 1, 4096);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = pinned_free_.find(cls);
    if (it != pinned_free_.end()) {
      void* p = it->second;
      pinned_live_[p] = cls;
      pinned_free_.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu_);
  pinned_live_[p] = cls;
  return p;
}

void DevicePool::release_pinned(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = pinned_live_.find(p);
  if (it == pinned_live_.end()) return;
  pinned_free_.emplace(it->second, p);
  pinned_live_.erase(it);
}

size_t DevicePool::chunk_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return held_;
}

size_t DevicePool::live_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return live_bytes_;
}

size_t DevicePool::peak_live_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return peak_live_;
}

DevicePool::~DevicePool() {
  // Called once no mesh of the pool is alive.
  for (auto& c : chunks_) (void)hipFree(c->base);
  for (auto& b : pinned_free_) (void)hipHostFree(b.second);
  for (auto& b : pinned_live_) (void)hipHostFree(b.first);
}

symx_status dev_alloc(DevicePool* pool, void** p, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (pool) {
    *p = pool->alloc(bytes);
  } else if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
  }
  if (!*p) {
    set_error("device allocation failed");
    return SYMX_ERR_OUT_OF_MEMORY;
  }
  return SYMX_OK;
}

void dev_free(DevicePool* pool, void* p) {
  if (!p) return;
  if (pool)
    pool->release(p);
  else
    (void)hipFree(p);
}

symx_status pinned_alloc(DevicePool* pool, void** p, size_t bytes) {
  if (pool) {
    *p = pool->alloc_pinned(bytes);
  } else if (hipHostMalloc(p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
  }
  if (!*p) {
    set_error("pinned host allocation failed");
    return SYMX_ERR_OUT_OF_MEMORY;
  }
  return SYMX_OK;
}

void pinned_free(DevicePool* pool, void* p) {
  if (!p) return;
  if (pool)
    pool->release_pinned(p);
  else
    (void)hipHostFree(p);
}

// ---------------------------------------------------------------------------
// Topology
// ---------------------------------------------------------------------------

Topology::~Topology() {
  void* dev[] = {row_ptr,  col_idx,   diag_pos, lrow_ptr, cv,         inc_ptr,
                 inc_code, inc_nodes, batch_row, blk_info, centry, batch_entry};
  for (void* p : dev) dev_free(pool, p);
  for (TopoSet& s : sets) {
    dev_free(pool, s.d_conn);
    dev_free(pool, s.d_conn_ho);
  }
}

bool Topology::matches(const symx_mesh_desc& d) const {
  if (d.n_nodes != N || d.n_energies != (int)sets.size()) return false;
  for (int s = 0; s < d.n_energies; ++s) {
    const symx_energy_desc& e = d.energies[s];
    if (e.kind != sets[s].kind || e.n_elem != sets[s].n_elem) return false;
    const size_t n = size_t(e.n_elem) * kind_nodes(e.kind);
    if (n && std::memcmp(e.conn, sets[s].conn.data(), n * sizeof(int32_t)) != 0) return false;
  }
  return true;
}

// The hash only selects candidates; matches() compares the full connectivity.
// It mixes the sizes and kinds and at most 4096 connectivity words per set,
// evenly spaced, so a lookup costs O(1) before the final compare.
uint64_t topology_hash(const symx_mesh_desc& d) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t w) {
    h ^= w;
    h *= 1099511628211ull;
    h ^= h >> 29;
  };
  mix(uint64_t(d.n_nodes));
  mix(uint64_t(d.n_energies));
  for (int s = 0; s < d.n_energies; ++s) {
    const symx_energy_desc& e = d.energies[s];
    mix(uint64_t(uint32_t(e.kind)));
    mix(uint64_t(e.n_elem));
    if (e.n_elem <= 0 || !e.conn) continue;
    const size_t n = size_t(e.n_elem) * kind_nodes(e.kind);
    const size_t step = std::max<size_t>(1, n / 4096);
    for (size_t i = 0; i < n; i += step) mix(uint64_t(uint32_t(e.conn[i])) | (uint64_t(i) << 32));
    mix(uint64_t(uint32_t(e.conn[n - 1])));
  }
  return h;
}

// ---------------------------------------------------------------------------
// TopologyCache
// ---------------------------------------------------------------------------

std::shared_ptr<Topology> TopologyCache::find(const symx_mesh_desc& d, uint64_t hash) {
  std::lock_guard<std::mutex> lk(mu_);
  for (auto it = lru_.begin(); it != lru_.end(); ++it) {
    if ((*it)->hash == hash && (*it)->matches(d)) {
      std::shared_ptr<Topology> t = *it;
      lru_.erase(it);
      lru_.push_front(t);
      ++hits;
      return t;
    }
  }
  ++misses;
  return nullptr;
}

void TopologyCache::insert(const std::shared_ptr<Topology>& t) {
  std::lock_guard<std::mutex> lk(mu_);
  lru_.push_front(t);
  // bound the number of entries: drop idle ones from the back
  for (auto it = lru_.end(); lru_.size() > max_entries_ && it != lru_.begin();) {
    --it;
    if (it->use_count() == 1) it = lru_.erase(it);
  }
}

size_t TopologyCache::idle_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  size_t b = 0;
  for (auto& t : lru_)
    if (t.use_count() == 1) b += t->device_bytes;
  return b;
}

size_t TopologyCache::evict_idle(size_t need) {
  std::lock_guard<std::mutex> lk(mu_);
  size_t freed = 0;
  for (auto it = lru_.end(); freed < need && it != lru_.begin();) {
    --it;
    if (it->use_count() == 1) {
      freed += (*it)->device_bytes;
      it = lru_.erase(it);
    }
  }
  return freed;
}

}  // namespace symxi
