// Device memory for the serving loop: a caching allocator and a cache of
// device-resident mesh topologies.
//
// A request of the serving loop builds a mesh, runs one time step and frees
// the mesh.  Without a pool every request would call hipMalloc / hipFree some
// forty times, and hipFree may wait for kernels of other requests.  The pool
// keeps freed blocks for reuse instead.  Requests whose scenes have the same
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

// Size classes: 4 KiB granules up to 64 KiB, then 1/8 of the next power of
// two (at most 12.5% slack), so repeated requests of one scene size reuse
// exactly the blocks they freed.
size_t DevicePool::round_size(size_t bytes) {
  if (bytes <= (size_t(64) << 10)) return std::max<size_t>(4096, (bytes + 4095) & ~size_t(4095));
  size_t p2 = 1;
  while (p2 < bytes) p2 <<= 1;
  const size_t g = p2 >> 3;
  return (bytes + g - 1) / g * g;
}

void* DevicePool::alloc(size_t bytes) {
  const size_t cls = round_size(bytes ? bytes : 1);
  {
    std::lock_guard<std::mutex> lk(mu_);
    // smallest cached block of at least cls bytes, if not much larger
    auto it = free_.lower_bound(cls);
    if (it != free_.end() && it->first <= cls + cls / 2) {
      void* p = it->second;
      live_[p] = it->first;
      cached_ -= it->first;
      free_.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) != hipSuccess) {
    (void)hipGetLastError();
    trim();
    if (hipMalloc(&p, cls) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(mu_);
  live_[p] = cls;
  return p;
}

void DevicePool::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = live_.find(p);
  if (it == live_.end()) return;  // not ours: leave it alone
  free_.emplace(it->second, p);
  cached_ += it->second;
  live_.erase(it);
}

void* DevicePool::alloc_pinned(size_t bytes) {
  const size_t cls = round_size(bytes ? bytes : 1);
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

void DevicePool::trim() {
  std::multimap<size_t, void*> blocks;
  {
    std::lock_guard<std::mutex> lk(mu_);
    blocks.swap(free_);
    cached_ = 0;
  }
  for (auto& b : blocks) (void)hipFree(b.second);
}

size_t DevicePool::cached_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return cached_;
}

DevicePool::~DevicePool() {
  // Called once no mesh of the pool is alive: every block is idle.
  for (auto& b : free_) (void)hipFree(b.second);
  for (auto& b : live_) (void)hipFree(b.first);
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
  void* dev[] = {row_ptr, col_idx, diag_pos, inc_ptr, inc_code, inc_slots,
                 batch_row, blk_info, centry, batch_entry};
  for (void* p : dev) dev_free(pool, p);
  for (TopoSet& s : sets) dev_free(pool, s.d_conn);
}

static int kind_nodes(int kind) { return kind == SYMX_STVK_TRI3 ? 3 : 4; }

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
