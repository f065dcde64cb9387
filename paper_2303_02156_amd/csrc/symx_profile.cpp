// Per-kernel timing with HIP events (enabled by symx_mesh_set_profiling).
#include <cstring>

#include "symx_internal.h"

namespace symxi {

int Profiler::id_of(const char* name) {
  for (size_t i = 0; i < names.size(); ++i)
    if (names[i] == name) return (int)i;
  names.push_back(name);
  dur.emplace_back();
  return (int)names.size() - 1;
}

hipEvent_t Profiler::take() {
  if (pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = pool.back();
  pool.pop_back();
  return e;
}

void Profiler::resolve() {
  for (Pending& p : pending) {
    float t = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess)
      dur[p.id].push_back(t);
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

// Create events ahead of time so that profiled launches do not create them.
void Profiler::reserve(size_t n) {
  while (pool.size() < n) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    pool.push_back(e);
  }
}

void Profiler::reset() {
  resolve();
  for (auto& d : dur) d.clear();
}

void Profiler::destroy() {
  resolve();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

ProfPair prof_begin(Mesh& m, const char* name) {
  ProfPair p;
  if (!m.prof.on) return p;
  p.a = m.prof.take();
  p.b = m.prof.take();
  if (!p.a || !p.b) {
    if (p.a) m.prof.pool.push_back(p.a);
    if (p.b) m.prof.pool.push_back(p.b);
    return ProfPair();
  }
  p.id = m.prof.id_of(name);
  return p;
}

void prof_end(Mesh& m, const ProfPair& p) {
  if (p.id < 0) return;
  m.prof.pending.push_back({p.id, p.a, p.b});
}

}  // namespace symxi
