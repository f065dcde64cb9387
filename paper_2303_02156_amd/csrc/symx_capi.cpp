// C-ABI of libsymx.so (declared in include/symx.h).  Thin wrappers: argument
// validation, error reporting and dispatch to the mesh, kernel and Newton
// code.  No C++ exception crosses the boundary.
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "symx_internal.h"

struct symx_mesh_s {
  symxi::Mesh* m;
};

namespace symxi {
struct Server;
symx_status server_create(uint64_t budget, int32_t max_slots, Server** out);
void server_destroy(Server* s);
symx_status server_submit(Server* s, const symx_mesh_desc* d, const double* x, const double* v,
                          const symx_step_params* P, int64_t* ticket);
symx_status server_poll(Server* s, int64_t ticket, int32_t wait, double* x_out, double* v_out,
                        symx_step_report* rep, double* times_ms);
void server_stats(Server* s, symx_server_stats* out);
size_t estimate_request_bytes(const symx_mesh_desc& d, int precision, bool project);
}  // namespace symxi

struct symx_server_s {
  symxi::Server* s;
};

namespace symxi {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

symx_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SYMX_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? SYMX_ERR_OUT_OF_MEMORY : SYMX_ERR_DEVICE;
}

symx_status mesh_create(const symx_mesh_desc* d, Mesh** out, DevicePool* pool = nullptr,
                        TopologyCache* cache = nullptr);
void build_scatter(Mesh& m);
void free_workspace(Mesh& m);
symx_status assemble(Mesh& m, const double* x, const double* xt, double dt, bool want_g,
                     bool want_H, int project, int precision, bool dirichlet, double* g_out,
                     void* dinv, float* dinv_lo);
symx_status energy(Mesh& m, const double* x, const double* xt, double dt, int precision, double* E);
symx_status assemble_noalloc(Mesh& m, const double* x, const double* xt, double dt, uint32_t flags,
                             int precision, double* energy_host, double* grad_dev,
                             void* values_dev);
symx_status newton_step(Mesh& m, double* x, double* v, const symx_step_params& P,
                        symx_step_report* out);

void mesh_free(Mesh* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  else (void)hipDeviceSynchronize();
  free_workspace(*m);
  contacts_free(*m);
  dev_free(m->pool, m->dyn.d_prm64);
  dev_free(m->pool, m->dyn.d_prm32);
  m->prof.destroy();
  void* dev[] = {m->X,       m->mass,    m->fixed,    m->vals32,   m->vals64, m->lvals32,
                 m->lvals64, m->inc_rows, m->inc_pos, m->partials, m->scalars};
  for (void* p : dev) dev_free(m->pool, p);
  for (SetHost& s : m->sets) {
    dev_free(m->pool, s.d_prm64);
    dev_free(m->pool, s.d_prm32);
    dev_free(m->pool, s.d_rot64);
    dev_free(m->pool, s.d_rot32);
  }
  pinned_free(m->pool, m->pinned);
  m->topo.reset();  // frees the pattern unless a cache or another mesh holds it
  delete m;
}

}  // namespace symxi

using namespace symxi;

#define GUARD_BEGIN try {
#define GUARD_END                                   \
  }                                                 \
  catch (const std::bad_alloc&) {                   \
    set_error("host allocation failed");            \
    return SYMX_ERR_OUT_OF_MEMORY;                  \
  }                                                 \
  catch (const std::exception& ex) {                \
    set_error(ex.what());                           \
    return SYMX_ERR_DEVICE;                         \
  }                                                 \
  catch (...) {                                     \
    set_error("unknown exception");                 \
    return SYMX_ERR_DEVICE;                         \
  }

static bool valid_mesh(symx_mesh h) {
  if (!h || !h->m) {
    set_error("null mesh handle");
    return false;
  }
  return true;
}

extern "C" {

void symx_step_params_default(symx_step_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->dt = 0.01;
  p->gravity[2] = -9.81;
  p->newton_rtol = 1e-6;
  p->max_newton = 100;
  p->max_pcg = 500;
  p->project = 0;
  p->precision = SYMX_F64;
  p->max_halvings = 8;
  p->regrow_after = 3;
  p->max_refine = 4;
  p->forcing_max = 0.5;
}

symx_status symx_mesh_create(const symx_mesh_desc* desc, symx_mesh* out) {
  GUARD_BEGIN
  if (!out) {
    set_error("null output handle");
    return SYMX_ERR_INVALID_ARG;
  }
  *out = nullptr;
  Mesh* m = nullptr;
  symx_status st = mesh_create(desc, &m);
  if (st != SYMX_OK) {
    mesh_free(m);
    return st;
  }
  symx_mesh h = new symx_mesh_s{m};
  *out = h;
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_destroy(symx_mesh mesh) {
  GUARD_BEGIN
  if (!mesh) return SYMX_OK;
  mesh_free(mesh->m);
  delete mesh;
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_get_info(symx_mesh mesh, symx_mesh_info* info) {
  GUARD_BEGIN
  if (!valid_mesh(mesh) || !info) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  std::memset(info, 0, sizeof *info);
  info->n_nodes = m.N;
  info->nnzb = m.nnzb;
  info->n_incidences = m.n_inc;
  info->n_batches = m.n_batch;
  info->n_energies = (int32_t)m.sets.size();
  for (size_t s = 0; s < m.sets.size(); ++s) info->n_elem[s] = m.sets[s].n_elem;
  info->max_row_blocks = m.max_row_blocks;
  info->total_mass = m.total_mass;
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_get_pattern(symx_mesh mesh, int32_t* row_ptr, int32_t* col_idx,
                                  int32_t* scatter_map) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  const Topology& t = *m.topo;
  if (row_ptr) std::memcpy(row_ptr, t.h_row_ptr.data(), t.h_row_ptr.size() * sizeof(int32_t));
  if (col_idx) std::memcpy(col_idx, t.h_col_idx.data(), t.h_col_idx.size() * sizeof(int32_t));
  if (scatter_map) {
    build_scatter(m);
    std::memcpy(scatter_map, m.h_scatter.data(), m.h_scatter.size() * sizeof(int32_t));
  }
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_get_masses(symx_mesh mesh, double* mass_host) {
  GUARD_BEGIN
  if (!valid_mesh(mesh) || !mass_host) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  std::memcpy(mass_host, m.h_mass.data(), m.h_mass.size() * sizeof(double));
  return SYMX_OK;
  GUARD_END
}

symx_status symx_eval_derivatives(symx_mesh mesh, int32_t energy_index, const double* x_dev,
                                  uint32_t flags, int32_t precision, void* elem_E,
                                  void* elem_grad, void* elem_hess) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  if (energy_index < 0 || energy_index >= (int)m.sets.size() || !x_dev ||
      (precision != SYMX_F64 && precision != SYMX_F32)) {
    set_error("invalid energy index, positions or precision");
    return SYMX_ERR_INVALID_ARG;
  }
  void* E = (flags & SYMX_EVAL_E) ? elem_E : nullptr;
  void* g = (flags & SYMX_EVAL_GRAD) ? elem_grad : nullptr;
  void* H = (flags & SYMX_EVAL_HESS) ? elem_hess : nullptr;
  const bool filter = (flags & SYMX_PROJECT_FILTER) != 0;
  const bool proj = filter || (flags & SYMX_PROJECT_PSD) != 0;
  if (proj && !H) {
    set_error("SYMX_PROJECT_PSD and SYMX_PROJECT_FILTER need SYMX_EVAL_HESS and a Hessian buffer");
    return SYMX_ERR_INVALID_ARG;
  }
  if (proj && m.sets[energy_index].k >= 10) {
    set_error("per-element PSD projection is not available for quadratic or cubic tets");
    return SYMX_ERR_INVALID_ARG;
  }
  if (filter && m.sets[energy_index].kind == SYMX_SNH_TET4) {
    symx_status st = launch_elem_filtered(m, energy_index, x_dev, precision, E, g, H);
    if (st != SYMX_OK) return st;
    return hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
  }
  symx_status st = launch_elem_eval(m, energy_index, x_dev, (int)flags, precision, E, g, H);
  if (st != SYMX_OK) return st;
  if (proj) {
    const SetHost& s = m.sets[energy_index];
    st = launch_project(m, precision, H, s.n_elem, 3 * s.k);
    if (st != SYMX_OK) return st;
  }
  return hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
  GUARD_END
}

symx_status symx_assemble_bsr(symx_mesh mesh, const double* x_dev, const double* x_tilde_dev,
                              double dt, uint32_t flags, int32_t precision, double* energy_host,
                              double* grad_dev, symx_bsr_view* H_out) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  if (!x_dev || (precision != SYMX_F64 && precision != SYMX_F32) ||
      (x_tilde_dev && !(dt > 0.0)) || ((flags & SYMX_EVAL_E) && !energy_host) ||
      ((flags & SYMX_EVAL_GRAD) && !grad_dev) || ((flags & SYMX_EVAL_HESS) && !H_out)) {
    set_error("invalid arguments to symx_assemble_bsr");
    return SYMX_ERR_INVALID_ARG;
  }
  const bool want_g = (flags & SYMX_EVAL_GRAD) != 0;
  const bool want_H = (flags & SYMX_EVAL_HESS) != 0;
  const int project = (flags & SYMX_PROJECT_FILTER) ? 2 : (flags & SYMX_PROJECT_PSD) ? 1 : 0;
  symx_status st = assemble(m, x_dev, x_tilde_dev, dt, want_g, want_H, project, precision,
                            (flags & SYMX_DIRICHLET) != 0, grad_dev, nullptr, nullptr);
  if (st != SYMX_OK) return st;
  if (flags & SYMX_EVAL_E) {
    st = energy(m, x_dev, x_tilde_dev, dt, precision, energy_host);
    if (st != SYMX_OK) return st;
  }
  if (want_H) {
    H_out->n_block_rows = m.N;
    H_out->nnzb = m.nnzb;
    H_out->row_ptr = m.row_ptr;
    H_out->col_idx = m.col_idx;
    H_out->values = precision == SYMX_F64 ? (const void*)m.vals64 : (const void*)m.vals32;
    H_out->precision = precision;
  }
  return hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
  GUARD_END
}

symx_status symx_assemble_bsr_noalloc(symx_mesh mesh, const double* x_dev,
                                      const double* x_tilde_dev, double dt, uint32_t flags,
                                      int32_t precision, double* energy_host, double* grad_dev,
                                      void* values_dev) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  if (!x_dev || (precision != SYMX_F64 && precision != SYMX_F32) ||
      (x_tilde_dev && !(dt > 0.0)) || ((flags & SYMX_EVAL_E) && !energy_host) ||
      ((flags & SYMX_EVAL_GRAD) && !grad_dev) || ((flags & SYMX_EVAL_HESS) && !values_dev)) {
    set_error("invalid arguments to symx_assemble_bsr_noalloc");
    return SYMX_ERR_INVALID_ARG;
  }
  return assemble_noalloc(*mesh->m, x_dev, x_tilde_dev, dt, flags, precision, energy_host,
                          grad_dev, values_dev);
  GUARD_END
}

symx_status symx_newton_step(symx_mesh mesh, double* x_dev, double* v_dev,
                             const symx_step_params* params, symx_step_report* report) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  if (!x_dev || !v_dev || !params || !step_params_valid(*params)) {
    set_error("invalid arguments to symx_newton_step");
    return SYMX_ERR_INVALID_ARG;
  }
  return newton_step(*mesh->m, x_dev, v_dev, *params, report);
  GUARD_END
}

symx_status symx_mesh_set_contacts(symx_mesh mesh, int64_t n, const int32_t* tuples_host,
                                   double k_c, double d_hat) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  return contacts_set(*mesh->m, n, tuples_host, k_c, d_hat);
  GUARD_END
}

symx_status symx_mesh_set_dynamic_elements(symx_mesh mesh, const symx_energy_desc* set) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  return dynamic_set(*mesh->m, set);
  GUARD_END
}

symx_status symx_mesh_set_contact_mode(symx_mesh mesh, int32_t mode) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  if (mode != SYMX_CONTACT_COMPACT && mode != SYMX_CONTACT_BRANCH) {
    set_error("invalid contact mode");
    return SYMX_ERR_INVALID_ARG;
  }
  mesh->m->contact_mode = mode;
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_get_contact_bsr(symx_mesh mesh, int32_t precision, symx_bsr_view* view) {
  GUARD_BEGIN
  if (!valid_mesh(mesh) || !view || (precision != SYMX_F64 && precision != SYMX_F32)) {
    set_error("invalid arguments to symx_mesh_get_contact_bsr");
    return SYMX_ERR_INVALID_ARG;
  }
  Mesh& m = *mesh->m;
  const Contacts* c = m.contacts;
  view->n_block_rows = m.N;
  view->nnzb = c ? c->nnzb : 0;
  view->row_ptr = c ? c->row_ptr : nullptr;
  view->col_idx = c ? c->col_idx : nullptr;
  view->values = c ? (precision == SYMX_F64 ? (const void*)c->vals64 : (const void*)c->vals32)
                   : nullptr;
  view->precision = precision;
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_update_rotations(symx_mesh mesh, const double* x_dev) {
  GUARD_BEGIN
  if (!valid_mesh(mesh) || !x_dev) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  symx_status st = launch_lagged_rotations(m, x_dev);
  if (st != SYMX_OK) return st;
  return hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
  GUARD_END
}

symx_status symx_mesh_set_profiling(symx_mesh mesh, int32_t enable) {
  GUARD_BEGIN
  if (!valid_mesh(mesh)) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  m.prof.reset();
  m.prof.on = enable != 0;
  if (m.prof.on) m.prof.reserve(1 << 15);  // events for 16k launches, created up front
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_get_kernel_time(symx_mesh mesh, const char* name, double min_ms,
                                      int64_t* launches, double* total_ms) {
  GUARD_BEGIN
  if (!valid_mesh(mesh) || !name || !launches || !total_ms) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  m.prof.resolve();
  *launches = 0;
  *total_ms = 0.0;
  for (size_t i = 0; i < m.prof.names.size(); ++i)
    if (m.prof.names[i] == name)
      for (float t : m.prof.dur[i])
        if (t >= min_ms) {
          *launches += 1;
          *total_ms += t;
        }
  return SYMX_OK;
  GUARD_END
}

symx_status symx_mesh_kernel_names(symx_mesh mesh, char* buf, int64_t buf_len) {
  GUARD_BEGIN
  if (!valid_mesh(mesh) || !buf || buf_len < 1) return SYMX_ERR_INVALID_ARG;
  Mesh& m = *mesh->m;
  std::string all;
  for (size_t i = 0; i < m.prof.names.size(); ++i) {
    if (i) all += ",";
    all += m.prof.names[i];
  }
  if ((int64_t)all.size() + 1 > buf_len) {
    set_error("buffer too small for kernel names");
    return SYMX_ERR_INVALID_ARG;
  }
  std::memcpy(buf, all.c_str(), all.size() + 1);
  return SYMX_OK;
  GUARD_END
}

symx_status symx_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, symx_server* out) {
  GUARD_BEGIN
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes == 0) {
    set_error("invalid server arguments");
    return SYMX_ERR_INVALID_ARG;
  }
  *out = nullptr;
  Server* s = nullptr;
  symx_status st = server_create(hbm_budget_bytes, max_slots, &s);
  if (st != SYMX_OK) return st;
  *out = new symx_server_s{s};
  return SYMX_OK;
  GUARD_END
}

symx_status symx_server_submit(symx_server server, const symx_mesh_desc* scene,
                               const double* x_host, const double* v_host,
                               const symx_step_params* params, int64_t* ticket) {
  GUARD_BEGIN
  if (!server || !server->s) {
    set_error("null server handle");
    return SYMX_ERR_INVALID_ARG;
  }
  return server_submit(server->s, scene, x_host, v_host, params, ticket);
  GUARD_END
}

symx_status symx_server_poll(symx_server server, int64_t ticket, int32_t wait, double* x_out,
                             double* v_out, symx_step_report* report, double* times_ms) {
  GUARD_BEGIN
  if (!server || !server->s) {
    set_error("null server handle");
    return SYMX_ERR_INVALID_ARG;
  }
  return server_poll(server->s, ticket, wait, x_out, v_out, report, times_ms);
  GUARD_END
}

symx_status symx_server_get_stats(symx_server server, symx_server_stats* stats) {
  GUARD_BEGIN
  if (!server || !server->s || !stats) {
    set_error("null server handle or stats");
    return SYMX_ERR_INVALID_ARG;
  }
  server_stats(server->s, stats);
  return SYMX_OK;
  GUARD_END
}

symx_status symx_server_estimate_bytes(const symx_mesh_desc* scene, int32_t precision,
                                       uint64_t* bytes) {
  GUARD_BEGIN
  if (!scene || !bytes || scene->n_energies < 1 || scene->n_energies > kMaxSets ||
      !scene->energies) {
    set_error("invalid scene descriptor");
    return SYMX_ERR_INVALID_ARG;
  }
  *bytes = estimate_request_bytes(*scene, precision, true);
  return SYMX_OK;
  GUARD_END
}

symx_status symx_server_destroy(symx_server server) {
  GUARD_BEGIN
  if (!server) return SYMX_OK;
  server_destroy(server->s);
  delete server;
  return SYMX_OK;
  GUARD_END
}

const char* symx_status_string(symx_status s) {
  switch (s) {
    case SYMX_OK: return "ok";
    case SYMX_ERR_INVALID_ARG: return "invalid argument";
    case SYMX_ERR_OUT_OF_MEMORY: return "out of memory";
    case SYMX_ERR_DEVICE: return "device error";
    case SYMX_ERR_NONFINITE: return "non-finite value";
    case SYMX_ERR_NOT_CONVERGED: return "not converged";
    case SYMX_ERR_LINE_SEARCH: return "line search failed";
    case SYMX_ERR_BUDGET: return "memory budget exceeded";
    case SYMX_PENDING: return "pending";
  }
  return "unknown status";
}

const char* symx_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
