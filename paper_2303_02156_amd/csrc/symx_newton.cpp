// Assembly entry points and the Newton driver on the mesh's stream.
//
// Newton step (Eq. 2-3, Sec. 7): minimise the incremental potential from
// x(t); per iteration assemble the gradient and Hessian, stop when
// |g_free| <= rtol |g_free(x(t))|, solve H dx = -g with block-Jacobi PCG to the
// forcing tolerance min(forcing_max, sqrt(r_k / r_0)) (forcing_max 0.5 by
// default), backtrack along dx with the
// Armijo test E(x + a dx) <= E(x) + 1e-4 a g.dx + 1e-12 |E(x)| (a halves, at
// most 30 times; the last term is the rounding of the float64 energy sum, so
// that a step whose decrease the energy can no longer resolve, close to the
// minimiser, is taken whole), and restart the whole step with dt/2 when the
// line search fails or Newton exceeds its iteration limit (the paper's
// benchmark protocol, Sec. 7).
//
// Precision modes: SYMX_F64 runs everything in float64.  SYMX_F32_REFINED
// evaluates energies, gradient and Hessian in float64 and keeps a float32
// copy of the Hessian (each value rounded) for the SpMV and PCG, which run in
// float32; the solution update stays float64, and each linear solve is
// refined in float64: the residual b - H dx is formed with the float64
// Hessian, and while it exceeds the forcing tolerance a float32 PCG solve of
// H c = r gives the correction dx += c (mixed-precision iterative
// refinement).  SYMX_F32 evaluates all element quantities in float32 (sums in
// float64).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "symx_internal.h"

namespace symxi {


enum { S_DONE = 0, S_ITERS };  // PCG flags (see the PCG kernels)
// device scalar slots used by the driver (after the PCG scalars)
enum { D_ENERGY = 16, D_DOT = 17, D_GG = 18, D_GD = 19, D_E0 = 20, D_ET = 21, D_FLAG = 24 };
// the device non-finite flag is the int stored at scalars[D_FLAG], so one copy
// of scalars[D_ENERGY .. D_FLAG] returns results and the flag together

#define TRY(expr)                 \
  do {                            \
    symx_status s_ = (expr);      \
    if (s_ != SYMX_OK) return s_; \
  } while (0)

struct Workspace {
  int64_t N = 0;
  double *x_t = nullptr, *v_t = nullptr, *xt = nullptr, *xk = nullptr, *xtrial = nullptr;
  double *g = nullptr, *dx = nullptr, *b = nullptr, *res = nullptr;
  void* pcg[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // Dinv xs r z p q (max size)
  double* dinv64 = nullptr;  // F32_REFINED: float64 block inverses before rounding (kDinv N)
};

bool step_params_valid(const symx_step_params& P) {
  return P.dt > 0.0 && P.max_newton >= 0 && P.max_pcg >= 1 && P.precision >= SYMX_F64 &&
         P.precision <= SYMX_F32_REFINED && P.max_halvings >= 0 && P.newton_rtol >= 0.0 &&
         P.project >= 0 && P.project <= 2 && P.max_refine >= 0 && P.forcing_max > 0.0 &&
         P.forcing_max < 1.0;
}


// Value arrays of the Hessian in `precision`: the block arrays of the public
// assembly, or (half) the half storage of the Newton solve.
static symx_status ensure_values(Mesh& m, int precision, bool half) {
  if (half) {
    if (precision == SYMX_F64 && !m.lvals64)
      return dev_alloc(m.pool, (void**)&m.lvals64, 9 * m.nnzl * sizeof(double));
    if (precision != SYMX_F64 && !m.lvals32)
      return dev_alloc(m.pool, (void**)&m.lvals32, 9 * m.nnzl * sizeof(float));
    return SYMX_OK;
  }
  if (precision == SYMX_F64 && !m.vals64) return dev_alloc(m.pool, (void**)&m.vals64, 9 * m.nnzb * sizeof(double));
  if (precision != SYMX_F64 && !m.vals32) return dev_alloc(m.pool, (void**)&m.vals32, 9 * m.nnzb * sizeof(float));
  return SYMX_OK;
}

static symx_status ensure_workspace(Mesh& m) {
  if (m.ws) return SYMX_OK;
  Workspace* w = new Workspace();
  m.ws = w;
  w->N = m.N;
  const size_t v64 = 3 * m.N * sizeof(double);
  double** vecs[] = {&w->x_t, &w->v_t, &w->xt, &w->xk, &w->xtrial, &w->g, &w->dx, &w->b, &w->res};
  for (double** p : vecs) TRY(dev_alloc(m.pool, (void**)p, v64));
  TRY(dev_alloc(m.pool, &w->pcg[0], kDinv * m.N * sizeof(double)));
  for (int i = 1; i < 6; ++i) TRY(dev_alloc(m.pool, &w->pcg[i], v64));
  return SYMX_OK;
}

static symx_status ensure_dinv64(Mesh& m) {
  Workspace* w = m.ws;
  if (w->dinv64) return SYMX_OK;
  return dev_alloc(m.pool, (void**)&w->dinv64, kDinv * m.N * sizeof(double));
}

void free_workspace(Mesh& m) {
  if (!m.ws) return;
  Workspace* w = m.ws;
  double* vecs[] = {w->x_t, w->v_t, w->xt, w->xk, w->xtrial, w->g, w->dx, w->b, w->res};
  for (double* p : vecs) dev_free(m.pool, p);
  for (void* p : w->pcg) dev_free(m.pool, p);
  dev_free(m.pool, w->dinv64);
  delete w;
  m.ws = nullptr;
}

static symx_status sync_read(Mesh& m, const double* dev, int n, double* host) {
  TRY(hip_check(hipMemcpyAsync(m.pinned, dev, n * sizeof(double), hipMemcpyDeviceToHost, m.stream),
                "hipMemcpyAsync"));
  TRY(hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize"));
  std::memcpy(host, m.pinned, n * sizeof(double));
  return SYMX_OK;
}

static symx_status check_nonfinite(Mesh& m) {
  int flag = 0;
  TRY(hip_check(hipMemcpyAsync(m.pinned, m.nonfinite, sizeof(int), hipMemcpyDeviceToHost, m.stream),
                "hipMemcpyAsync"));
  TRY(hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize"));
  std::memcpy(&flag, m.pinned, sizeof(int));
  if (flag) {
    TRY(hip_check(hipMemsetAsync(m.nonfinite, 0, sizeof(int), m.stream), "hipMemsetAsync"));
    set_error("non-finite value in positions, energy or gradient");
    return SYMX_ERR_NONFINITE;
  }
  return SYMX_OK;
}

// Copy scalars[D_ENERGY .. D_FLAG] to the host; returns true in *bad (and
// clears the device flag) if a kernel met a non-finite value since the last read.
static symx_status read_window(Mesh& m, double* win, bool* bad) {
  const int n = D_FLAG - D_ENERGY + 1;
  TRY(sync_read(m, m.scalars + D_ENERGY, n, win));
  int flag = 0;
  std::memcpy(&flag, &win[D_FLAG - D_ENERGY], sizeof(int));
  *bad = flag != 0;
  if (*bad) TRY(hip_check(hipMemsetAsync(m.nonfinite, 0, sizeof(int), m.stream), "hipMemsetAsync"));
  return SYMX_OK;
}

// Projected path: incidence positions and records (allocated on first use),
// then the fused evaluation + projection of every element into the records.
static symx_status project_into_records(Mesh& m, const double* x, int precision, int mode) {
  if (!m.inc_pos) {
    TRY(dev_alloc(m.pool, (void**)&m.inc_pos, m.n_inc * sizeof(int)));
    TRY(launch_incidence_positions(m, m.inc_pos));
  }
  const size_t need = m.n_inc * kIncRec * (precision == SYMX_F64 ? 8 : 4);
  if (need > m.inc_rows_bytes) {
    dev_free(m.pool, m.inc_rows);
    m.inc_rows = nullptr;
    m.inc_rows_bytes = 0;
    TRY(dev_alloc(m.pool, &m.inc_rows, need));
    m.inc_rows_bytes = need;
  }
  return launch_incidence_rows_projected(m, x, precision, mode, m.inc_pos, m.inc_rows);
}

static symx_status assemble_main(Mesh& m, const double* x, const double* xt, double dt,
                                 bool want_g, bool want_H, int project, int precision,
                                 bool dirichlet, double* g_out, void* dinv, float* dinv_lo);

// Assemble gradient (float64) and/or Hessian values (precision) at x.  With
// dinv (the Newton solve), the block-Jacobi inverses (N x kDinv, precision's
// type) are produced too and the Hessian goes to the solver's half storage
// (m.lvals64 / m.lvals32); without, to the block arrays (m.vals64 /
// m.vals32).  With dinv_lo (float64 Hessian and dinv only), also the float32
// copies of the values (m.lvals32) and of the inverses (dinv_lo).
symx_status assemble(Mesh& m, const double* x, const double* xt, double dt, bool want_g, bool want_H,
                     int project, int precision, bool dirichlet, double* g_out,
                     void* dinv = nullptr, float* dinv_lo = nullptr) {
  if (dinv_lo) {
    if (precision != SYMX_F64 || !want_H || !dinv) {
      set_error("float32 copies need a float64 Hessian with its inverses");
      return SYMX_ERR_INVALID_ARG;
    }
    TRY(ensure_values(m, SYMX_F32, true));
  }
  TRY(assemble_main(m, x, xt, dt, want_g, want_H, project, precision, dirichlet, g_out, dinv,
                    dinv_lo));
  // copies the row kernel does not write: higher-order meshes (all values),
  // contacts (their values, and the inverses of the nodes they touch)
  if (dinv_lo && (m.ho || m.contacts))
    TRY(launch_round_values(m, m.ho != 0, (const double*)dinv, dinv_lo, kDinv * m.N));
  return SYMX_OK;
}

static symx_status assemble_main(Mesh& m, const double* x, const double* xt, double dt,
                                 bool want_g, bool want_H, int project, int precision,
                                 bool dirichlet, double* g_out, void* dinv, float* dinv_lo) {
  if (project && want_H && m.ho) {
    set_error("per-element PSD projection is not available for quadratic or cubic tets");
    return SYMX_ERR_INVALID_ARG;
  }
  const bool half = dinv != nullptr;
  if (want_H) TRY(ensure_values(m, precision, half));
  if (project && want_H) {
    // filter mode on a Stable Neo-Hookean mesh: the row kernel evaluates the
    // filtered rows itself; otherwise element-wise records, then assembly
    bool snh_only = true;
    for (const SetHost& s : m.sets) snh_only = snh_only && s.kind == SYMX_SNH_TET4;
    if (project == 2 && snh_only) {
      TRY(launch_row_assemble(m, x, xt, dt, want_g, true, precision, dirichlet, nullptr, true,
                              g_out, dinv, dinv_lo, half));
    } else {
      TRY(project_into_records(m, x, precision, project));
      TRY(launch_row_assemble(m, x, xt, dt, want_g, true, precision, dirichlet, m.inc_rows, false,
                              g_out, dinv, dinv_lo, half));
    }
    // contact element Hessians take the nearest-PSD projection in both modes
    return launch_contact_assemble(m, x, want_g, true, true, precision, dirichlet, g_out, dinv);
  }
  if (!want_g && !want_H) return SYMX_OK;
  TRY(launch_row_assemble(m, x, xt, dt, want_g, want_H, precision, dirichlet, nullptr, false,
                          g_out, want_H ? dinv : nullptr, want_H ? dinv_lo : nullptr, half));
  return launch_contact_assemble(m, x, want_g, want_H, false, precision, dirichlet, g_out,
                                 want_H ? dinv : nullptr);
}

symx_status energy(Mesh& m, const double* x, const double* xt, double dt, int precision, double* E) {
  TRY(launch_energy(m, x, xt, dt, precision, m.scalars + D_ENERGY));
  // one synchronisation: the energy and the non-finite flag come back together
  double win[D_FLAG - D_ENERGY + 1];
  bool bad = false;
  TRY(read_window(m, win, &bad));
  if (bad) {
    set_error("non-finite value in positions, energy or gradient");
    return SYMX_ERR_NONFINITE;
  }
  *E = win[0];
  return SYMX_OK;
}

static symx_status dot(Mesh& m, const double* a, const double* b, double* out) {
  TRY(launch_dot64(m, a, b, 3 * m.N, m.scalars + D_DOT));
  return sync_read(m, m.scalars + D_DOT, 1, out);
}

// PCG on H y = b (b float64), y accumulated into dx (float64).  Returns
// iterations through *iters.
static symx_status pcg_solve(Mesh& m, int precision, const double* b, double rtol, int max_iter,
                             double* dx, int* iters, bool* breakdown, int slot) {
  Workspace* w = m.ws;
  PcgBuffers B{w->pcg[0], w->pcg[1], w->pcg[2], w->pcg[3], w->pcg[4], w->pcg[5]};
  const int pp = precision == SYMX_F64 ? SYMX_F64 : SYMX_F32;
  TRY(launch_pcg_init(m, pp, B, b, rtol * rtol, max_iter));
  double S[2];
  int done_iters = 0;
  // first chunk sized from the previous solve, so that few launches run past
  // convergence and few host synchronisations are needed
  const int target = std::max(8, (7 * m.last_pcg_iters[slot]) / 8);
  int chunk = target;
  int k = 0;
  *breakdown = false;
  while (true) {
    // the SpMV kernel of iteration max_iter only records the stop
    const int n = std::min(chunk, max_iter + 1 - k);
    int ran = n;
    if (m.batcher) {
      // serving: the chunk runs in a batched launch with other meshes'
      // chunks, which may run fewer iterations than asked (`ran`)
      TRY(m.batcher->run(m, pp, B, k, n, S, &ran));
    } else {
      TRY(launch_pcg_iters(m, pp, B, k, n));
      TRY(sync_read(m, m.scalars, 2, S));
    }
    k += ran;
    if (S[S_DONE] != 0.0) {
      done_iters = (int)S[S_ITERS];
      *breakdown = S[S_DONE] == 2.0;
      break;
    }
    if (k > max_iter) {  // cannot happen: the last SpMV sets the flag
      set_error("PCG did not stop");
      return SYMX_ERR_DEVICE;
    }
    // the rest of the predicted chunk, then short chunks past the prediction;
    // with no prediction (a fresh mesh), chunks that double, so both the
    // launches that run past convergence and the host synchronisations stay few
    chunk = k < target ? target - k
                       : (m.last_pcg_iters[slot] > 0 ? 8 : std::min(64, std::max(8, k)));
  }
  m.last_pcg_iters[slot] = done_iters;
  *iters = done_iters;
  return launch_accumulate(m, pp, dx, B.xs);
}

// Linear solve H dx = -g with float64 refinement (F32_REFINED).
// `slot` indexes the solve within a step (its Newton iteration); the iteration
// count of the same solve in the previous step sizes the first PCG chunk.
// In F32_REFINED mode the float32 PCG solution is checked against the float64
// Hessian: r = b - H dx in float64; while |r| > eta |b| and passes remain, a
// float32 PCG solve of H c = r (to the relative tolerance that would meet eta,
// but no tighter than 1e-6, what one float32 solve can deliver) is added in
// float64.  *lin_res receives |r| / |b| of the final dx (-1 in other modes).
static symx_status linear_solve(Mesh& m, const symx_step_params& P, const double* g, double eta,
                                double gnorm, int* pcg_iters, int* refinements, int slot,
                                double* lin_res) {
  Workspace* w = m.ws;
  const int n = (int)(3 * m.N);
  *lin_res = -1.0;
  // b = -g ; dx = 0
  TRY(hip_check(hipMemsetAsync(w->dx, 0, n * sizeof(double), m.stream), "hipMemsetAsync"));
  TRY(launch_lincomb64(m, w->b, w->dx, g, -1.0, n));
  int it = 0;
  bool bd = false;
  TRY(pcg_solve(m, P.precision, w->b, eta, P.max_pcg, w->dx, &it, &bd, slot));
  *pcg_iters += it;
  if (P.precision != SYMX_F32_REFINED) return SYMX_OK;
  // A solve that stopped at its iteration limit (or on breakdown) is not
  // corrected: another solve would restart CG, not correct rounding; it is
  // used as is, as in float64 mode (its residual is still reported).
  bool correct = !(bd || it >= P.max_pcg);
  for (int k = 0;; ++k) {
    TRY(launch_residual64(m, SYMX_F64, w->dx, w->b, w->res));
    double rr = 0.0;
    TRY(dot(m, w->res, w->res, &rr));
    const double rn = std::sqrt(rr);
    *lin_res = gnorm > 0.0 ? rn / gnorm : 0.0;
    if (rn <= eta * gnorm || !correct || k >= P.max_refine) break;
    int it2 = 0;
    const double tol = std::max(eta * gnorm / rn, 1e-6);
    TRY(pcg_solve(m, P.precision, w->res, std::min(tol, 0.5), P.max_pcg, w->dx, &it2, &bd,
                  kPcgHistory - 1));
    *pcg_iters += it2;
    *refinements += 1;
    correct = !(bd || it2 >= P.max_pcg);
  }
  return SYMX_OK;
}

// Relative rounding allowance of the line search's energy comparison (the
// float64 sum of the element energies is exact to about 1e-14 relative).
constexpr double kEnergyRound = 1e-12;

using clk = std::chrono::steady_clock;
static double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// One attempt at fixed dt from (x_t, v_t) in the workspace; result in w->xk.
// Host synchronisations per Newton iteration: one after assembly (residual),
// the PCG chunk checks, and one per line-search trial.
static symx_status solve_step(Mesh& m, const symx_step_params& P, double dt, symx_step_report* R) {
  Workspace* w = m.ws;
  const int64_t n = 3 * m.N;
  const int pe = P.precision == SYMX_F32 ? SYMX_F32 : SYMX_F64;  // energies and gradient
  const int ph = P.precision == SYMX_F64 ? SYMX_F64 : SYMX_F32;  // Hessian and PCG
  double win[D_FLAG - D_ENERGY + 1];
  auto at = [&](int slot) { return win[slot - D_ENERGY]; };
  bool bad = false;
  TRY(launch_x_tilde(m, w->x_t, w->v_t, dt, P.gravity, w->xt));
  // lagged rotations (co-rotational and ARAP sets) are those of x(t) for the
  // whole step
  TRY(launch_lagged_rotations(m, w->x_t));
  TRY(hip_check(hipMemcpyAsync(w->xk, w->x_t, n * sizeof(double), hipMemcpyDeviceToDevice, m.stream),
                "hipMemcpyAsync"));
  double r0 = -1.0, E0 = 0.0;
  bool have_E0 = false;
  for (int it = 0;; ++it) {
    auto t0 = clk::now();
    // gradient, Hessian and the block-Jacobi inverses (workspace pcg[0]); in
    // F32_REFINED mode all in float64, then the float32 copies for the PCG
    if (P.precision == SYMX_F32_REFINED) {
      TRY(ensure_dinv64(m));
      TRY(assemble(m, w->xk, w->xt, dt, true, true, P.project, SYMX_F64, true, w->g, w->dinv64,
                   (float*)w->pcg[0]));
    } else {
      TRY(assemble(m, w->xk, w->xt, dt, true, true, P.project, ph, true, w->g, w->pcg[0]));
    }
    TRY(launch_dot64(m, w->g, w->g, n, m.scalars + D_GG));
    if (!have_E0) TRY(launch_energy(m, w->xk, w->xt, dt, pe, m.scalars + D_E0));
    TRY(read_window(m, win, &bad));
    R->ms_assemble += ms_since(t0);
    if (bad) {
      set_error("non-finite value in energy or gradient");
      return SYMX_ERR_NONFINITE;
    }
    if (!have_E0) {
      E0 = at(D_E0);
      have_E0 = true;
    }
    const double r = std::sqrt(at(D_GG));
    if (r0 < 0.0) {
      r0 = r;
      R->residual0 = r0;
    }
    R->residual = r;
    R->energy = E0;
    if (r <= P.newton_rtol * r0) return SYMX_OK;
    if (it >= P.max_newton) {
      set_error("Newton did not converge within max_newton iterations");
      return SYMX_ERR_NOT_CONVERGED;
    }
    auto t1 = clk::now();
    const double eta = std::min(P.forcing_max, std::sqrt(r / r0));
    double lin_res = -1.0;
    TRY(linear_solve(m, P, w->g, eta, r, &R->pcg_iters, &R->refinements,
                     std::min(it, kPcgHistory - 2), &lin_res));
    R->lin_residual = std::max(R->lin_residual, lin_res);
    R->ms_pcg += ms_since(t1);
    auto t2 = clk::now();
    // slope and the full step's energy in one round trip
    TRY(launch_dot64(m, w->g, w->dx, n, m.scalars + D_GD));
    double alpha = 1.0;
    TRY(launch_lincomb64(m, w->xtrial, w->xk, w->dx, alpha, n));
    TRY(launch_energy(m, w->xtrial, w->xt, dt, pe, m.scalars + D_ET));
    TRY(read_window(m, win, &bad));
    const double gd = at(D_GD);
    if (!(gd < 0.0)) {
      set_error("Newton direction is not a descent direction");
      return SYMX_ERR_LINE_SEARCH;
    }
    bool ok = false;
    double Et = at(D_ET);
    for (int ls = 0;; ++ls) {
      if (!bad && Et <= E0 + 1e-4 * alpha * gd + kEnergyRound * std::fabs(E0)) {
        ok = true;
        break;
      }
      if (ls == 30) break;
      alpha *= 0.5;
      R->ls_backtracks++;
      TRY(launch_lincomb64(m, w->xtrial, w->xk, w->dx, alpha, n));
      TRY(launch_energy(m, w->xtrial, w->xt, dt, pe, m.scalars + D_ET));
      TRY(read_window(m, win, &bad));
      Et = at(D_ET);
    }
    R->ms_linesearch += ms_since(t2);
    if (!ok) {
      set_error("line search failed");
      return SYMX_ERR_LINE_SEARCH;
    }
    std::swap(w->xk, w->xtrial);
    E0 = Et;
    R->newton_iters++;
  }
}

symx_status newton_step(Mesh& m, double* x, double* v, const symx_step_params& P,
                        symx_step_report* out) {
  TRY(ensure_workspace(m));
  Workspace* w = m.ws;
  const int64_t n = 3 * m.N;
  symx_step_report R;
  std::memset(&R, 0, sizeof R);
  auto t0 = clk::now();
  TRY(launch_check_finite(m, x, n));
  TRY(launch_check_finite(m, v, n));
  TRY(check_nonfinite(m));
  TRY(hip_check(hipMemcpyAsync(w->x_t, x, n * sizeof(double), hipMemcpyDeviceToDevice, m.stream),
                "hipMemcpyAsync"));
  TRY(hip_check(hipMemcpyAsync(w->v_t, v, n * sizeof(double), hipMemcpyDeviceToDevice, m.stream),
                "hipMemcpyAsync"));
  // Step control: with max_halvings > 0 the mesh carries a reduced dt from
  // step to step (and doubles it back after regrow_after successes); with
  // max_halvings == 0 the step is taken at exactly P.dt and the mesh's step
  // control state is neither used nor changed (e.g. replaying a given dt
  // sequence).
  const bool control = P.max_halvings > 0;
  if (control && m.dt_nominal != P.dt) {
    m.dt_nominal = P.dt;
    m.dt_cur = P.dt;
    m.successes = 0;
  }
  double dt = control ? m.dt_cur : P.dt;
  int halvings = 0;
  symx_status st;
  while (true) {
    symx_step_report attempt;
    std::memset(&attempt, 0, sizeof attempt);
    attempt.lin_residual = -1.0;
    st = solve_step(m, P, dt, &attempt);
    R.newton_iters += attempt.newton_iters;
    R.pcg_iters += attempt.pcg_iters;
    R.ls_backtracks += attempt.ls_backtracks;
    R.refinements += attempt.refinements;
    R.ms_assemble += attempt.ms_assemble;
    R.ms_pcg += attempt.ms_pcg;
    R.ms_linesearch += attempt.ms_linesearch;
    R.residual0 = attempt.residual0;
    R.residual = attempt.residual;
    R.energy = attempt.energy;
    R.lin_residual = attempt.lin_residual;
    if (st == SYMX_OK) break;
    if (st != SYMX_ERR_LINE_SEARCH && st != SYMX_ERR_NOT_CONVERGED) break;
    if (halvings >= P.max_halvings) break;
    dt *= 0.5;
    ++halvings;
  }
  R.dt_halvings = halvings;
  R.dt_used = dt;
  R.status = st;
  if (st == SYMX_OK) {
    TRY(launch_velocity(m, v, w->xk, w->x_t, 1.0 / dt, n));
    TRY(hip_check(hipMemcpyAsync(x, w->xk, n * sizeof(double), hipMemcpyDeviceToDevice, m.stream),
                  "hipMemcpyAsync"));
    TRY(hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize"));
    if (!control) {
      // no step control: the mesh's state stays as it was
    } else if (halvings) {
      m.dt_cur = dt;
      m.successes = 0;
    } else if (++m.successes >= P.regrow_after && m.dt_cur < m.dt_nominal) {
      m.dt_cur = std::min(2.0 * m.dt_cur, m.dt_nominal);
      m.successes = 0;
    }
  }
  R.ms_total = ms_since(t0);
  if (out) *out = R;
  return st;
}

}  // namespace symxi
