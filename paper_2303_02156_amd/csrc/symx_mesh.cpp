// Mesh setup: rest data, block sparsity pattern, scatter map, incidence lists
// and row batches, uploaded once to the device.
//
// Pattern (Sec. 5.3, BCRS with 3x3 blocks; Alg. 1 BlockExists): block (i, j)
// exists iff nodes i and j share an element of any energy set; every node has
// its diagonal block; columns ascend within a row.  The scatter map gives, for
// element e of set s and local nodes (a, b), the position of block
// (conn[e][a], conn[e][b]).
//
// The device assembles row by row.  For every node i the incidence list holds
// its (set, element, local node a) entries in (set, element id) order, which
// fixes the summation order of every block and gradient row.  Each incidence
// also stores the row-local slots of the blocks it touches, in the relabelled
// node order (a first, then the others ascending) that the row kernels use.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "symx_internal.h"

namespace symxi {

namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

template <typename T>
symx_status upload(T** dst, const T* src, size_t n) {
  if (n == 0) n = 1;
  if (hipMalloc((void**)dst, n * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    set_error("device allocation failed");
    return SYMX_ERR_OUT_OF_MEMORY;
  }
  if (src) return hip_check(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return SYMX_OK;
}

#define TRY(expr)                         \
  do {                                    \
    symx_status s_ = (expr);              \
    if (s_ != SYMX_OK) return s_;         \
  } while (0)

}  // namespace

SetsDev Mesh::sets_dev() const {
  SetsDev d{};
  d.n = (int)sets.size();
  for (int s = 0; s < d.n; ++s) {
    const SetHost& h = sets[s];
    d.s[s].kind = h.kind;
    d.s[s].k = h.k;
    d.s[s].n_elem = h.n_elem;
    d.s[s].conn = h.d_conn;
    d.s[s].prm64 = h.d_prm64;
    d.s[s].prm32 = h.d_prm32;
    d.s[s].prm_stride = h.uniform ? 0 : kPrm;
  }
  return d;
}

static symx_status build_set(Mesh& m, const symx_energy_desc& d, SetHost& s) {
  s.kind = d.kind;
  if (d.kind == SYMX_SNH_TET4 || d.kind == SYMX_HINGE4)
    s.k = 4;
  else if (d.kind == SYMX_STVK_TRI3)
    s.k = 3;
  else {
    set_error("unknown energy kind " + std::to_string(d.kind));
    return SYMX_ERR_INVALID_ARG;
  }
  if (d.n_elem < 0 || (d.n_elem > 0 && !d.conn) || d.n_elem >= (int64_t(1) << 28)) {
    set_error("invalid element count or connectivity pointer");
    return SYMX_ERR_INVALID_ARG;
  }
  s.n_elem = d.n_elem;
  s.conn.assign(d.conn, d.conn + d.n_elem * s.k);
  for (int64_t e = 0; e < s.n_elem; ++e)
    for (int a = 0; a < s.k; ++a) {
      int32_t v = s.conn[e * s.k + a];
      if (v < 0 || v >= m.N) {
        set_error("node id out of range in element " + std::to_string(e));
        return SYMX_ERR_INVALID_ARG;
      }
      for (int b = 0; b < a; ++b)
        if (s.conn[e * s.k + b] == v) {
          set_error("repeated node in element " + std::to_string(e));
          return SYMX_ERR_INVALID_ARG;
        }
    }
  const double* X = m.h_X.data();
  auto P = [&](int64_t e, int a) {
    int64_t n = s.conn[e * s.k + a];
    return V3{X[3 * n], X[3 * n + 1], X[3 * n + 2]};
  };
  bool per_elem = (d.young != nullptr) && d.kind != SYMX_HINGE4;
  s.uniform = !per_elem;
  s.prm.assign((per_elem ? s.n_elem : 1) * kPrm, 0.0);
  auto lame = [&](double E, double nu, double* mu, double* lam) {
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  };
  if (d.kind == SYMX_SNH_TET4 || d.kind == SYMX_STVK_TRI3) {
    if (!(d.poisson > -1.0 && d.poisson < 0.5)) {
      set_error("Poisson ratio must lie in (-1, 0.5)");
      return SYMX_ERR_INVALID_ARG;
    }
    for (int64_t e = 0; e < (per_elem ? s.n_elem : 1); ++e) {
      double E = per_elem ? d.young[e] : d.young_const;
      double* p = &s.prm[e * kPrm];
      lame(E, d.poisson, &p[0], &p[1]);
      p[2] = d.thickness;
    }
  }
  // rest measures, masses, hinge weights
  if (d.kind == SYMX_SNH_TET4) {
    for (int64_t e = 0; e < s.n_elem; ++e) {
      V3 x0 = P(e, 0);
      V3 d1 = sub(P(e, 1), x0), d2 = sub(P(e, 2), x0), d3 = sub(P(e, 3), x0);
      double vol = std::fabs(dot(d1, cross(d2, d3))) / 6.0;
      if (!(vol > 0.0)) {
        set_error("degenerate rest tet " + std::to_string(e));
        return SYMX_ERR_INVALID_ARG;
      }
      for (int a = 0; a < 4; ++a) m.h_mass[s.conn[e * 4 + a]] += d.density * vol / 4.0;
    }
  } else if (d.kind == SYMX_STVK_TRI3) {
    for (int64_t e = 0; e < s.n_elem; ++e) {
      V3 x0 = P(e, 0);
      double area = 0.5 * norm(cross(sub(P(e, 1), x0), sub(P(e, 2), x0)));
      if (!(area > 0.0)) {
        set_error("degenerate rest triangle " + std::to_string(e));
        return SYMX_ERR_INVALID_ARG;
      }
      for (int a = 0; a < 3; ++a)
        m.h_mass[s.conn[e * 3 + a]] += d.density * d.thickness * area / 3.0;
    }
  } else {  // hinge: per-element K and c (Eq. 13, Bergou et al. 2006)
    s.uniform = false;
    s.prm.assign(s.n_elem * kPrm, 0.0);
    auto cot = [](V3 u, V3 v) { return dot(u, v) / norm(cross(u, v)); };
    for (int64_t e = 0; e < s.n_elem; ++e) {
      V3 X0 = P(e, 0), X1 = P(e, 1), X2 = P(e, 2), X3 = P(e, 3);
      V3 e01 = sub(X1, X0);
      double A0 = 0.5 * norm(cross(e01, sub(X2, X0)));
      double A1 = 0.5 * norm(cross(e01, sub(X3, X0)));
      if (!(A0 > 0.0) || !(A1 > 0.0)) {
        set_error("degenerate rest hinge " + std::to_string(e));
        return SYMX_ERR_INVALID_ARG;
      }
      // interior angles at X0 (a_t) and X1 (b_t) of wing triangles t = 0, 1
      double ca0 = cot(sub(X1, X0), sub(X2, X0)), cb0 = cot(sub(X0, X1), sub(X2, X1));
      double ca1 = cot(sub(X1, X0), sub(X3, X0)), cb1 = cot(sub(X0, X1), sub(X3, X1));
      double* p = &s.prm[e * kPrm];
      p[0] = cb0 + cb1;
      p[1] = ca0 + ca1;
      p[2] = -(ca0 + cb0);
      p[3] = -(ca1 + cb1);
      p[4] = 3.0 / (A0 + A1);
      p[5] = d.bend_kb;
    }
  }
  return SYMX_OK;
}

static symx_status build_pattern(Mesh& m) {
  const int64_t N = m.N;
  // node -> incidences (set, element, local node), in (set, element) order
  std::vector<int64_t> cnt(N + 1, 0);
  for (const SetHost& s : m.sets)
    for (int32_t v : s.conn) cnt[v + 1]++;
  for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  m.n_inc = cnt[N];
  if (m.n_inc >= (int64_t(1) << 31)) {
    set_error("too many incidences");
    return SYMX_ERR_INVALID_ARG;
  }
  std::vector<uint32_t> code(m.n_inc);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int si = 0; si < (int)m.sets.size(); ++si) {
    const SetHost& s = m.sets[si];
    for (int64_t e = 0; e < s.n_elem; ++e)
      for (int a = 0; a < s.k; ++a) code[fill[s.conn[e * s.k + a]]++] = inc_make(si, a, e);
  }
  // rows: sorted unique neighbour sets
  m.h_row_ptr.assign(N + 1, 0);
  std::vector<int32_t> cols;
  cols.reserve(m.n_inc * 3 + N);
  std::vector<int32_t> nb;
  m.max_row_blocks = 0;
  for (int64_t i = 0; i < N; ++i) {
    nb.clear();
    nb.push_back((int32_t)i);
    for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q) {
      const SetHost& s = m.sets[inc_set(code[q])];
      int64_t e = inc_elem(code[q]);
      for (int b = 0; b < s.k; ++b) nb.push_back(s.conn[e * s.k + b]);
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    if ((int)nb.size() > kMaxRowBlocks) {
      set_error("node " + std::to_string(i) + " couples to more than 255 nodes");
      return SYMX_ERR_INVALID_ARG;
    }
    if (cnt[i + 1] - cnt[i] > kRowWG) {
      set_error("node " + std::to_string(i) + " belongs to more than 256 elements");
      return SYMX_ERR_INVALID_ARG;
    }
    m.max_row_blocks = std::max(m.max_row_blocks, (int)nb.size());
    cols.insert(cols.end(), nb.begin(), nb.end());
    m.h_row_ptr[i + 1] = (int32_t)cols.size();
  }
  if (cols.size() >= (size_t(1) << 31)) {
    set_error("too many blocks");
    return SYMX_ERR_INVALID_ARG;
  }
  m.h_col_idx.swap(cols);
  m.nnzb = (int64_t)m.h_col_idx.size();
  auto slot_of = [&](int32_t i, int32_t j) -> int {
    const int32_t* b = m.h_col_idx.data() + m.h_row_ptr[i];
    const int32_t* e = m.h_col_idx.data() + m.h_row_ptr[i + 1];
    const int32_t* p = std::lower_bound(b, e, j);
    return int(p - b);
  };
  // scatter map (all sets concatenated)
  size_t total = 0;
  for (const SetHost& s : m.sets) total += size_t(s.n_elem) * s.k * s.k;
  m.h_scatter.resize(total);
  size_t off = 0;
  for (const SetHost& s : m.sets) {
    for (int64_t e = 0; e < s.n_elem; ++e)
      for (int a = 0; a < s.k; ++a) {
        int32_t i = s.conn[e * s.k + a];
        for (int b = 0; b < s.k; ++b)
          m.h_scatter[off++] = m.h_row_ptr[i] + slot_of(i, s.conn[e * s.k + b]);
      }
  }
  // incidence slots in the relabelled order (a first, then the others)
  std::vector<uint32_t> slots(m.n_inc);
  std::vector<std::vector<int32_t>> inc_pos(m.sets.size());
  for (size_t si = 0; si < m.sets.size(); ++si) inc_pos[si].assign(m.sets[si].n_elem * m.sets[si].k, -1);
  for (int64_t i = 0; i < N; ++i)
    for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q) {
      int si = inc_set(code[q]);
      const SetHost& s = m.sets[si];
      int a = inc_local(code[q]);
      int64_t e = inc_elem(code[q]);
      uint32_t w = 0;
      int bp = 0;
      int order[4] = {a, -1, -1, -1};
      for (int b = 0, t = 1; b < s.k; ++b)
        if (b != a) order[t++] = b;
      for (bp = 0; bp < 4; ++bp) {
        uint32_t sl = kNoSlot;
        if (bp < s.k) sl = (uint32_t)slot_of((int32_t)i, s.conn[e * s.k + order[bp]]);
        w |= sl << (8 * bp);
      }
      slots[q] = w;
      inc_pos[si][e * s.k + a] = (int32_t)q;
    }
  // row batches: consecutive rows with <= kRowWG incidences and <= kRowWG blocks
  std::vector<int32_t> batch{0};
  int64_t bi = 0, bb = 0;
  for (int64_t i = 0; i < N; ++i) {
    int64_t ni = cnt[i + 1] - cnt[i];
    int64_t nbk = m.h_row_ptr[i + 1] - m.h_row_ptr[i];
    if (i > batch.back() && (bi + ni > kRowWG || bb + nbk > kRowWG)) {
      batch.push_back((int32_t)i);
      bi = bb = 0;
    }
    bi += ni;
    bb += nbk;
  }
  batch.push_back((int32_t)N);
  m.n_batch = (int)batch.size() - 1;
  // Off-diagonal contribution lists.  For every off-diagonal block of a batch,
  // the (incidence, relabelled node b >= 1) pairs that add to it, in incidence
  // order; entries are u16 = (incidence index within the batch << 2) | b.
  // blk_info[p] = (first entry relative to the batch's base << 8) | count.
  std::vector<uint32_t> blk_info(m.nnzb, 0);
  std::vector<uint16_t> centry;
  centry.reserve(m.n_inc * 3);
  std::vector<int32_t> batch_entry(m.n_batch + 1, 0);
  std::vector<int32_t> cnt_blk, fillp;
  for (int b = 0; b < m.n_batch; ++b) {
    const int64_t r0 = batch[b], r1 = batch[b + 1];
    const int64_t q0 = cnt[r0], p0 = m.h_row_ptr[r0];
    const int64_t np = m.h_row_ptr[r1] - p0;
    batch_entry[b] = (int32_t)centry.size();
    cnt_blk.assign(np + 1, 0);
    for (int64_t r = r0; r < r1; ++r)
      for (int64_t q = cnt[r]; q < cnt[r + 1]; ++q) {
        const int k = m.sets[inc_set(code[q])].k;
        for (int bp = 1; bp < k; ++bp) {
          const int64_t pl = m.h_row_ptr[r] + ((slots[q] >> (8 * bp)) & 0xFFu) - p0;
          cnt_blk[pl + 1]++;
        }
      }
    for (int64_t i = 0; i < np; ++i) {
      if (cnt_blk[i + 1] > 255) {
        set_error("more than 255 elements share one node pair");
        return SYMX_ERR_INVALID_ARG;
      }
      blk_info[p0 + i] = (uint32_t(cnt_blk[i]) << 8) | uint32_t(cnt_blk[i + 1]);
      cnt_blk[i + 1] += cnt_blk[i];
    }
    if (cnt_blk[np] >= (1 << 24)) {
      set_error("batch contribution list too long");
      return SYMX_ERR_INVALID_ARG;
    }
    const size_t base = centry.size();
    centry.resize(base + cnt_blk[np]);
    fillp.assign(cnt_blk.begin(), cnt_blk.end() - 1);
    for (int64_t r = r0; r < r1; ++r)
      for (int64_t q = cnt[r]; q < cnt[r + 1]; ++q) {
        const int k = m.sets[inc_set(code[q])].k;
        for (int bp = 1; bp < k; ++bp) {
          const int64_t pl = m.h_row_ptr[r] + ((slots[q] >> (8 * bp)) & 0xFFu) - p0;
          centry[base + fillp[pl]++] = (uint16_t)(((q - q0) << 2) | bp);
        }
      }
  }
  batch_entry[m.n_batch] = (int32_t)centry.size();
  // device upload
  std::vector<int32_t> inc_ptr32(N + 1);
  for (int64_t i = 0; i <= N; ++i) inc_ptr32[i] = (int32_t)cnt[i];
  std::vector<int32_t> diag(N);
  for (int64_t i = 0; i < N; ++i) diag[i] = m.h_row_ptr[i] + slot_of((int32_t)i, (int32_t)i);
  TRY(upload(&m.row_ptr, m.h_row_ptr.data(), N + 1));
  TRY(upload(&m.col_idx, m.h_col_idx.data(), m.nnzb));
  TRY(upload(&m.diag_pos, diag.data(), N));
  TRY(upload(&m.inc_ptr, inc_ptr32.data(), N + 1));
  TRY(upload(&m.inc_code, code.data(), m.n_inc));
  TRY(upload(&m.inc_slots, slots.data(), m.n_inc));
  TRY(upload(&m.batch_row, batch.data(), batch.size()));
  TRY(upload(&m.blk_info, blk_info.data(), blk_info.size()));
  TRY(upload(&m.centry, centry.data(), centry.size()));
  TRY(upload(&m.batch_entry, batch_entry.data(), batch_entry.size()));
  for (size_t si = 0; si < m.sets.size(); ++si)
    TRY(upload(&m.sets[si].d_inc_pos, inc_pos[si].data(), inc_pos[si].size()));
  return SYMX_OK;
}

static symx_status upload_mesh(Mesh& m) {
  TRY(upload(&m.X, m.h_X.data(), m.h_X.size()));
  TRY(upload(&m.mass, m.h_mass.data(), m.h_mass.size()));
  TRY(upload(&m.fixed, m.h_fixed.data(), m.h_fixed.size()));
  for (SetHost& s : m.sets) {
    std::vector<int4> c4(std::max<int64_t>(s.n_elem, 1));
    for (int64_t e = 0; e < s.n_elem; ++e) {
      int v[4] = {-1, -1, -1, -1};
      for (int a = 0; a < s.k; ++a) v[a] = s.conn[e * s.k + a];
      c4[e] = make_int4(v[0], v[1], v[2], v[3]);
    }
    TRY(upload(&s.d_conn, c4.data(), c4.size()));
    std::vector<float> p32(s.prm.begin(), s.prm.end());
    TRY(upload(&s.d_prm64, s.prm.data(), s.prm.size()));
    TRY(upload(&s.d_prm32, p32.data(), p32.size()));
  }
  TRY(upload<double>(&m.partials, nullptr, kMaxPartials));
  TRY(upload<double>(&m.scalars, nullptr, 64));
  TRY(hip_check(hipMemset(m.scalars, 0, 64 * sizeof(double)), "hipMemset"));
  // the non-finite flag shares the scalar array (slot 24) so the Newton driver
  // reads results and flag with one copy
  m.nonfinite = reinterpret_cast<int*>(m.scalars + 24);
  if (hipHostMalloc((void**)&m.pinned, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    m.pinned = nullptr;
    set_error("pinned host allocation failed");
    return SYMX_ERR_OUT_OF_MEMORY;
  }
  return SYMX_OK;
}

symx_status mesh_create(const symx_mesh_desc* d, Mesh** out) {
  if (!d || !out || d->n_nodes < 1 || !d->x_rest || d->n_energies < 1 ||
      d->n_energies > kMaxSets || !d->energies) {
    set_error("invalid mesh descriptor");
    return SYMX_ERR_INVALID_ARG;
  }
  if (d->n_nodes >= (int64_t(1) << 31) / 3) {
    set_error("too many nodes");
    return SYMX_ERR_INVALID_ARG;
  }
  Mesh* m = new (std::nothrow) Mesh();
  if (!m) return SYMX_ERR_OUT_OF_MEMORY;
  *out = m;  // the caller destroys on error
  TRY(hip_check(hipGetDevice(&m->device), "hipGetDevice"));
  m->stream = (hipStream_t)d->hip_stream;
  m->N = d->n_nodes;
  m->h_X.assign(d->x_rest, d->x_rest + 3 * m->N);
  for (double v : m->h_X)
    if (!std::isfinite(v)) {
      set_error("non-finite rest position");
      return SYMX_ERR_INVALID_ARG;
    }
  m->h_fixed.assign(m->N, 0);
  if (d->fixed)
    for (int64_t i = 0; i < m->N; ++i) m->h_fixed[i] = d->fixed[i] ? 1 : 0;
  m->h_mass.assign(m->N, 0.0);
  m->sets.resize(d->n_energies);
  for (int s = 0; s < d->n_energies; ++s) TRY(build_set(*m, d->energies[s], m->sets[s]));
  m->total_mass = 0.0;
  for (double v : m->h_mass) m->total_mass += v;
  TRY(build_pattern(*m));
  TRY(upload_mesh(*m));
  return SYMX_OK;
}

void mesh_free(Mesh* m);

}  // namespace symxi
