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
// fixes the summation order of every block and gradient row.  The row-local
// slots of the blocks an incidence touches (relabelled node order: a first,
// then the others ascending) define each block's contribution list: the
// (incidence, node) pairs that add to it, in incidence order.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>

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

// Allocate n elements (through the pool, if any) and copy src to them on
// `stream`; returns when the copy is done, so src may be freed at once.
// *bytes accumulates the allocation size.
template <typename T>
symx_status upload(DevicePool* pool, hipStream_t stream, T** dst, const T* src, size_t n,
                   size_t* bytes = nullptr) {
  if (n == 0) n = 1;
  void* p = nullptr;
  symx_status st = dev_alloc(pool, &p, n * sizeof(T));
  *dst = static_cast<T*>(p);
  if (st != SYMX_OK) return st;
  if (bytes) *bytes += n * sizeof(T);
  if (!src) return SYMX_OK;
  st = hip_check(hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, stream),
                 "hipMemcpyAsync");
  if (st == SYMX_OK) st = hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  return st;
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
    d.s[s].rot64 = h.d_rot64;
    d.s[s].rot32 = h.d_rot32;
    d.s[s].conn_ho = h.d_conn_ho;
  }
  return d;
}

SetDev Mesh::dyn_dev() const {
  SetDev d{};
  d.kind = dyn.kind;
  d.k = 4;
  d.n_elem = contacts && contacts->kind >= 0 ? contacts->n : 0;
  d.conn = d.n_elem ? reinterpret_cast<const int4*>(contacts->tuples) : nullptr;
  d.prm64 = dyn.d_prm64;
  d.prm32 = dyn.d_prm32;
  d.prm_stride = dyn.uniform ? 0 : kPrm;
  d.rot64 = nullptr;
  d.rot32 = nullptr;
  d.conn_ho = nullptr;
  return d;
}

static int host_threads() {
  return (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
}

// Run f(th) for th = 0..T-1 on T host threads.
template <typename F>
static void parallel_for_threads(int T, F f) {
  if (T <= 1) {
    f(0);
    return;
  }
  std::vector<std::thread> th;
  for (int i = 1; i < T; ++i) th.emplace_back(f, i);
  f(0);
  for (auto& x : th) x.join();
}

// Run f(lo, hi) over [0, n) split into contiguous chunks on host threads.
template <typename F>
static void parallel_chunks(int64_t n, int64_t min_chunk, F f) {
  int T = host_threads();
  T = (int)std::max<int64_t>(1, std::min<int64_t>(T, n / std::max<int64_t>(min_chunk, 1)));
  if (T <= 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) th.emplace_back(f, n * t / T, n * (t + 1) / T);
  for (auto& x : th) x.join();
}

// Nodes per element, 0 for an unknown kind.
static int known_kind_nodes(int kind) {
  return kind >= SYMX_SNH_TET4 && kind <= SYMX_SNH_TET20 ? kind_nodes(kind) : 0;
}

// Element kind, count and connectivity of one energy set.  check_nodes: node
// ids in range and distinct within each element (skipped when the
// connectivity equals that of a cached, already validated topology).
static symx_status validate_set(const symx_energy_desc& d, int64_t N, bool check_nodes) {
  const int k = known_kind_nodes(d.kind);
  if (k == 0) {
    set_error("unknown energy kind " + std::to_string(d.kind));
    return SYMX_ERR_INVALID_ARG;
  }
  if (d.n_elem < 0 || (d.n_elem > 0 && !d.conn) || d.n_elem >= (int64_t(1) << kMaxElemBits)) {
    set_error("invalid element count or connectivity pointer");
    return SYMX_ERR_INVALID_ARG;
  }
  if (!check_nodes) return SYMX_OK;
  std::atomic<int64_t> bad_range{-1}, bad_repeat{-1};
  const int32_t* conn = d.conn;
  parallel_chunks(d.n_elem, 16384, [&](int64_t e0, int64_t e1) {
    for (int64_t e = e0; e < e1; ++e)
      for (int a = 0; a < k; ++a) {
        const int32_t v = conn[e * k + a];
        if (v < 0 || v >= N) bad_range = e;
        for (int b = 0; b < a; ++b)
          if (conn[e * k + b] == v) bad_repeat = e;
      }
  });
  if (bad_range >= 0) {
    set_error("node id out of range in element " + std::to_string(bad_range.load()));
    return SYMX_ERR_INVALID_ARG;
  }
  if (bad_repeat >= 0) {
    set_error("repeated node in element " + std::to_string(bad_repeat.load()));
    return SYMX_ERR_INVALID_ARG;
  }
  return SYMX_OK;
}

// Keep the smallest element id that failed a check.
static void note_first(std::atomic<int64_t>& first, int64_t e) {
  int64_t cur = first.load();
  while ((cur < 0 || e < cur) && !first.compare_exchange_weak(cur, e)) {
  }
}

// HRZ lumping of higher-order tets: node a's share of the element mass is its
// consistent-mass diagonal, the integral of N_a^2, over the sum of the
// diagonal.  With the integral of L0^p L1^q L2^r L3^s over a tet of volume V
// equal to 6V p!q!r!s!/(p+q+r+s+3)!, the diagonal is V/70 at a corner and
// 8V/105 at an edge node of a quadratic tet; V/280 at a corner, 27V/1120 at an
// edge node and 27V/280 at a face node of a cubic tet.  Other kinds: 1 (their
// element mass is per node).
static double ho_mass_share(int k, int a) {
  if (k == 10) {
    const double dc = 1.0 / 70.0, de = 8.0 / 105.0;
    return (a < 4 ? dc : de) / (4.0 * dc + 6.0 * de);
  }
  if (k == 20) {
    const double dc = 1.0 / 280.0, de = 27.0 / 1120.0, df = 27.0 / 280.0;
    return (a < 4 ? dc : a < 16 ? de : df) / (4.0 * dc + 12.0 * de + 4.0 * df);
  }
  return 1.0;
}

// Per-mesh data of one energy set: parameters and rest measures.  elem_mass
// receives each element's lumped mass per node (rho V / 4 per tet, rho h A / 3
// per triangle; hinges carry none), or for higher-order tets the element mass
// rho V that ho_mass_share splits over the nodes.
static symx_status build_set(Mesh& m, const symx_energy_desc& d, SetHost& s,
                             std::vector<double>& elem_mass) {
  s.kind = d.kind;
  s.k = kind_nodes(d.kind);
  s.n_elem = d.n_elem;
  const int32_t* conn = d.conn;
  const double* X = m.h_X.data();
  auto P = [&](int64_t e, int a) {
    int64_t n = conn[e * s.k + a];
    return V3{X[3 * n], X[3 * n + 1], X[3 * n + 2]};
  };
  bool per_elem = (d.young != nullptr) && d.kind != SYMX_HINGE4;
  s.uniform = !per_elem;
  s.prm.assign((per_elem ? s.n_elem : 1) * kPrm, 0.0);
  auto lame = [&](double E, double nu, double* mu, double* lam) {
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  };
  if (d.kind != SYMX_HINGE4) {
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
  // rest measures, element masses, hinge weights
  std::atomic<int64_t> bad{-1};
  if ((s.k == 4 && d.kind != SYMX_HINGE4) || s.k >= 10) {
    // linear tets: rho V / 4 per node; higher-order tets: rho V (V of the
    // corner tet)
    const double share = s.k >= 10 ? 1.0 : 0.25;
    elem_mass.resize(s.n_elem);
    parallel_chunks(s.n_elem, 16384, [&](int64_t e0, int64_t e1) {
      for (int64_t e = e0; e < e1; ++e) {
        V3 x0 = P(e, 0);
        V3 d1 = sub(P(e, 1), x0), d2 = sub(P(e, 2), x0), d3 = sub(P(e, 3), x0);
        const double vol = std::fabs(dot(d1, cross(d2, d3))) / 6.0;
        if (!(vol > 0.0)) note_first(bad, e);
        elem_mass[e] = d.density * vol * share;
      }
    });
    if (bad >= 0) {
      set_error("degenerate rest tet " + std::to_string(bad.load()));
      return SYMX_ERR_INVALID_ARG;
    }
  } else if (d.kind == SYMX_STVK_TRI3) {
    elem_mass.resize(s.n_elem);
    parallel_chunks(s.n_elem, 16384, [&](int64_t e0, int64_t e1) {
      for (int64_t e = e0; e < e1; ++e) {
        V3 x0 = P(e, 0);
        const double area = 0.5 * norm(cross(sub(P(e, 1), x0), sub(P(e, 2), x0)));
        if (!(area > 0.0)) note_first(bad, e);
        elem_mass[e] = d.density * d.thickness * area / 3.0;
      }
    });
    if (bad >= 0) {
      set_error("degenerate rest triangle " + std::to_string(bad.load()));
      return SYMX_ERR_INVALID_ARG;
    }
  } else {  // hinge: per-element K and c (Eq. 13, Bergou et al. 2006)
    elem_mass.clear();
    s.uniform = false;
    s.prm.assign(s.n_elem * kPrm, 0.0);
    auto cot = [](V3 u, V3 v) { return dot(u, v) / norm(cross(u, v)); };
    parallel_chunks(s.n_elem, 16384, [&](int64_t e0, int64_t e1) {
      for (int64_t e = e0; e < e1; ++e) {
        V3 X0 = P(e, 0), X1 = P(e, 1), X2 = P(e, 2), X3 = P(e, 3);
        V3 e01 = sub(X1, X0);
        double A0 = 0.5 * norm(cross(e01, sub(X2, X0)));
        double A1 = 0.5 * norm(cross(e01, sub(X3, X0)));
        if (!(A0 > 0.0) || !(A1 > 0.0)) {
          note_first(bad, e);
          continue;
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
    });
    if (bad >= 0) {
      set_error("degenerate rest hinge " + std::to_string(bad.load()));
      return SYMX_ERR_INVALID_ARG;
    }
  }
  return SYMX_OK;
}

// Pattern, incidence lists, row batches and contribution lists of the
// connectivity in `d` (already validated), uploaded on `stream`.
static symx_status build_topology(const symx_mesh_desc& d, DevicePool* pool, hipStream_t stream,
                                  std::shared_ptr<Topology>* out) {
  auto tp = std::make_shared<Topology>();
  Topology& t = *tp;
  t.pool = pool;
  t.hash = topology_hash(d);
  t.N = d.n_nodes;
  t.sets.resize(d.n_energies);
  for (int si = 0; si < d.n_energies; ++si) {
    TopoSet& ts = t.sets[si];
    ts.kind = d.energies[si].kind;
    ts.k = kind_nodes(ts.kind);
    ts.n_elem = d.energies[si].n_elem;
    ts.conn.assign(d.energies[si].conn, d.energies[si].conn + ts.n_elem * ts.k);
    t.ho = std::max(t.ho, kind_high_order(ts.kind));
  }
  // incidences per batch, and slot bytes per incidence (see below)
  const int inc_cap = t.ho == 20 ? kCubicInc : t.ho == 10 ? kQuadInc : kRowWG;
  const int KS = t.ho ? t.ho : 4;
  const int64_t N = t.N;
  // Node -> incidences (set, element, local node), in (set, element) order:
  // a counting sort over the concatenated element list, split into
  // contiguous ranges, one per host thread.  Thread ranges are taken in
  // order for every node, so each node's list keeps (set, element) order.
  int64_t n_all = 0;
  std::vector<int64_t> set_first(t.sets.size() + 1, 0);
  for (size_t si = 0; si < t.sets.size(); ++si) set_first[si + 1] = set_first[si] + t.sets[si].n_elem;
  n_all = set_first.back();
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n_all / 16384));
  std::vector<uvector<int32_t>> local(T);
  auto for_range = [&](int th, auto&& f) {  // f(set, element) over thread th's range
    const int64_t g0 = n_all * th / T, g1 = n_all * (th + 1) / T;
    for (size_t si = 0; si < t.sets.size(); ++si) {
      const int64_t lo = std::max(g0, set_first[si]), hi = std::min(g1, set_first[si + 1]);
      for (int64_t g = lo; g < hi; ++g) f((int)si, g - set_first[si]);
    }
  };
  parallel_for_threads(T, [&](int th) {
    local[th].assign(N, 0);
    for_range(th, [&](int si, int64_t e) {
      const TopoSet& s = t.sets[si];
      for (int a = 0; a < s.k; ++a) local[th][s.conn[e * s.k + a]]++;
    });
  });
  std::vector<int64_t> cnt(N + 1, 0);
  std::atomic<int64_t> crowded{-1};
  parallel_chunks(N, 16384, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int32_t c = 0;
      for (int th = 0; th < T; ++th) {
        const int32_t n = local[th][i];
        local[th][i] = c;  // becomes the thread's offset within node i's list
        c += n;
      }
      cnt[i + 1] = c;
      if (c > inc_cap) crowded = i;
    }
  });
  if (crowded >= 0) {
    set_error("node " + std::to_string(crowded.load()) + " belongs to more than " +
              std::to_string(inc_cap) + " elements");
    return SYMX_ERR_INVALID_ARG;
  }
  for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  t.n_inc = cnt[N];
  if (t.n_inc >= (int64_t(1) << 31)) {
    set_error("too many incidences");
    return SYMX_ERR_INVALID_ARG;
  }
  uvector<uint32_t> code(t.n_inc);
  parallel_for_threads(T, [&](int th) {
    for_range(th, [&](int si, int64_t e) {
      const TopoSet& s = t.sets[si];
      for (int a = 0; a < s.k; ++a) {
        const int32_t v = s.conn[e * s.k + a];
        code[cnt[v] + local[th][v]++] = inc_make(si, a, e);
      }
    });
  });
  local.clear();
  t.h_inc_ptr = cnt;
  // Rows in parallel chunks: sorted unique neighbour list of each node, and
  // for each incidence the row-local slots of its blocks in the relabelled
  // node order.  Up to four nodes: a first, then the others ascending
  // (slots[KS q + b], b = 0..3).  Higher-order tets (k nodes): the k - 1
  // other nodes in the order of the row function (kTet10Perm or kTet20Perm,
  // position ho_row_pos(k, a) left out), slots[KS q + j], j = 0..k-2.  Each thread marks the nodes already in
  // the current row (mark[j] == row) and maps node -> slot (pos[j]), so a row
  // costs O(incidences) plus a sort of its few columns.
  uvector<uint8_t> slots(t.n_inc * KS);
  std::vector<int32_t> row_len(N);
  const int64_t n_chunks = std::min<int64_t>(64, std::max<int64_t>(1, N / 2048));
  std::vector<std::vector<int32_t>> chunk_cols(n_chunks);
  std::vector<int> chunk_bad(n_chunks, 0);
  parallel_chunks(n_chunks, 1, [&](int64_t c0, int64_t c1) {
    std::vector<int32_t> nb;
    uvector<int32_t> mark(N), pos(N);
    for (int64_t i = 0; i < N; ++i) mark[i] = -1;
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t r0 = N * c / n_chunks, r1 = N * (c + 1) / n_chunks;
      std::vector<int32_t>& cols = chunk_cols[c];
      for (int64_t i = r0; i < r1; ++i) {
        nb.clear();
        nb.push_back((int32_t)i);
        mark[i] = (int32_t)i;
        for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q) {
          const TopoSet& s = t.sets[inc_set(code[q])];
          const int64_t e = inc_elem(code[q]);
          for (int b = 0; b < s.k; ++b) {
            const int32_t j = s.conn[e * s.k + b];
            if (mark[j] != (int32_t)i) {
              mark[j] = (int32_t)i;
              nb.push_back(j);
            }
          }
        }
        std::sort(nb.begin(), nb.end());
        if ((int)nb.size() > kMaxRowBlocks) chunk_bad[c] = 1;
        row_len[i] = (int32_t)nb.size();
        for (size_t sl = 0; sl < nb.size(); ++sl) pos[nb[sl]] = (int32_t)sl;
        for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q) {
          const int si = inc_set(code[q]);
          const TopoSet& s = t.sets[si];
          const int a = inc_local(code[q]);
          const int64_t e = inc_elem(code[q]);
          uint8_t* sq = slots.data() + KS * q;
          if (s.k >= 10) {
            const int r = ho_row_pos(s.k, a);
            const int8_t* perm = s.k == 10 ? kTet10Perm.p[a] : kTet20Perm.p[a];
            for (int bp = 0, j = 0; bp < s.k; ++bp)
              if (bp != r) sq[j++] = (uint8_t)pos[s.conn[e * s.k + perm[bp]]];
          } else {
            int order[4] = {a, -1, -1, -1};
            for (int b = 0, o = 1; b < s.k; ++b)
              if (b != a) order[o++] = b;
            for (int bp = 0; bp < 4; ++bp)
              sq[bp] = bp < s.k ? (uint8_t)pos[s.conn[e * s.k + order[bp]]] : (uint8_t)kNoSlot;
          }
        }
        cols.insert(cols.end(), nb.begin(), nb.end());
      }
    }
  });
  for (int64_t c = 0; c < n_chunks; ++c)
    if (chunk_bad[c]) {
      set_error("a node couples to more than 255 nodes");
      return SYMX_ERR_INVALID_ARG;
    }
  t.h_row_ptr.assign(N + 1, 0);
  t.max_row_blocks = 0;
  for (int64_t i = 0; i < N; ++i) {
    t.h_row_ptr[i + 1] = t.h_row_ptr[i] + row_len[i];
    t.max_row_blocks = std::max(t.max_row_blocks, (int)row_len[i]);
  }
  if ((int64_t)t.h_row_ptr[N] >= (int64_t(1) << 31) - 1) {
    set_error("too many blocks");
    return SYMX_ERR_INVALID_ARG;
  }
  t.nnzb = t.h_row_ptr[N];
  t.h_col_idx.resize(t.nnzb);
  {
    std::vector<int64_t> off(n_chunks + 1, 0);
    for (int64_t c = 0; c < n_chunks; ++c) off[c + 1] = off[c] + (int64_t)chunk_cols[c].size();
    parallel_chunks(n_chunks, 1, [&](int64_t c0, int64_t c1) {
      for (int64_t c = c0; c < c1; ++c)
        std::copy(chunk_cols[c].begin(), chunk_cols[c].end(), t.h_col_idx.begin() + off[c]);
    });
  }
  chunk_cols.clear();
  // row batches: consecutive rows with <= inc_cap incidences and <= kRowWG
  // blocks
  std::vector<int32_t> batch{0};
  int64_t bi = 0, bb = 0;
  for (int64_t i = 0; i < N; ++i) {
    const int64_t ni = cnt[i + 1] - cnt[i];
    const int64_t nbk = row_len[i];
    if (i > batch.back() && (bi + ni > inc_cap || bb + nbk > kRowWG)) {
      batch.push_back((int32_t)i);
      bi = bb = 0;
    }
    bi += ni;
    bb += nbk;
  }
  batch.push_back((int32_t)N);
  t.n_batch = (int)batch.size() - 1;
  // Off-diagonal contribution lists.  For every off-diagonal block of a batch,
  // the (incidence, relabelled node) pairs that add to it, in incidence order;
  // entries are u16 = (incidence index within the batch << 2) | b with b >= 1
  // the relabelled position, or (incidence << 4) | j for quadratic tets and
  // (incidence << 5) | j for cubic tets (j = 0..k-2, the row function's
  // order).  blk_info[p] = (first entry relative to
  // the batch's base << 8) | count.
  std::vector<int32_t> batch_entry(t.n_batch + 1, 0);
  for (int b = 0; b < t.n_batch; ++b) {
    int64_t ne = 0;
    for (int64_t q = cnt[batch[b]]; q < cnt[batch[b + 1]]; ++q) ne += t.sets[inc_set(code[q])].k - 1;
    batch_entry[b + 1] = batch_entry[b] + (int32_t)ne;
  }
  uvector<uint32_t> blk_info(t.nnzb);
  uvector<uint16_t> centry(batch_entry[t.n_batch]);
  std::vector<int> batch_bad(t.n_batch, 0);
  parallel_chunks(t.n_batch, 256, [&](int64_t b0, int64_t b1) {
    std::vector<int32_t> cnt_blk, fillp;
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t r0 = batch[b], r1 = batch[b + 1];
      const int64_t q0 = cnt[r0], p0 = t.h_row_ptr[r0];
      const int64_t np = t.h_row_ptr[r1] - p0;
      cnt_blk.assign(np + 1, 0);
      // the blocks an incidence adds to: slots j0..j0+k-2 of its entry
      const int j0 = t.ho ? 0 : 1;
      const int shift = t.ho == 20 ? 5 : t.ho == 10 ? 4 : 2;
      for (int64_t r = r0; r < r1; ++r)
        for (int64_t q = cnt[r]; q < cnt[r + 1]; ++q) {
          const int k = t.sets[inc_set(code[q])].k;
          for (int j = j0; j < j0 + k - 1; ++j)
            cnt_blk[t.h_row_ptr[r] + slots[KS * q + j] - p0 + 1]++;
        }
      for (int64_t i = 0; i < np; ++i) {
        if (cnt_blk[i + 1] > 255) batch_bad[b] = 1;
        blk_info[p0 + i] = (uint32_t(cnt_blk[i]) << 8) | uint32_t(cnt_blk[i + 1]);
        cnt_blk[i + 1] += cnt_blk[i];
      }
      if (cnt_blk[np] >= (1 << 24)) batch_bad[b] = 1;
      uint16_t* base = centry.data() + batch_entry[b];
      fillp.assign(cnt_blk.begin(), cnt_blk.end() - 1);
      for (int64_t r = r0; r < r1; ++r)
        for (int64_t q = cnt[r]; q < cnt[r + 1]; ++q) {
          const int k = t.sets[inc_set(code[q])].k;
          for (int j = j0; j < j0 + k - 1; ++j) {
            const int64_t pl = t.h_row_ptr[r] + slots[KS * q + j] - p0;
            base[fillp[pl]++] = (uint16_t)(((q - q0) << shift) | j);
          }
        }
    }
  });
  for (int b = 0; b < t.n_batch; ++b)
    if (batch_bad[b]) {
      set_error("more than 255 elements share one node pair");
      return SYMX_ERR_INVALID_ARG;
    }
  // device upload
  std::vector<int32_t> inc_ptr32(N + 1);
  for (int64_t i = 0; i <= N; ++i) inc_ptr32[i] = (int32_t)cnt[i];
  std::vector<int32_t> diag(N);
  for (int64_t i = 0; i < N; ++i) {
    const int32_t* b = t.h_col_idx.data() + t.h_row_ptr[i];
    diag[i] = t.h_row_ptr[i] + (int32_t)(std::lower_bound(b, b + row_len[i], (int32_t)i) - b);
  }
  // The solver's half storage: row i keeps its blocks (i, j) with j <= i
  // (the pattern is symmetric); an upper block (i, j), j > i, is read as the
  // transpose of block (j, i).  cv[p] pairs each pattern slot's column with
  // the half position it reads (bitwise complement for a transpose), so that
  // one load per block gives the solver both.
  std::vector<int32_t> lrow(N + 1, 0);
  for (int64_t i = 0; i < N; ++i) lrow[i + 1] = lrow[i] + (diag[i] - t.h_row_ptr[i] + 1);
  t.nnzl = lrow[N];
  uvector<int2> cv(t.nnzb);
  std::atomic<int> asym{0};
  parallel_chunks(N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      for (int32_t p = t.h_row_ptr[i]; p <= diag[i]; ++p)
        cv[p] = make_int2(t.h_col_idx[p], lrow[i] + (p - t.h_row_ptr[i]));
      for (int32_t p = diag[i] + 1; p < t.h_row_ptr[i + 1]; ++p) {
        const int32_t j = t.h_col_idx[p];
        const int32_t* b = t.h_col_idx.data() + t.h_row_ptr[j];
        const int32_t* e = t.h_col_idx.data() + diag[j];
        const int32_t* f = std::lower_bound(b, e, (int32_t)i);
        if (f == e || *f != (int32_t)i) asym = 1;
        cv[p] = make_int2(j, ~(lrow[j] + (int32_t)(f - b)));
      }
    }
  });
  if (asym) {
    set_error("block pattern is not symmetric");
    return SYMX_ERR_INVALID_ARG;
  }
  size_t& nb = t.device_bytes;
  TRY(upload(pool, stream, &t.row_ptr, t.h_row_ptr.data(), N + 1, &nb));
  TRY(upload(pool, stream, &t.col_idx, t.h_col_idx.data(), t.nnzb, &nb));
  TRY(upload(pool, stream, &t.diag_pos, diag.data(), N, &nb));
  TRY(upload(pool, stream, &t.lrow_ptr, lrow.data(), N + 1, &nb));
  TRY(upload(pool, stream, &t.cv, cv.data(), cv.size(), &nb));
  TRY(upload(pool, stream, &t.inc_ptr, inc_ptr32.data(), N + 1, &nb));
  TRY(upload(pool, stream, &t.inc_code, code.data(), t.n_inc, &nb));
  if (t.ho) {
    // each incidence's element node ids in the relabelled order of its node,
    // so that the row kernel reads them contiguously per batch
    const int K = t.ho;
    uvector<int32_t> nodes(t.n_inc * K);
    parallel_chunks(t.n_inc, 65536, [&](int64_t q0, int64_t q1) {
      for (int64_t q = q0; q < q1; ++q) {
        const TopoSet& s = t.sets[inc_set(code[q])];
        const int a = inc_local(code[q]);
        const int8_t* perm = K == 10 ? kTet10Perm.p[a] : kTet20Perm.p[a];
        const int32_t* c = s.conn.data() + (int64_t)K * inc_elem(code[q]);
        for (int b = 0; b < K; ++b) nodes[q * K + b] = c[perm[b]];
      }
    });
    TRY(upload(pool, stream, &t.inc_nodes, nodes.data(), nodes.size(), &nb));
  }
  t.h_inc_code = std::move(code);
  TRY(upload(pool, stream, &t.batch_row, batch.data(), batch.size(), &nb));
  TRY(upload(pool, stream, &t.blk_info, blk_info.data(), blk_info.size(), &nb));
  TRY(upload(pool, stream, &t.centry, centry.data(), centry.size(), &nb));
  TRY(upload(pool, stream, &t.batch_entry, batch_entry.data(), batch_entry.size(), &nb));
  for (TopoSet& ts : t.sets) {
    if (ts.k >= 10) {
      TRY(upload(pool, stream, &ts.d_conn_ho, ts.conn.data(), ts.conn.size(), &nb));
      continue;
    }
    uvector<int4> c4(std::max<int64_t>(ts.n_elem, 1));
    parallel_chunks(ts.n_elem, 65536, [&](int64_t e0, int64_t e1) {
      for (int64_t e = e0; e < e1; ++e) {
        int v[4] = {-1, -1, -1, -1};
        for (int a = 0; a < ts.k; ++a) v[a] = ts.conn[e * ts.k + a];
        c4[e] = make_int4(v[0], v[1], v[2], v[3]);
      }
    });
    TRY(upload(pool, stream, &ts.d_conn, c4.data(), c4.size(), &nb));
  }
  *out = std::move(tp);
  return SYMX_OK;
}

// Scatter map of every set (element e, local a, b -> block position), built
// on demand for symx_mesh_get_pattern.
void build_scatter(Mesh& m) {
  if (!m.h_scatter.empty()) return;
  const Topology& t = *m.topo;
  size_t total = 0;
  for (const TopoSet& s : t.sets) total += size_t(s.n_elem) * s.k * s.k;
  m.h_scatter.resize(total);
  size_t off = 0;
  for (const TopoSet& s : t.sets) {
    for (int64_t e = 0; e < s.n_elem; ++e)
      for (int a = 0; a < s.k; ++a) {
        const int32_t i = s.conn[e * s.k + a];
        const int32_t* b = t.h_col_idx.data() + t.h_row_ptr[i];
        const int32_t* en = t.h_col_idx.data() + t.h_row_ptr[i + 1];
        for (int c = 0; c < s.k; ++c)
          m.h_scatter[off++] =
              t.h_row_ptr[i] + (int32_t)(std::lower_bound(b, en, s.conn[e * s.k + c]) - b);
      }
  }
}

// Point the mesh at its topology's arrays.
static void attach_topology(Mesh& m, std::shared_ptr<Topology> tp) {
  const Topology& t = *tp;
  m.nnzb = t.nnzb;
  m.n_inc = t.n_inc;
  m.n_batch = t.n_batch;
  m.max_row_blocks = t.max_row_blocks;
  m.row_ptr = t.row_ptr;
  m.col_idx = t.col_idx;
  m.diag_pos = t.diag_pos;
  m.nnzl = t.nnzl;
  m.lrow_ptr = t.lrow_ptr;
  m.cv = t.cv;
  m.inc_ptr = t.inc_ptr;
  m.inc_code = t.inc_code;
  m.inc_nodes = t.inc_nodes;
  m.batch_row = t.batch_row;
  m.blk_info = t.blk_info;
  m.centry = t.centry;
  m.batch_entry = t.batch_entry;
  for (size_t s = 0; s < m.sets.size(); ++s) {
    m.sets[s].conn = t.sets[s].conn.data();
    m.sets[s].d_conn = t.sets[s].d_conn;
    m.sets[s].d_conn_ho = t.sets[s].d_conn_ho;
  }
  m.ho = t.ho;
  m.topo = std::move(tp);
}

// Per-mesh device data: rest positions, masses, Dirichlet flags, element
// parameters, reduction scratch.
static symx_status upload_instance(Mesh& m) {
  DevicePool* pool = m.pool;
  TRY(upload(pool, m.stream, &m.X, m.h_X.data(), m.h_X.size()));
  TRY(upload(pool, m.stream, &m.mass, m.h_mass.data(), m.h_mass.size()));
  TRY(upload(pool, m.stream, &m.fixed, m.h_fixed.data(), m.h_fixed.size()));
  std::vector<std::vector<float>> p32(m.sets.size());
  for (size_t i = 0; i < m.sets.size(); ++i) {
    SetHost& s = m.sets[i];
    p32[i].assign(s.prm.begin(), s.prm.end());
    TRY(upload(pool, m.stream, &s.d_prm64, s.prm.data(), s.prm.size()));
    TRY(upload(pool, m.stream, &s.d_prm32, p32[i].data(), p32[i].size()));
    if (kind_has_rotation(s.kind)) {
      // lagged rotations start at the identity (the rest state's rotation)
      std::vector<double> r64(size_t(s.n_elem) * 9, 0.0);
      for (int64_t e = 0; e < s.n_elem; ++e) r64[9 * e] = r64[9 * e + 4] = r64[9 * e + 8] = 1.0;
      std::vector<float> r32(r64.begin(), r64.end());
      TRY(upload(pool, m.stream, &s.d_rot64, r64.data(), r64.size()));
      TRY(upload(pool, m.stream, &s.d_rot32, r32.data(), r32.size()));
    }
  }
  TRY(upload<double>(pool, m.stream, &m.partials, nullptr, kMaxPartials));
  TRY(upload<double>(pool, m.stream, &m.scalars, nullptr, 64));
  // on the mesh's stream: a null-stream memset is not ordered with work on a
  // non-blocking stream, so the first flag read could see stale memory
  TRY(hip_check(hipMemsetAsync(m.scalars, 0, 64 * sizeof(double), m.stream), "hipMemsetAsync"));
  TRY(hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize"));
  // the non-finite flag shares the scalar array (slot 24) so the Newton driver
  // reads results and flag with one copy
  m.nonfinite = reinterpret_cast<int*>(m.scalars + 24);
  void* pin = nullptr;
  TRY(pinned_alloc(pool, &pin, 64 * sizeof(double)));
  m.pinned = static_cast<double*>(pin);
  return SYMX_OK;
}

symx_status mesh_create(const symx_mesh_desc* d, Mesh** out, DevicePool* pool,
                        TopologyCache* cache) {
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
  m->pool = pool;
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
  for (int s = 0; s < d->n_energies; ++s) TRY(validate_set(d->energies[s], m->N, false));
  int ho_kind = -1, n_same = 0;
  for (int s = 0; s < d->n_energies; ++s)
    if (ho_kind < 0 && kind_high_order(d->energies[s].kind)) ho_kind = d->energies[s].kind;
  for (int s = 0; s < d->n_energies; ++s) n_same += d->energies[s].kind == ho_kind;
  if (ho_kind >= 0 && n_same < d->n_energies) {
    set_error("a mesh with quadratic or cubic tets holds no other set");
    return SYMX_ERR_INVALID_ARG;
  }
  std::shared_ptr<Topology> topo;
  if (cache) topo = cache->find(*d, topology_hash(*d));
  if (!topo) {
    for (int s = 0; s < d->n_energies; ++s) TRY(validate_set(d->energies[s], m->N, true));
    TRY(build_topology(*d, pool, m->stream, &topo));
    if (cache) cache->insert(topo);
  }
  m->sets.resize(d->n_energies);
  std::vector<std::vector<double>> elem_mass(d->n_energies);
  for (int s = 0; s < d->n_energies; ++s)
    TRY(build_set(*m, d->energies[s], m->sets[s], elem_mass[s]));
  // lumped masses: each node sums its incidences in (set, element) order
  const Topology& t = *topo;
  m->h_mass.assign(m->N, 0.0);
  parallel_chunks(m->N, 16384, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      double mi = 0.0;
      for (int64_t q = t.h_inc_ptr[i]; q < t.h_inc_ptr[i + 1]; ++q) {
        const uint32_t c = t.h_inc_code[q];
        const std::vector<double>& em = elem_mass[inc_set(c)];
        if (em.empty()) continue;
        mi += em[inc_elem(c)] * ho_mass_share(t.sets[inc_set(c)].k, inc_local(c));
      }
      m->h_mass[i] = mi;
    }
  });
  m->total_mass = 0.0;
  for (double v : m->h_mass) m->total_mass += v;
  attach_topology(*m, std::move(topo));
  TRY(upload_instance(*m));
  return SYMX_OK;
}

// Dynamic topology (Sec. 5.2, Alg. 1's rebuild step): a set of 4-node
// elements replaced between steps.  Its couplings form the mesh's second
// block matrix (built on the device, as for contacts); its parameters and
// rest data are computed like a static set's; its lumped masses are added to
// the static sets' (static sets first, then the dynamic elements in order,
// the summation order of a mesh that held the set from the start).
symx_status dynamic_set(Mesh& m, const symx_energy_desc* d) {
  if (!d) {
    set_error("null dynamic element set");
    return SYMX_ERR_INVALID_ARG;
  }
  if (m.ho) {
    set_error("dynamic elements are not available on meshes of quadratic or cubic tets");
    return SYMX_ERR_INVALID_ARG;
  }
  if (m.contacts && m.contacts->kind < 0) {
    set_error("the mesh has contacts: contacts and dynamic elements share the second block "
              "matrix, remove the contacts first");
    return SYMX_ERR_INVALID_ARG;
  }
  if (d->kind != SYMX_SNH_TET4 && d->kind != SYMX_NH_TET4 && d->kind != SYMX_STVK_TET4 &&
      d->kind != SYMX_HINGE4) {
    set_error("dynamic elements: Stable Neo-Hookean, Neo-Hookean or StVK tets, or hinges");
    return SYMX_ERR_INVALID_ARG;
  }
  const int64_t n = d->n_elem;
  if (n < 0 || (n > 0 && !d->conn) || n >= (int64_t(1) << 26)) {
    set_error("invalid dynamic element list");
    return SYMX_ERR_INVALID_ARG;
  }
  for (int64_t i = 0; i < 4 * n; ++i)
    if (d->conn[i] < 0 || d->conn[i] >= m.N) {
      set_error("node id out of range in dynamic element " + std::to_string(i / 4));
      return SYMX_ERR_INVALID_ARG;
    }
  if (m.h_mass_static.empty()) m.h_mass_static = m.h_mass;
  SetHost s;
  std::vector<double> em;
  if (n > 0) TRY(build_set(m, *d, s, em));
  TRY(dual_set(m, n, d->conn, 1.0, 1.0, d->kind));  // n = 0 frees the set
  dev_free(m.pool, m.dyn.d_prm64);
  dev_free(m.pool, m.dyn.d_prm32);
  m.dyn = SetHost();
  if (n > 0) {
    m.dyn.kind = s.kind;
    m.dyn.k = 4;
    m.dyn.n_elem = n;
    m.dyn.uniform = s.uniform;
    m.dyn.prm = std::move(s.prm);
    std::vector<float> p32(m.dyn.prm.begin(), m.dyn.prm.end());
    TRY(upload(m.pool, m.stream, &m.dyn.d_prm64, m.dyn.prm.data(), m.dyn.prm.size()));
    TRY(upload(m.pool, m.stream, &m.dyn.d_prm32, p32.data(), p32.size()));
  }
  m.h_mass = m.h_mass_static;
  if (!em.empty())
    for (int64_t e = 0; e < n; ++e)
      for (int a = 0; a < 4; ++a) m.h_mass[d->conn[4 * e + a]] += em[e];
  m.total_mass = 0.0;
  for (double v : m.h_mass) m.total_mass += v;
  TRY(hip_check(hipMemcpyAsync(m.mass, m.h_mass.data(), m.N * sizeof(double),
                               hipMemcpyHostToDevice, m.stream),
                "hipMemcpyAsync"));
  return hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
}

void mesh_free(Mesh* m);

}  // namespace symxi
