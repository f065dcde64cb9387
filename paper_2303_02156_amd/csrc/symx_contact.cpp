// Candidate contacts of the conditional point-plane barrier: the host build of
// the contact block pattern and of the contribution lists that the device
// assembly sums in candidate order.
//
// The mesh's own pattern is static; contacts appear and disappear with the
// candidate list (the dynamic topology of Sec. 5.2).  Following the dual
// storage of the paper's assembly (Alg. 1: blocks that exist are added in
// place, new ones go to per-row buckets and the matrix is rebuilt when the
// sparsity changes), the couplings of the candidates live in a second block
// matrix that is rebuilt whenever the list changes, while the mesh pattern
// and its assembly are left as they are.  Every block of a candidate is in
// the contact matrix, also the diagonal ones; inactive candidates add zero.
#include <algorithm>
#include <cmath>
#include <string>

#include "symx_internal.h"

namespace symxi {

void contacts_free(Mesh& m) {
  Contacts* c = m.contacts;
  if (!c) return;
  void* dev[] = {c->tuples, c->row_ptr, c->col_idx, c->blk_row, c->blk_ptr, c->blk_src,
                 c->gnode,  c->gptr,    c->gsrc,    c->gdiag,   c->vals32,  c->vals64,
                 c->flag,   c->slot,    c->act,     c->chunk_count, c->n_active, c->eval};
  for (void* p : dev) dev_free(m.pool, p);
  delete c;
  m.contacts = nullptr;
}

#define TRY_STATUS(expr)          \
  do {                            \
    symx_status s_ = (expr);      \
    if (s_ != SYMX_OK) return s_; \
  } while (0)

namespace {
template <typename T>
symx_status put(Mesh& m, T** dst, const T* src, size_t n) {
  void* p = nullptr;
  symx_status st = dev_alloc(m.pool, &p, std::max<size_t>(n, 1) * sizeof(T));
  *dst = static_cast<T*>(p);
  if (st != SYMX_OK || !src || n == 0) return st;
  st = hip_check(hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, m.stream),
                 "hipMemcpyAsync");
  if (st == SYMX_OK) st = hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
  return st;
}
}  // namespace

symx_status contacts_set(Mesh& m, int64_t n, const int32_t* tuples, double kc, double dhat) {
  if (n < 0 || (n > 0 && !tuples) || n >= (int64_t(1) << 26) || !(kc > 0.0) || !(dhat > 0.0) ||
      !std::isfinite(kc) || !std::isfinite(dhat)) {
    set_error("invalid contact list or barrier parameters");
    return SYMX_ERR_INVALID_ARG;
  }
  if (m.ho) {
    set_error("contacts are not available on meshes of quadratic or cubic tets");
    return SYMX_ERR_INVALID_ARG;
  }
  for (int64_t c = 0; c < n; ++c)
    for (int a = 0; a < 4; ++a) {
      const int32_t v = tuples[4 * c + a];
      if (v < 0 || v >= m.N) {
        set_error("node id out of range in contact " + std::to_string(c));
        return SYMX_ERR_INVALID_ARG;
      }
      for (int b = 0; b < a; ++b)
        if (tuples[4 * c + b] == v) {
          set_error("repeated node in contact " + std::to_string(c));
          return SYMX_ERR_INVALID_ARG;
        }
    }
  if (m.stream)
    (void)hipStreamSynchronize(m.stream);
  else
    (void)hipDeviceSynchronize();
  contacts_free(m);
  if (n == 0) return SYMX_OK;
  auto* c = new Contacts();
  m.contacts = c;
  c->n = n;
  c->kc = kc;
  c->dhat = dhat;
  // blocks: (row, col, candidate * 16 + 4 a + b) sorted by (row, col, source)
  struct Ent {
    int32_t row, col, src;
  };
  std::vector<Ent> ent(16 * n);
  for (int64_t q = 0; q < n; ++q)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        ent[16 * q + 4 * a + b] = {tuples[4 * q + a], tuples[4 * q + b], int32_t(16 * q + 4 * a + b)};
  std::sort(ent.begin(), ent.end(), [](const Ent& x, const Ent& y) {
    return x.row != y.row ? x.row < y.row : x.col != y.col ? x.col < y.col : x.src < y.src;
  });
  std::vector<int32_t> row_ptr(m.N + 1, 0), col, brow, bptr{0}, bsrc(16 * n);
  for (size_t i = 0; i < ent.size(); ++i) {
    if (i == 0 || ent[i].row != ent[i - 1].row || ent[i].col != ent[i - 1].col) {
      if (i > 0) bptr.push_back((int32_t)i);
      col.push_back(ent[i].col);
      brow.push_back(ent[i].row);
      row_ptr[ent[i].row + 1]++;
    }
    bsrc[i] = ent[i].src;
  }
  bptr.push_back((int32_t)ent.size());
  for (int64_t i = 0; i < m.N; ++i) row_ptr[i + 1] += row_ptr[i];
  c->nnzb = (int64_t)col.size();
  // gradient rows: (node, candidate * 4 + a) sorted by (node, source)
  std::vector<std::pair<int32_t, int32_t>> gent(4 * n);
  for (int64_t q = 0; q < n; ++q)
    for (int a = 0; a < 4; ++a) gent[4 * q + a] = {tuples[4 * q + a], int32_t(4 * q + a)};
  std::sort(gent.begin(), gent.end());
  std::vector<int32_t> gnode, gptr{0}, gsrc(4 * n), gdiag;
  for (size_t i = 0; i < gent.size(); ++i) {
    if (i == 0 || gent[i].first != gent[i - 1].first) {
      if (i > 0) gptr.push_back((int32_t)i);
      const int32_t v = gent[i].first;
      gnode.push_back(v);
      const auto b0 = col.begin() + row_ptr[v], b1 = col.begin() + row_ptr[v + 1];
      gdiag.push_back(row_ptr[v] + (int32_t)(std::lower_bound(b0, b1, v) - b0));
    }
    gsrc[i] = gent[i].second;
  }
  gptr.push_back((int32_t)gent.size());
  c->n_gnode = (int64_t)gnode.size();
  TRY_STATUS(put(m, &c->tuples, tuples, 4 * n));
  TRY_STATUS(put(m, &c->row_ptr, row_ptr.data(), row_ptr.size()));
  TRY_STATUS(put(m, &c->col_idx, col.data(), col.size()));
  TRY_STATUS(put(m, &c->blk_row, brow.data(), brow.size()));
  TRY_STATUS(put(m, &c->blk_ptr, bptr.data(), bptr.size()));
  TRY_STATUS(put(m, &c->blk_src, bsrc.data(), bsrc.size()));
  TRY_STATUS(put(m, &c->gnode, gnode.data(), gnode.size()));
  TRY_STATUS(put(m, &c->gptr, gptr.data(), gptr.size()));
  TRY_STATUS(put(m, &c->gsrc, gsrc.data(), gsrc.size()));
  TRY_STATUS(put(m, &c->gdiag, gdiag.data(), gdiag.size()));
  TRY_STATUS(put<uint8_t>(m, &c->flag, nullptr, n));
  TRY_STATUS(put<int>(m, &c->slot, nullptr, n));
  TRY_STATUS(put<int>(m, &c->act, nullptr, n));
  TRY_STATUS(put<int>(m, &c->chunk_count, nullptr, (n + kContactChunk - 1) / kContactChunk + 1));
  TRY_STATUS(put<int>(m, &c->n_active, nullptr, 1));
  return SYMX_OK;
}

}  // namespace symxi
