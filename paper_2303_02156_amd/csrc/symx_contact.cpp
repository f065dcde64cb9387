// Candidate contacts of the conditional point-plane barrier: validation of the
// candidate list and the device arrays of the contact pattern (built on the
// device, symx_contact_pattern.hip) and of the per-evaluation compaction.
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
  void* dev[] = {c->tuples,    c->row_ptr,   c->col_idx, c->blk_row, c->blk_ptr,
                 c->blk_src,   c->gnode,     c->gptr,    c->gsrc,    c->gdiag,
                 c->vals32,    c->vals64,    c->flag,    c->slot,    c->act,
                 c->chunk_count, c->n_active, c->eval,   c->bkey_in, c->bkey,
                 c->bval_in,   c->gkey_in,   c->gkey,    c->gval_in, c->head,
                 c->idx,       c->row_count, c->counts,  c->sort_temp};
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
  if (!(kc > 0.0) || !(dhat > 0.0) || !std::isfinite(kc) || !std::isfinite(dhat)) {
    set_error("invalid contact list or barrier parameters");
    return SYMX_ERR_INVALID_ARG;
  }
  if (m.contacts && m.contacts->kind >= 0) {
    set_error("the mesh has a dynamic element set: contacts and dynamic elements share the "
              "second block matrix, remove the dynamic set first");
    return SYMX_ERR_INVALID_ARG;
  }
  return dual_set(m, n, tuples, kc, dhat, -1);
}

symx_status dual_set(Mesh& m, int64_t n, const int32_t* tuples, double kc, double dhat, int kind) {
  if (n < 0 || (n > 0 && !tuples) || n >= (int64_t(1) << 26)) {
    set_error("invalid tuple list");
    return SYMX_ERR_INVALID_ARG;
  }
  if (m.ho) {
    set_error("contacts and dynamic elements are not available on meshes of quadratic or cubic "
              "tets");
    return SYMX_ERR_INVALID_ARG;
  }
  for (int64_t c = 0; c < n; ++c)
    for (int a = 0; a < 4; ++a) {
      const int32_t v = tuples[4 * c + a];
      const char* what = kind < 0 ? " in contact " : " in dynamic element ";
      if (v < 0 || v >= m.N) {
        set_error(std::string("node id out of range") + what + std::to_string(c));
        return SYMX_ERR_INVALID_ARG;
      }
      for (int b = 0; b < a; ++b)
        if (tuples[4 * c + b] == v) {
          set_error(std::string("repeated node") + what + std::to_string(c));
          return SYMX_ERR_INVALID_ARG;
        }
    }
  if (m.stream)
    (void)hipStreamSynchronize(m.stream);
  else
    (void)hipDeviceSynchronize();
  if (n == 0) {
    contacts_free(m);
    return SYMX_OK;
  }
  // a list that fits the buffers of the previous one reuses them
  const bool reuse = m.contacts && m.contacts->cap >= n;
  if (!reuse) {
    contacts_free(m);
    m.contacts = new Contacts();
  }
  Contacts* c = m.contacts;
  c->kind = kind;
  c->n = n;
  c->kc = kc;
  c->dhat = dhat;
  auto build = [&]() -> symx_status {
    if (!reuse) {
      TRY_STATUS(put<int>(m, &c->tuples, nullptr, 4 * n));
      TRY_STATUS(put<uint8_t>(m, &c->flag, nullptr, n));
      TRY_STATUS(put<int>(m, &c->slot, nullptr, n));
      TRY_STATUS(put<int>(m, &c->act, nullptr, n));
      TRY_STATUS(
          put<int>(m, &c->chunk_count, nullptr, (n + kContactChunk - 1) / kContactChunk + 1));
      TRY_STATUS(put<int>(m, &c->n_active, nullptr, 1));
      TRY_STATUS(contacts_reserve_pattern(m, *c, n));
      c->cap = n;
    }
    TRY_STATUS(hip_check(hipMemcpyAsync(c->tuples, tuples, 4 * n * sizeof(int32_t),
                                        hipMemcpyHostToDevice, m.stream),
                         "hipMemcpyAsync"));
    return contacts_build_pattern(m, *c);  // ends with a stream synchronisation
  };
  const symx_status st = build();
  if (st != SYMX_OK) contacts_free(m);  // no half-built contact list stays attached
  return st;
}

}  // namespace symxi
