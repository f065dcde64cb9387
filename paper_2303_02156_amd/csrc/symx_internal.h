// Internal data structures of libsymx (host side and kernel arguments).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "symx.h"

namespace symxi {

constexpr int kMaxSets = 4;
constexpr int kRowWG = 256;         // lanes of a row-assembly workgroup
constexpr int kMaxRowBlocks = 255;  // slots per row are stored as uint8
constexpr int kRedWG = 256;         // reduction workgroup size
constexpr int kPrm = 8;             // parameter slots per element (doubles)
constexpr uint32_t kNoSlot = 0xFFu;
constexpr int kPcgHistory = 64;    // remembered PCG iteration counts
constexpr int kDinv = 6;           // values per block-Jacobi inverse: the upper triangle
                                    // (d00, d01, d02, d11, d12, d22) of the symmetric 3x3
constexpr int kIncRec = 32;        // values per incidence record (projected path)
constexpr int kQuadInc = 64;       // incidences per row batch of a quadratic-tet mesh
constexpr int kCubicInc = 32;      // incidences per row batch of a cubic-tet mesh
constexpr int kMaxElemBits = 25;   // element ids per set < 2^25

// Nodes per element of an energy kind.
__host__ __device__ constexpr int kind_nodes(int kind) {
  return kind == SYMX_STVK_TRI3  ? 3
         : kind == SYMX_SNH_TET10 ? 10
         : kind == SYMX_SNH_TET20 ? 20
                                  : 4;
}
// Higher-order tets (10 or 20 nodes), 0 for any other kind.
__host__ __device__ constexpr int kind_high_order(int kind) {
  return kind == SYMX_SNH_TET10 ? 10 : kind == SYMX_SNH_TET20 ? 20 : 0;
}

// Parameter layout per element (kPrm doubles):
//   SNH tet4:  mu, lambda (linear-elasticity Lame pair)
//   StVK tri3: mu, lambda, thickness
//   hinge4:    K0, K1, K2, K3, c = 3/(A0+A1), k_b
struct SetDev {
  int kind;
  int k;                 // nodes per element
  int64_t n_elem;
  const int4* conn;      // n_elem (unused components = -1)
  const double* prm64;   // n_elem * kPrm, or kPrm when uniform
  const float* prm32;
  int prm_stride;        // kPrm, or 0 when every element has the same parameters
  const double* rot64;   // lagged-rotation materials: n_elem x 9 (row-major R), else null
  const float* rot32;
  const int* conn_ho;    // higher-order tets: n_elem x k node ids (conn is null)
};

// Higher-order tet node orders (App. A).  Corners 0-3; edges k = (0,1),
// (1,2), (2,0), (0,3), (1,3), (2,3).  Quadratic tets (10 nodes): node 4 + k
// at the middle of edge k.  Cubic tets (20 nodes): nodes 4 + 2k and 5 + 2k on
// edge k = (i, j), a third of the way from i and from j; node 16 + c at the
// centroid of the face opposite corner c.  The element energy is unchanged
// when the corners are permuted and the other nodes follow their edges and
// faces (both quadrature rules are symmetric), so the Hessian row of any node
// comes from the row function of one node per class: node 0 (a corner, moved
// to corner 0), node 4 (an edge node: its edge moved to (0, 1) with its own
// end at 0) or node 19 (a cubic face node: the opposite corner moved to 3).
// HoPerm<K>::p[a][b] is the original local node at position b of node a's
// relabelled order.
constexpr int kTetEdge[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
template <int K>
struct HoPerm {
  int8_t p[K][K];
};
// position of node a in its relabelled order (the row function it uses)
__host__ __device__ constexpr int ho_row_pos(int K, int a) {
  return a < 4 ? 0 : (K == 20 && a >= 16) ? 19 : 4;
}
template <int K>
constexpr HoPerm<K> make_ho_perm() {
  HoPerm<K> t{};
  for (int a = 0; a < K; ++a) {
    int sig[4] = {0, 0, 0, 0};  // new corner c is original corner sig[c]
    int n = 0;
    const int last = (K == 20 && a >= 16) ? a - 16 : -1;
    if (a < 4) {
      sig[n++] = a;
    } else if (last < 0) {
      const int k = K == 10 ? a - 4 : (a - 4) / 2;
      const int own = K == 10 ? 0 : (a - 4) % 2;  // the end the node is nearer
      sig[n++] = kTetEdge[k][own];
      sig[n++] = kTetEdge[k][1 - own];
    }
    for (int c = 0; c < 4; ++c) {
      bool used = c == last;
      for (int u = 0; u < n; ++u) used = used || sig[u] == c;
      if (!used) sig[n++] = c;
    }
    if (last >= 0) sig[n++] = last;
    for (int c = 0; c < 4; ++c) t.p[a][c] = int8_t(sig[c]);
    for (int k = 0; k < 6; ++k) {
      const int u = sig[kTetEdge[k][0]], v = sig[kTetEdge[k][1]];
      for (int m = 0; m < 6; ++m) {
        const bool same = kTetEdge[m][0] == u && kTetEdge[m][1] == v;
        const bool flipped = kTetEdge[m][0] == v && kTetEdge[m][1] == u;
        if (!same && !flipped) continue;
        if (K == 10) {
          t.p[a][4 + k] = int8_t(4 + m);
        } else {
          t.p[a][4 + 2 * k] = int8_t(same ? 4 + 2 * m : 5 + 2 * m);
          t.p[a][5 + 2 * k] = int8_t(same ? 5 + 2 * m : 4 + 2 * m);
        }
      }
    }
    if (K == 20)
      for (int c = 0; c < 4; ++c) t.p[a][16 + c] = int8_t(16 + sig[c]);
  }
  return t;
}
template <int K>
constexpr bool ho_perm_valid(const HoPerm<K>& t) {
  for (int a = 0; a < K; ++a) {
    if (t.p[a][ho_row_pos(K, a)] != a) return false;
    int seen[K] = {};
    for (int b = 0; b < K; ++b) {
      if (t.p[a][b] < 0 || t.p[a][b] >= K || seen[t.p[a][b]]) return false;
      seen[t.p[a][b]] = 1;
    }
  }
  return true;
}
constexpr HoPerm<10> kTet10Perm = make_ho_perm<10>();
constexpr HoPerm<20> kTet20Perm = make_ho_perm<20>();
static_assert(ho_perm_valid(kTet10Perm) && ho_perm_valid(kTet20Perm),
              "relabelled node orders must be permutations that put node a at its row position");

// Fixed co-rotational and ARAP tets carry a lagged rotation per element.
inline bool kind_has_rotation(int kind) {
  return kind == SYMX_FCR_TET4 || kind == SYMX_ARAP_TET4;
}

struct SetsDev {
  SetDev s[kMaxSets];
  int n;
};

// Incidence code: element id (bits 0-24), local node a (25-29), set (30-31).
__host__ __device__ inline uint32_t inc_make(int set, int a, int64_t e) {
  return (uint32_t(set) << 30) | (uint32_t(a) << 25) | uint32_t(e);
}
__host__ __device__ inline int inc_set(uint32_t c) { return int(c >> 30); }
__host__ __device__ inline int inc_local(uint32_t c) { return int((c >> 25) & 31u); }
__host__ __device__ inline int inc_elem(uint32_t c) { return int(c & 0x01FFFFFFu); }

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------

// Device memory of one server: large chunks from hipMalloc, carved into
// blocks by best fit and coalesced on release, so a stream of requests does
// not call hipMalloc / hipFree (hipFree can wait for work on other streams).
// Chunks are added while the total stays within `capacity` (0: no limit; a
// request that still does not fit gets a chunk of its own) and are returned
// to the device only by the destructor.  Pinned host blocks are kept in
// size-keyed free lists.
class DevicePool {
 public:
  DevicePool(int device, size_t capacity) : device_(device), capacity_(capacity) {}
  ~DevicePool();
  DevicePool(const DevicePool&) = delete;
  DevicePool& operator=(const DevicePool&) = delete;
  void* alloc(size_t bytes);  // 256-byte aligned; null on failure
  void release(void* p);
  void* alloc_pinned(size_t bytes);
  void release_pinned(void* p);
  size_t chunk_bytes();       // device bytes held
  size_t live_bytes();        // device bytes handed out
  size_t peak_live_bytes();   // most device bytes handed out at once
 private:
  struct Chunk {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_at;  // offset -> length of each free range
  };
  using FreeKey = std::pair<Chunk*, size_t>;
  void add_free(Chunk* c, size_t off, size_t len);
  void remove_free(Chunk* c, size_t off, size_t len);
  bool add_chunk(size_t min_bytes);
  int device_;
  size_t capacity_;
  std::mutex mu_;
  std::vector<std::unique_ptr<Chunk>> chunks_;
  std::multimap<size_t, FreeKey> free_by_len_;                   // length -> (chunk, offset)
  std::unordered_map<void*, std::pair<Chunk*, size_t>> live_;  // block -> (chunk, length)
  size_t held_ = 0, live_bytes_ = 0, peak_live_ = 0;
  std::multimap<size_t, void*> pinned_free_;
  std::unordered_map<void*, size_t> pinned_live_;
};

// Through the pool when there is one, else hipMalloc / hipFree.
symx_status dev_alloc(DevicePool* pool, void** p, size_t bytes);
void dev_free(DevicePool* pool, void* p);
symx_status pinned_alloc(DevicePool* pool, void** p, size_t bytes);
void pinned_free(DevicePool* pool, void* p);

// std::vector whose resize leaves new elements uninitialised (for large
// arrays that are written in full right after, often by several threads).
template <typename T>
struct UninitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = UninitAlloc<U>;
  };
  UninitAlloc() = default;
  template <typename U>
  UninitAlloc(const UninitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <typename T>
using uvector = std::vector<T, UninitAlloc<T>>;

// Everything derived from the connectivity alone: block pattern, incidence
// lists, row batches and contribution lists (host and device copies).  Meshes
// with the same node count, energy kinds and connectivity can share one.
struct TopoSet {
  int kind = 0;
  int k = 0;
  int64_t n_elem = 0;
  std::vector<int32_t> conn;        // n_elem * k
  int4* d_conn = nullptr;           // n_elem (unused components = -1); k <= 4
  int* d_conn_ho = nullptr;         // n_elem * k; higher-order tets
};

struct Topology {
  DevicePool* pool = nullptr;
  uint64_t hash = 0;
  size_t device_bytes = 0;
  int64_t N = 0, n_inc = 0, nnzb = 0;
  int n_batch = 0, max_row_blocks = 0;
  // higher-order tets (k = 10 or 20 nodes, else 0): batches of at most
  // kQuadInc or kCubicInc incidences, k - 1 contribution entries per incidence
  // (u16 = incidence << 4 | other node j, or incidence << 5 | j when k = 20)
  int ho = 0;
  std::vector<TopoSet> sets;
  std::vector<int32_t> h_row_ptr;
  uvector<int32_t> h_col_idx;
  std::vector<int64_t> h_inc_ptr;   // N+1: incidences of each node
  uvector<uint32_t> h_inc_code;     // n_inc, in (set, element) order per node
  int* row_ptr = nullptr;           // N+1
  int* col_idx = nullptr;           // nnzb
  int* diag_pos = nullptr;          // N: index of block (i,i)
  // the solver's half storage (blocks (i, j) with j <= i, row by row): first
  // half block of each row (N+1), and for every pattern slot (i, j) the pair
  // (j, half position of block (i, j)), or (j, ~half position of its
  // transpose (j, i)) when j > i
  int64_t nnzl = 0;
  int* lrow_ptr = nullptr;
  int2* cv = nullptr;
  int* inc_ptr = nullptr;           // N+1
  uint32_t* inc_code = nullptr;     // n_inc
  int* inc_nodes = nullptr;         // higher-order tets: n_inc x k node ids of the
                                    // incidence's element in its node's relabelled order
  int* batch_row = nullptr;         // n_batch+1
  uint32_t* blk_info = nullptr;     // nnzb: off-diagonal contribution list (start << 8 | count)
  uint16_t* centry = nullptr;       // contribution entries (incidence << 2 | node b),
                                    // or incidence << 4 (5) | j for higher-order tets
  int* batch_entry = nullptr;       // n_batch+1: first entry of each batch
  ~Topology();
  bool matches(const symx_mesh_desc& d) const;  // same N, kinds and connectivity
};

// Hash of node count, energy kinds and a sample of the connectivity.
uint64_t topology_hash(const symx_mesh_desc& d);

// Topologies kept on the device between requests of a server, least recently
// used first out.  Entries not used by any mesh are "idle" and may be evicted.
class TopologyCache {
 public:
  explicit TopologyCache(size_t max_entries) : max_entries_(max_entries) {}
  std::shared_ptr<Topology> find(const symx_mesh_desc& d, uint64_t hash);
  void insert(const std::shared_ptr<Topology>& t);
  size_t idle_bytes();
  size_t evict_idle(size_t need);  // evict idle entries until `need` bytes are freed
  std::atomic<int64_t> hits{0}, misses{0};
 private:
  std::mutex mu_;
  std::list<std::shared_ptr<Topology>> lru_;  // front: most recently used
  size_t max_entries_;
};

struct SetHost {
  int kind = 0;
  int k = 0;
  int64_t n_elem = 0;
  const int32_t* conn = nullptr;    // n_elem * k (the topology's host copy)
  std::vector<double> prm;          // n_elem * kPrm or kPrm
  bool uniform = true;
  // device
  const int4* d_conn = nullptr;     // the topology's
  const int* d_conn_ho = nullptr;
  double* d_prm64 = nullptr;
  float* d_prm32 = nullptr;
  double* d_rot64 = nullptr;        // lagged rotations (FCR / ARAP sets)
  float* d_rot32 = nullptr;
};

struct Workspace;   // Newton / PCG buffers (symx_newton.cpp)
class PcgBatcher;   // batched PCG of the serving loop (symx_batch.cpp)

// Candidate contacts of the conditional point-plane barrier (node p against
// the plane of nodes t0, t1, t2) and the block pattern of their couplings: a
// second block-sparse matrix beside the mesh's own (the dual storage of the
// assembly: the mesh pattern stays, the contact pattern is rebuilt whenever
// the candidate list changes).  Blocks of inactive candidates hold zero.
constexpr int kContactVals = 12 + 144;  // gradient and Hessian of one element
constexpr int kContactChunk = 2048;     // candidates per workgroup of the compaction scan
struct Contacts {
  int kind = -1;                   // -1: contact candidates of the point-plane barrier;
                                   // else the element kind of the mesh's dynamic
                                   // element set, whose elements are the tuples
  int64_t n = 0;                   // candidate tuples
  double kc = 0.0, dhat = 0.0;
  int* tuples = nullptr;           // n x 4
  int64_t nnzb = 0;
  int* row_ptr = nullptr;          // N+1
  int* col_idx = nullptr;          // nnzb, ascending within each row
  int* blk_row = nullptr;          // nnzb
  int* blk_ptr = nullptr;          // nnzb+1 into blk_src
  int* blk_src = nullptr;          // 16 n: candidate * 16 + 4 a + b, candidate order per block
  int64_t n_gnode = 0;
  int* gnode = nullptr;            // nodes of the candidates
  int* gptr = nullptr;             // n_gnode+1 into gsrc
  int* gsrc = nullptr;             // 4 n: candidate * 4 + a, candidate order per node
  int* gdiag = nullptr;            // n_gnode: the node's diagonal block
  float* vals32 = nullptr;         // 9 x nnzb, component-major
  double* vals64 = nullptr;
  // per evaluation: activation and compaction
  uint8_t* flag = nullptr;         // n
  int* slot = nullptr;             // n: compacted index, or -1 when inactive
  int* act = nullptr;              // n: the active candidates in order
  int* chunk_count = nullptr;      // per scan chunk
  int* n_active = nullptr;         // device scalar
  void* eval = nullptr;            // n x kContactVals in the evaluation's precision
  size_t eval_bytes = 0;
  // capacities: the buffers above hold `cap` candidates (the pattern arrays
  // 16 cap blocks), vals32 / vals64 the given numbers of blocks; a new list
  // of at most cap candidates reuses them
  int64_t cap = 0;
  int64_t vals_cap32 = 0, vals_cap64 = 0;
  // scratch of the device pattern build
  uint64_t* bkey_in = nullptr;
  uint64_t* bkey = nullptr;
  int* bval_in = nullptr;
  uint32_t* gkey_in = nullptr;
  uint32_t* gkey = nullptr;
  int* gval_in = nullptr;
  int* head = nullptr;
  int* idx = nullptr;
  int* row_count = nullptr;        // N+1
  int* counts = nullptr;           // nnzb, n_gnode
  void* sort_temp = nullptr;
  size_t sort_temp_bytes = 0;
};

// Optional per-kernel timing: HIP events recorded around every launch on the
// mesh's stream, resolved lazily.
struct Profiler {
  bool on = false;
  std::vector<std::string> names;
  std::vector<std::vector<float>> dur;  // per name: device time of each launch (ms)
  struct Pending {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int id_of(const char* name);
  hipEvent_t take();
  void resolve();
  void reset();
  void reserve(size_t n);
  void destroy();
};

struct Mesh {
  int device = 0;
  hipStream_t stream = nullptr;
  DevicePool* pool = nullptr;       // null: plain hipMalloc / hipFree
  std::shared_ptr<Topology> topo;   // owns the pattern arrays below
  int64_t N = 0;
  int64_t nnzb = 0;
  int64_t n_inc = 0;
  int n_batch = 0;
  int max_row_blocks = 0;
  int ho = 0;                       // higher-order tets: 10 or 20 nodes (the topology's)
  double total_mass = 0.0;
  std::vector<SetHost> sets;
  std::vector<double> h_X, h_mass;
  std::vector<uint8_t> h_fixed;
  std::vector<int32_t> h_scatter;   // all sets concatenated

  // device data
  double* X = nullptr;              // N*3
  double* mass = nullptr;           // N
  uint8_t* fixed = nullptr;         // N
  // pattern arrays, borrowed from `topo`
  const int* row_ptr = nullptr;
  const int* col_idx = nullptr;
  const int* diag_pos = nullptr;
  int64_t nnzl = 0;                 // half storage of the solver (the topology's)
  const int* lrow_ptr = nullptr;
  const int2* cv = nullptr;
  const int* inc_ptr = nullptr;
  const uint32_t* inc_code = nullptr;
  const int* inc_nodes = nullptr;
  const int* batch_row = nullptr;
  const uint32_t* blk_info = nullptr;
  const uint16_t* centry = nullptr;
  const int* batch_entry = nullptr;
  float* vals32 = nullptr;          // 9*nnzb, component-major
  double* vals64 = nullptr;
  // the Newton solve's matrix: half storage, nine values per block (row-major)
  float* lvals32 = nullptr;         // 9*nnzl
  double* lvals64 = nullptr;
  // projected path: incidence positions (n_inc) and records (n_inc x 32)
  int* inc_pos = nullptr;
  void* inc_rows = nullptr;
  size_t inc_rows_bytes = 0;
  // reductions
  double* partials = nullptr;       // kMaxPartials
  double* scalars = nullptr;        // small device scalars
  double* pinned = nullptr;         // host pinned scalars
  int* nonfinite = nullptr;         // device flag (inside `scalars`)
  Workspace* ws = nullptr;
  Contacts* contacts = nullptr;     // conditional contact barrier or dynamic elements, or null
  SetHost dyn;                      // the dynamic element set (when contacts->kind >= 0)
  std::vector<double> h_mass_static;  // masses of the static sets (dynamic ones added on top)
  int contact_mode = SYMX_CONTACT_COMPACT;  // symx_contact_mode
  PcgBatcher* batcher = nullptr;    // serving: PCG chunks go through the server's batcher
  // dt control
  double dt_cur = 0.0, dt_nominal = 0.0;
  int successes = 0;
  int last_pcg_iters[kPcgHistory] = {};  // per Newton iteration index
  Profiler prof;

  SetsDev sets_dev() const;
  SetDev dyn_dev() const;           // the dynamic set's device view (conn = the tuples)
};

constexpr int kMaxPartials = 1 << 16;

// Event pair for one profiled launch (null events when profiling is off).
struct ProfPair {
  hipEvent_t a = nullptr, b = nullptr;
  int id = -1;
};
ProfPair prof_begin(Mesh& m, const char* name);
void prof_end(Mesh& m, const ProfPair& p);

// ---------------------------------------------------------------------------
// kernel launchers (symx_kernels.hip)
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
symx_status hip_check(hipError_t e, const char* what);

// Per-element E/g/H of one set into caller buffers (T = float | double).
symx_status launch_elem_eval(Mesh& m, int set, const double* x, int want, int precision,
                             void* E, void* g, void* H);
// In-place nearest-PSD projection of n element Hessians (dim x dim each).
symx_status launch_project(Mesh& m, int precision, void* H, int64_t n, int dim);
// Per-element E, g and filtered H of a Stable Neo-Hookean set.
symx_status launch_elem_filtered(Mesh& m, int set, const double* x, int precision, void* E,
                                 void* g, void* H);
// Row assembly: gradient (FP64, may be null) and/or Hessian (precision).
// inc_rows: projected path, read each incidence's row from the incidence
// records (kIncRec values each) instead of evaluating it.  filter: every set
// is Stable Neo-Hookean; evaluate each row with the filtered density Hessian.
// dinv (optional): the kernel also writes the inverses of the final diagonal
// blocks (N x kDinv upper triangles, precision's type).  half: the Hessian
// goes to the solver's half storage (m.lvals64 / m.lvals32) instead of the
// block arrays (m.vals64 / m.vals32).  dinv_lo (float64 only, optional): the
// linear-tet kernels also write the values and inverses rounded to float32
// (into m.lvals32 or m.vals32, and dinv_lo; the higher-order kernels do not).
symx_status launch_row_assemble(Mesh& m, const double* x, const double* x_tilde, double dt,
                                bool want_g, bool want_H, int precision, bool dirichlet,
                                const void* inc_rows, bool filter, double* g_out, void* dinv,
                                float* dinv_lo = nullptr, bool half = false);
// Incidence positions (inverse of the incidence codes), n_inc ints.
symx_status launch_incidence_positions(Mesh& m, int* inc_pos);
// Projected element rows into the incidence records (n_inc x 32, precision).
// mode 1: nearest-PSD element Hessians; 2: Stable Neo-Hookean sets filtered
// (analytic eigensystem of the density Hessian), other sets as mode 1.
symx_status launch_incidence_rows_projected(Mesh& m, const double* x, int precision, int mode,
                                            const int* inc_pos, void* rows);
// Lagged rotations of every fixed co-rotational / ARAP set: the rotation
// closest to each element's deformation gradient at positions x.
symx_status launch_lagged_rotations(Mesh& m, const double* x);
// Contact barrier at positions x: activation and compaction, then the
// active elements' derivatives into the contact matrix (want_H, precision's
// type, element Hessians projected to PSD when `project`, Dirichlet when
// `dirichlet`), their gradient rows added into g (want_g),
// and the block-Jacobi inverses of the nodes with contact blocks recomputed
// from the mesh's and the contact diagonal (dinv).  Run after the mesh's row
// assembly.
symx_status launch_contact_assemble(Mesh& m, const double* x, bool want_g, bool want_H,
                                    bool project, int precision, bool dirichlet, double* g,
                                    void* dinv);
// Replace the candidate contacts (host n x 4 node ids) and free them.
symx_status contacts_set(Mesh& m, int64_t n, const int32_t* tuples, double kc, double dhat);
void contacts_free(Mesh& m);
// The second block matrix of n 4-node tuples (contacts: kind -1; dynamic
// elements: their kind), validated and built on the device.
symx_status dual_set(Mesh& m, int64_t n, const int32_t* tuples, double kc, double dhat, int kind);
// Replace the mesh's dynamic element set (symx_mesh_set_dynamic_elements).
symx_status dynamic_set(Mesh& m, const symx_energy_desc* d);
// Device buffers of the contact pattern and of its build for cap candidates.
symx_status contacts_reserve_pattern(Mesh& m, Contacts& c, int64_t cap);
// Contact block pattern and contribution lists of the c.n candidates in
// c.tuples (on the device; the buffers reserved for at least c.n).
symx_status contacts_build_pattern(Mesh& m, Contacts& c);
// Total energy (float64 sum of per-element energies in `precision`).
symx_status launch_energy(Mesh& m, const double* x, const double* x_tilde, double dt,
                          int precision, double* E_dev);

// Vector / solver kernels (symx_kernels.hip)
symx_status launch_x_tilde(Mesh& m, const double* x, const double* v, double dt, const double g[3],
                           double* xt);
symx_status launch_dot64(Mesh& m, const double* a, const double* b, int64_t n, double* out_dev);
symx_status launch_lincomb64(Mesh& m, double* out, const double* a, const double* b,
                             double beta, int64_t n);     // out = a + beta b
symx_status launch_velocity(Mesh& m, double* v, const double* x_new, const double* x_old,
                            double inv_dt, int64_t n);
symx_status launch_check_finite(Mesh& m, const double* a, int64_t n);

// PCG buffers (device): block-Jacobi inverses (kDinv N) and the vectors of the
// iteration (3N each), float or double per the solve precision.
struct PcgBuffers {
  void* Dinv;
  void* xs;
  void* r;
  void* z;
  void* p;
  void* q;
};
symx_status launch_pcg_init(Mesh& m, int precision, const PcgBuffers& B, const double* b,
                            double tol2, int max_iter);
symx_status launch_pcg_iters(Mesh& m, int precision, const PcgBuffers& B, int k0, int n_iter);
symx_status launch_accumulate(Mesh& m, int precision, double* dx, const void* xs);

// One mesh's share of a batched PCG chunk (serving): iterations k0 .. k0+n-1
// of the solve in B, in the mesh's own arrays and grids.
struct PcgBatchItem {
  Mesh* m;
  int precision;  // SYMX_F32 or SYMX_F64 (the solve's type)
  PcgBuffers B;
  int k0, n;
};
// Device table storage of the batched launches and its pinned host staging,
// for up to `cap` meshes per (precision, contacts) group.
struct PcgBatchTables {
  void* dev = nullptr;
  void* host = nullptr;
  int cap = 0;
};
symx_status pcg_batch_tables_alloc(PcgBatchTables& t, int cap);
void pcg_batch_tables_free(PcgBatchTables& t);
// Enqueue on `stream` the items' iterations: per iteration one SpMV and one
// update launch per (precision, contacts) group, each covering all its meshes.
symx_status launch_pcg_batch(hipStream_t stream, PcgBatchTables& t, const PcgBatchItem* items,
                             int n_items);

// Gathers the PCG chunks of concurrently solving meshes and runs them as
// batched launches on its own stream (symx_batch.cpp).  run() is called by a
// mesh's Newton loop in place of its own chunk launches and returns the
// solve's stop flag and iteration count (scalars S_DONE, S_ITERS) and how many
// of the n iterations asked for the batch ran (the smallest chunk of the
// batch).  `active` reports how many requests are in flight (the batch waits
// for up to that many chunks, at most kGatherUs after the first).
class PcgBatcher {
 public:
  PcgBatcher(int device, int max_meshes, std::function<int()> active);
  ~PcgBatcher();
  PcgBatcher(const PcgBatcher&) = delete;
  PcgBatcher& operator=(const PcgBatcher&) = delete;
  symx_status run(Mesh& m, int precision, const PcgBuffers& B, int k0, int n, double S_out[2],
                  int* ran);
  int64_t batches();  // batched launches sequences so far
  int64_t chunks();   // mesh chunks they carried

 private:
  struct Job;
  void loop();
  static constexpr int kGatherUs = 50;
  int device_ = 0;
  int cap_ = 0;
  std::function<int()> active_;
  symx_status init_status_ = SYMX_OK;
  hipStream_t stream_ = nullptr;
  PcgBatchTables tables_;
  double* s_host_ = nullptr;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<Job*> pending_;
  bool stop_ = false;
  std::thread thread_;
  int64_t batches_ = 0, chunks_ = 0;
};
// r = b - A x in float64, A the solver's matrix (half storage of the mesh's
// blocks in `precision`, plus the contact matrix).
symx_status launch_residual64(Mesh& m, int precision, const double* x, const double* b, double* r);
// Rounds the float64 Hessian values of the mesh (half storage, if mesh_vals)
// and of its contacts to their float32 copies, and the n_inv float64 values of
// the block inverses dinv64 to dinv32 (if given).
symx_status launch_round_values(Mesh& m, bool mesh_vals, const double* dinv64, float* dinv32,
                                int64_t n_inv);

// Newton driver (symx_newton.cpp): the ranges symx_newton_step accepts.
bool step_params_valid(const symx_step_params& P);

}  // namespace symxi
