// Device build of the contact block pattern: the per-row buckets of the dual
// storage (Alg. 1), rebuilt on the GPU whenever the candidate list changes.
//
// Every candidate (p, t0, t1, t2) couples its four nodes pairwise: 16
// (row, col) block entries per candidate, with the contribution (candidate *
// 16 + 4a + b), and 4 (node, candidate * 4 + a) gradient entries.  A stable
// radix sort by (row, col) groups the entries of each block in candidate
// order (the order the assembly sums them in); the heads of the sorted runs
// give the blocks, a count per row and a scan give the row pointers.  Integer
// work only, so the pattern is the same on every run.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "symx_internal.h"

namespace symxi {

namespace {

__global__ __launch_bounds__(256) void k_contact_entries(int64_t n, const int* __restrict__ tuples,
                                                         uint64_t* __restrict__ bkey,
                                                         int* __restrict__ bval,
                                                         uint32_t* __restrict__ gkey,
                                                         int* __restrict__ gval) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 16 * n; i += stride) {
    const int64_t q = i >> 4;
    const int a = int(i >> 2) & 3, b = int(i) & 3;
    bkey[i] = (uint64_t(uint32_t(tuples[4 * q + a])) << 32) | uint32_t(tuples[4 * q + b]);
    bval[i] = int(i);
  }
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 4 * n; i += stride) {
    gkey[i] = uint32_t(tuples[i]);
    gval[i] = int(i);
  }
}

// head[i] = 1 where a run of equal keys starts.
template <typename K>
__global__ __launch_bounds__(256) void k_run_heads(int64_t m, const K* __restrict__ key,
                                                   int* __restrict__ head) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// Blocks from the sorted block entries; idx = inclusive scan of the heads.
__global__ __launch_bounds__(256) void k_contact_blocks_out(
    int64_t m, const uint64_t* __restrict__ key, const int* __restrict__ head,
    const int* __restrict__ idx, int* __restrict__ col_idx, int* __restrict__ blk_row,
    int* __restrict__ blk_ptr, int* __restrict__ row_count, int* __restrict__ counts) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    if (head[i]) {
      const int blk = idx[i] - 1;
      const int row = int(key[i] >> 32);
      col_idx[blk] = int(uint32_t(key[i]));
      blk_row[blk] = row;
      blk_ptr[blk] = int(i);
      atomicAdd(&row_count[row], 1);
    }
    if (i == m - 1) {
      blk_ptr[idx[i]] = int(m);
      counts[0] = idx[i];
    }
  }
}

// Gradient nodes from the sorted gradient entries.
__global__ __launch_bounds__(256) void k_contact_gnodes_out(int64_t m, const uint32_t* __restrict__ key,
                                                            const int* __restrict__ head,
                                                            const int* __restrict__ idx,
                                                            int* __restrict__ gnode,
                                                            int* __restrict__ gptr,
                                                            int* __restrict__ counts) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    if (head[i]) {
      gnode[idx[i] - 1] = int(key[i]);
      gptr[idx[i] - 1] = int(i);
    }
    if (i == m - 1) {
      gptr[idx[i]] = int(m);
      counts[1] = idx[i];
    }
  }
}

// Position of each gradient node's diagonal block (every candidate node has
// one: its (v, v) entry).
__global__ __launch_bounds__(256) void k_contact_gdiag(int64_t max_g, const int* __restrict__ counts,
                                                       const int* __restrict__ gnode,
                                                       const int* __restrict__ row_ptr,
                                                       const int* __restrict__ col_idx,
                                                       int* __restrict__ gdiag) {
  const int ng = counts[1];
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < max_g && k < ng;
       k += (int64_t)gridDim.x * 256) {
    const int v = gnode[k];
    int lo = row_ptr[v], hi = row_ptr[v + 1];
    while (lo < hi) {  // first column >= v
      const int mid = (lo + hi) >> 1;
      if (col_idx[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    gdiag[k] = lo;
  }
}

int grid_of(int64_t work) {
  const int64_t g = (work + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

#define CB_TRY(expr)              \
  do {                            \
    symx_status s_ = (expr);      \
    if (s_ != SYMX_OK) return s_; \
  } while (0)
#define CB_HIP(expr, what) CB_TRY(hip_check((expr), what))

namespace {
template <typename T>
symx_status alloc_n(Mesh& m, T** p, int64_t count) {
  void* q = nullptr;
  const symx_status st = dev_alloc(m.pool, &q, size_t(std::max<int64_t>(count, 1)) * sizeof(T));
  *p = (T*)q;
  return st;
}
}  // namespace

symx_status contacts_reserve_pattern(Mesh& m, Contacts& c, int64_t cap) {
  const int64_t mb = 16 * cap, mg = 4 * cap, N = m.N;
  // outputs (upper bounds: every entry its own block / node)
  CB_TRY(alloc_n(m, &c.row_ptr, N + 1));
  CB_TRY(alloc_n(m, &c.col_idx, mb));
  CB_TRY(alloc_n(m, &c.blk_row, mb));
  CB_TRY(alloc_n(m, &c.blk_ptr, mb + 1));
  CB_TRY(alloc_n(m, &c.blk_src, mb));
  CB_TRY(alloc_n(m, &c.gnode, mg));
  CB_TRY(alloc_n(m, &c.gptr, mg + 1));
  CB_TRY(alloc_n(m, &c.gsrc, mg));
  CB_TRY(alloc_n(m, &c.gdiag, mg));
  // scratch
  CB_TRY(alloc_n(m, &c.bkey_in, mb));
  CB_TRY(alloc_n(m, &c.bkey, mb));
  CB_TRY(alloc_n(m, &c.bval_in, mb));
  CB_TRY(alloc_n(m, &c.gkey_in, mg));
  CB_TRY(alloc_n(m, &c.gkey, mg));
  CB_TRY(alloc_n(m, &c.gval_in, mg));
  CB_TRY(alloc_n(m, &c.head, mb));
  CB_TRY(alloc_n(m, &c.idx, mb));
  CB_TRY(alloc_n(m, &c.row_count, N + 1));
  return alloc_n(m, &c.counts, 2);
}

symx_status contacts_build_pattern(Mesh& m, Contacts& c) {
  const int64_t n = c.n, mb = 16 * n, mg = 4 * n, N = m.N;
  hipStream_t s = m.stream;
  hipLaunchKernelGGL(k_contact_entries, dim3(grid_of(mb)), dim3(256), 0, s, n, c.tuples, c.bkey_in,
                     c.bval_in, c.gkey_in, c.gval_in);
  CB_HIP(hipGetLastError(), "k_contact_entries");
  // library scratch for the sorts and scans of this size
  size_t tb1 = 0, tb2 = 0, tb3 = 0, tb4 = 0;
  CB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb1, c.bkey_in, c.bkey, c.bval_in, c.blk_src,
                                            (int)mb, 0, 64, s),
         "radix sort size");
  CB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, c.gkey_in, c.gkey, c.gval_in, c.gsrc,
                                            (int)mg, 0, 32, s),
         "radix sort size");
  CB_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tb3, c.head, c.idx, (int)mb, s), "scan size");
  CB_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb4, c.row_count, c.row_ptr, (int)(N + 1), s),
         "scan size");
  const size_t tbytes = std::max(std::max(tb1, tb2), std::max(tb3, tb4));
  if (c.sort_temp_bytes < tbytes) {
    dev_free(m.pool, c.sort_temp);
    c.sort_temp = nullptr;
    c.sort_temp_bytes = 0;
    CB_TRY(dev_alloc(m.pool, &c.sort_temp, tbytes));
    c.sort_temp_bytes = tbytes;
  }
  void* temp = c.sort_temp;
  // stable radix sorts: block entries by (row, col), gradient entries by node
  size_t tb = tbytes;
  CB_HIP(hipcub::DeviceRadixSort::SortPairs(temp, tb, c.bkey_in, c.bkey, c.bval_in, c.blk_src,
                                            (int)mb, 0, 64, s),
         "radix sort");
  tb = tbytes;
  CB_HIP(hipcub::DeviceRadixSort::SortPairs(temp, tb, c.gkey_in, c.gkey, c.gval_in, c.gsrc,
                                            (int)mg, 0, 32, s),
         "radix sort");
  // blocks and row pointers
  CB_HIP(hipMemsetAsync(c.row_count, 0, (N + 1) * sizeof(int), s), "hipMemsetAsync");
  hipLaunchKernelGGL(k_run_heads<uint64_t>, dim3(grid_of(mb)), dim3(256), 0, s, mb, c.bkey, c.head);
  CB_HIP(hipGetLastError(), "k_run_heads");
  tb = tbytes;
  CB_HIP(hipcub::DeviceScan::InclusiveSum(temp, tb, c.head, c.idx, (int)mb, s), "scan");
  hipLaunchKernelGGL(k_contact_blocks_out, dim3(grid_of(mb)), dim3(256), 0, s, mb, c.bkey, c.head,
                     c.idx, c.col_idx, c.blk_row, c.blk_ptr, c.row_count, c.counts);
  CB_HIP(hipGetLastError(), "k_contact_blocks_out");
  tb = tbytes;
  CB_HIP(hipcub::DeviceScan::ExclusiveSum(temp, tb, c.row_count, c.row_ptr, (int)(N + 1), s),
         "scan");
  // gradient nodes and their diagonal blocks
  hipLaunchKernelGGL(k_run_heads<uint32_t>, dim3(grid_of(mg)), dim3(256), 0, s, mg, c.gkey, c.head);
  CB_HIP(hipGetLastError(), "k_run_heads");
  tb = tbytes;
  CB_HIP(hipcub::DeviceScan::InclusiveSum(temp, tb, c.head, c.idx, (int)mg, s), "scan");
  hipLaunchKernelGGL(k_contact_gnodes_out, dim3(grid_of(mg)), dim3(256), 0, s, mg, c.gkey, c.head,
                     c.idx, c.gnode, c.gptr, c.counts);
  CB_HIP(hipGetLastError(), "k_contact_gnodes_out");
  hipLaunchKernelGGL(k_contact_gdiag, dim3(grid_of(mg)), dim3(256), 0, s, mg, c.counts, c.gnode,
                     c.row_ptr, c.col_idx, c.gdiag);
  CB_HIP(hipGetLastError(), "k_contact_gdiag");
  int h_counts[2] = {0, 0};
  CB_HIP(hipMemcpyAsync(h_counts, c.counts, sizeof(h_counts), hipMemcpyDeviceToHost, s),
         "hipMemcpyAsync");
  CB_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  c.nnzb = h_counts[0];
  c.n_gnode = h_counts[1];
  return SYMX_OK;
}

}  // namespace symxi
