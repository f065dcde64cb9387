// Allocation-free global evaluation and assembly (symx_assemble_bsr_noalloc).
//
// The same kernels as symx_assemble_bsr, with every buffer that call would
// allocate replaced: the Hessian values go to a caller-provided array, and
// the scratch of the energy reduction (one partial sum per workgroup of the
// energy kernels, the total, the non-finite flag) lives in a static device
// array of the library, one copy per GPU, held until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress; host code
// uses only that address (the array's name is a host-side stand-in).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "symx_internal.h"

namespace symxi {

symx_status assemble(Mesh& m, const double* x, const double* xt, double dt, bool want_g,
                     bool want_H, int project, int precision, bool dirichlet, double* g_out,
                     void* dinv, float* dinv_lo);

// Partial sums: one per workgroup of each energy kernel (at most 8192 per
// energy set, four sets, plus the inertia term), then the total and the flag.
constexpr int64_t kScratchPartials = 5 * 8192;
constexpr int64_t kScratchTotal = kScratchPartials;      // the energy
constexpr int64_t kScratchFlag = kScratchPartials + 1;   // non-finite flag (int)
constexpr int64_t kScratchDoubles = kScratchPartials + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, taken once per device with that
// device current.
static symx_status scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("assemble_bsr_noalloc: device index out of range");
    return SYMX_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return hip_check(hipGetLastError(), "hipGetDevice");
    if (cur != device) {
      hipError_t e = hipSetDevice(device);
      if (e != hipSuccess) return hip_check(e, "hipSetDevice");
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      set_error("hipGetSymbolAddress(scratch) returned a null address");
      return SYMX_ERR_DEVICE;
    }
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return SYMX_OK;
}

__global__ void k_clear_flag(double* flag_slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag_slot = 0.0;
}

// The mesh's own partials, flag and value arrays, swapped for the scratch and
// the caller's array during one call, and put back on every return path.
struct SwapGuard {
  Mesh& m;
  double* partials;
  int* nonfinite;
  float* vals32;
  double* vals64;
  explicit SwapGuard(Mesh& mm)
      : m(mm), partials(mm.partials), nonfinite(mm.nonfinite), vals32(mm.vals32),
        vals64(mm.vals64) {}
  ~SwapGuard() {
    m.partials = partials;
    m.nonfinite = nonfinite;
    m.vals32 = vals32;
    m.vals64 = vals64;
  }
};

symx_status assemble_noalloc(Mesh& m, const double* x, const double* xt, double dt, uint32_t flags,
                             int precision, double* energy_host, double* grad_dev,
                             void* values_dev) {
  const bool want_g = (flags & SYMX_EVAL_GRAD) != 0;
  const bool want_H = (flags & SYMX_EVAL_HESS) != 0;
  const bool want_E = (flags & SYMX_EVAL_E) != 0;
  const int project = (flags & SYMX_PROJECT_FILTER) ? 2 : (flags & SYMX_PROJECT_PSD) ? 1 : 0;
  if (m.contacts) {
    set_error("assemble_bsr_noalloc: meshes with contacts are not supported (their buffers are "
              "allocated per candidate list)");
    return SYMX_ERR_INVALID_ARG;
  }
  if (want_H && project) {
    bool snh_only = true;
    for (const SetHost& s : m.sets) snh_only = snh_only && s.kind == SYMX_SNH_TET4;
    if (project != 2 || !snh_only) {
      set_error("assemble_bsr_noalloc: per-element projection needs a workspace of element "
                "records; only SYMX_PROJECT_FILTER on a Stable Neo-Hookean mesh is supported");
      return SYMX_ERR_INVALID_ARG;
    }
  }
  // partial sums the energy kernels will write (grid sizes as launch_energy)
  int64_t parts = 0;
  for (const SetHost& s : m.sets) parts += std::min<int64_t>(std::max<int64_t>((s.n_elem + 255) / 256, 1), 8192);
  if (xt) parts += std::min<int64_t>(std::max<int64_t>((m.N + 255) / 256, 1), 8192);
  if (want_E && parts > kScratchPartials) {
    set_error("assemble_bsr_noalloc: " + std::to_string(parts) +
              " energy partial sums exceed the scratch array (" +
              std::to_string(kScratchPartials) + ")");
    return SYMX_ERR_BUDGET;
  }
  double* sp = nullptr;
  symx_status st = scratch_address(m.device, &sp);
  if (st != SYMX_OK) return st;
  SwapGuard guard(m);
  m.partials = sp;
  m.nonfinite = reinterpret_cast<int*>(sp + kScratchFlag);
  if (want_H) {
    if (precision == SYMX_F64)
      m.vals64 = static_cast<double*>(values_dev);
    else
      m.vals32 = static_cast<float*>(values_dev);
  }
  // the flag must start at zero (a fill kernel, not a memset, so that the
  // call can be captured in a graph)
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, m.stream, sp + kScratchFlag);
  st = hip_check(hipGetLastError(), "k_clear_flag");
  if (st != SYMX_OK) return st;
  if (want_g || want_H) {
    st = assemble(m, x, xt, dt, want_g, want_H, project, precision,
                  (flags & SYMX_DIRICHLET) != 0, grad_dev, nullptr, nullptr);
    if (st != SYMX_OK) return st;
  }
  if (want_E) {
    st = launch_energy(m, x, xt, dt, precision, sp + kScratchTotal);
    if (st != SYMX_OK) return st;
  }
  // energy and flag in one copy, into the mesh's pinned host scalars
  st = hip_check(hipMemcpyAsync(m.pinned, sp + kScratchTotal, 2 * sizeof(double),
                                hipMemcpyDeviceToHost, m.stream),
                 "hipMemcpyAsync");
  if (st != SYMX_OK) return st;
  st = hip_check(hipStreamSynchronize(m.stream), "hipStreamSynchronize");
  if (st != SYMX_OK) return st;
  int flag = 0;
  std::memcpy(&flag, &m.pinned[1], sizeof(int));
  if (flag) {
    set_error("non-finite value in positions, energy or gradient");
    return SYMX_ERR_NONFINITE;
  }
  if (want_E) *energy_host = m.pinned[0];
  return SYMX_OK;
}

}  // namespace symxi
