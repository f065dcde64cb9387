// HIP kernels for gfx950: element evaluation, PSD projection, deterministic
// row assembly into 3x3 BSR, energies, and the vector kernels of the solver.
//
// Element kernels call the generated functions of symx_gen (symbolic
// derivatives of the energies of App. B and Eq. 13).  Every reduction uses a
// fixed order (per-workgroup trees plus a final pass by the last workgroup in
// a fixed order), so all results are bitwise reproducible from run to run; no
// floating-point atomics are used anywhere.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <utility>

#include "symx_generated.h"
#include "symx_internal.h"

namespace symxi {

// Launch on the mesh's stream; with profiling on, the launch carries start
// and stop events (hipExtLaunchKernelGGL), which time the kernel itself.
#define SYMX_LAUNCH(m, name, kernel, grid, block, shmem, ...)                                 \
  do {                                                                                        \
    const ProfPair pp_ = prof_begin((m), (name));                                             \
    if (pp_.a)                                                                                \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, (m).stream, pp_.a, pp_.b, 0,          \
                            __VA_ARGS__);                                                     \
    else                                                                                      \
      hipLaunchKernelGGL(kernel, grid, block, shmem, (m).stream, __VA_ARGS__);                \
    prof_end((m), pp_);                                                                       \
  } while (0)

// ---------------------------------------------------------------------------
// common helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on
// XCD i % 8).  Remap so that each XCD processes one contiguous range of work
// items: neighbouring rows share nodes, which then stay in one L2.
__device__ __forceinline__ int xcd_remap(int i, int n) {
  const int q = n >> 3, r = n & 7, x = i & 7, j = i >> 3;
  return x * q + (x < r ? x : r) + j;
}

// Reciprocal, reciprocal square root and square root of the small rotation
// solvers: the hardware approximations in float (about 1 ulp), correctly
// rounded in double.
__device__ __forceinline__ float rot_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rot_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rot_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// float64: the hardware approximation refined by one Newton step (a few ulp;
// the rotations only need c^2 + s^2 = 1 to rounding, not correctly rounded
// parameters).
__device__ __forceinline__ double rot_rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rot_rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
__device__ __forceinline__ double rot_sqrt(double x) { return sqrt(x); }

template <typename T>
__device__ __forceinline__ T ld_prm(const T* p, int stride, int64_t e, int k) {
  return p[(int64_t)stride * e + k];
}

template <typename T>
__device__ __forceinline__ const T* prm_ptr(const SetDev& S);
template <>
__device__ __forceinline__ const float* prm_ptr<float>(const SetDev& S) { return S.prm32; }
template <>
__device__ __forceinline__ const double* prm_ptr<double>(const SetDev& S) { return S.prm64; }

// Deterministic block sum of one double per thread (blockDim = 256): a fixed
// butterfly inside each 64-lane wave, then the four wave sums in order.
__device__ double block_sum_256(double v, double* sh) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Sum partials[0..n) written by an earlier kernel, in a fixed order; every
// workgroup that calls it gets the same value.  Visibility comes from the
// kernel boundary, so no fences or atomics are needed.
__device__ double sum_partials(const double* __restrict__ partials, int n, double* sh) {
  // A thread's loads are independent: eight are issued together, then added
  // in index order (the same order as one at a time, without a memory round
  // trip per partial).
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 8 * 256) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = i + k * 256 < n ? partials[i + k * 256] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
  }
  return block_sum_256(acc, sh);
}

// [valu-hash-begin row_inputs]
// ---------------------------------------------------------------------------
// element gather: node ids in relabelled order (node a first, then the other
// nodes in ascending local order), positions relative to node a
// ---------------------------------------------------------------------------
struct Relabel {
  int n[4];    // global node ids
  int loc[4];  // local indices
};

__device__ __forceinline__ Relabel relabel(int4 c, int a) {
  Relabel r;
  r.n[0] = a == 0 ? c.x : a == 1 ? c.y : a == 2 ? c.z : c.w;
  r.n[1] = a == 0 ? c.y : c.x;
  r.n[2] = a <= 1 ? c.z : c.y;
  r.n[3] = a <= 2 ? c.w : c.z;
  r.loc[0] = a;
  r.loc[1] = a == 0 ? 1 : 0;
  r.loc[2] = a <= 1 ? 2 : 1;
  r.loc[3] = a <= 2 ? 3 : 2;
  return r;
}

__device__ __forceinline__ Relabel identity_order(int4 c) {
  Relabel r;
  r.n[0] = c.x; r.n[1] = c.y; r.n[2] = c.z; r.n[3] = c.w;
  r.loc[0] = 0; r.loc[1] = 1; r.loc[2] = 2; r.loc[3] = 3;
  return r;
}

// Fill the generated function's inputs for element `e` of set S with nodes in
// order R (node R.n[0] moved to the origin; rest positions likewise).  K is the
// node count of the element, so every index into `in` is a compile-time
// constant and the array stays in registers.
template <typename T, int K>
__device__ __forceinline__ void fill_solid(const SetDev& S, int64_t e, const Relabel& R,
                                           const double* __restrict__ x,
                                           const double* __restrict__ X, T* in) {
  constexpr int rb = 3 * K;  // first rest slot
  const double* xo = x + 3 * (int64_t)R.n[0];
  const double* Xo = X + 3 * (int64_t)R.n[0];
  const double x0 = xo[0], x1 = xo[1], x2 = xo[2];
  const double X0 = Xo[0], X1 = Xo[1], X2 = Xo[2];
  in[0] = in[1] = in[2] = T(0);
  in[rb + 0] = in[rb + 1] = in[rb + 2] = T(0);
#pragma unroll
  for (int b = 1; b < K; ++b) {
    const double* xb = x + 3 * (int64_t)R.n[b];
    const double* Xb = X + 3 * (int64_t)R.n[b];
    in[3 * b + 0] = T(xb[0] - x0);
    in[3 * b + 1] = T(xb[1] - x1);
    in[3 * b + 2] = T(xb[2] - x2);
    in[rb + 3 * b + 0] = T(Xb[0] - X0);
    in[rb + 3 * b + 1] = T(Xb[1] - X1);
    in[rb + 3 * b + 2] = T(Xb[2] - X2);
  }
  const T* P = prm_ptr<T>(S);
  const int st = S.prm_stride;
  in[2 * rb + 0] = ld_prm(P, st, e, 0);
  in[2 * rb + 1] = ld_prm(P, st, e, 1);
  if (K == 3) in[2 * rb + 2] = ld_prm(P, st, e, 2);
}

template <typename T>
__device__ __forceinline__ void fill_hinge(const SetDev& S, int64_t e, const Relabel& R,
                                           const double* __restrict__ x, T* in) {
  const double* xo = x + 3 * (int64_t)R.n[0];
  const double x0 = xo[0], x1 = xo[1], x2 = xo[2];
  in[0] = in[1] = in[2] = T(0);
#pragma unroll
  for (int b = 1; b < 4; ++b) {
    const double* xb = x + 3 * (int64_t)R.n[b];
    in[3 * b + 0] = T(xb[0] - x0);
    in[3 * b + 1] = T(xb[1] - x1);
    in[3 * b + 2] = T(xb[2] - x2);
  }
  const T* P = prm_ptr<T>(S);
  const int st = S.prm_stride;
  const T K0 = ld_prm(P, st, e, 0), K1 = ld_prm(P, st, e, 1);
  const T K2 = ld_prm(P, st, e, 2), K3 = ld_prm(P, st, e, 3);
  const int a = R.loc[0];
  // weights follow the relabelled node order
  in[12] = a == 0 ? K0 : a == 1 ? K1 : a == 2 ? K2 : K3;
  in[13] = a == 0 ? K1 : K0;
  in[14] = a <= 1 ? K2 : K1;
  in[15] = a <= 2 ? K3 : K2;
  in[16] = ld_prm(P, st, e, 4);
  in[17] = ld_prm(P, st, e, 5);
}

// Lagged rotation of element e (row-major) into the 9 inputs after the
// 26-input tet layout.  Relabelling the nodes does not change F, so R is the
// same for every node order.
template <typename T>
__device__ __forceinline__ const T* rot_ptr(const SetDev& S);
template <>
__device__ __forceinline__ const float* rot_ptr<float>(const SetDev& S) { return S.rot32; }
template <>
__device__ __forceinline__ const double* rot_ptr<double>(const SetDev& S) { return S.rot64; }

// Inputs of the generated functions of kind KIND for element e, nodes in
// order R (largest layout: 35 inputs).
constexpr int kMaxIn = 35;
template <typename T, int KIND>
__device__ __forceinline__ void elem_inputs(const SetDev& S, int64_t e, const Relabel& R,
                                            const double* __restrict__ x,
                                            const double* __restrict__ X, T* in) {
  if constexpr (KIND == SYMX_STVK_TRI3) {
    fill_solid<T, 3>(S, e, R, x, X, in);
  } else if constexpr (KIND == SYMX_HINGE4) {
    fill_hinge<T>(S, e, R, x, in);
  } else {
    fill_solid<T, 4>(S, e, R, x, X, in);
    if constexpr (KIND == SYMX_FCR_TET4 || KIND == SYMX_ARAP_TET4) {
      const T* r = rot_ptr<T>(S) + 9 * e;
#pragma unroll
      for (int c = 0; c < 9; ++c) in[26 + c] = r[c];
    }
  }
}

// The generated functions of kind KIND, by evaluation level.
#define SYMX_GEN_DISPATCH(LEVEL)                                                   \
  template <typename T, int KIND>                                                 \
  __device__ __forceinline__ void gen_##LEVEL(const T* in, T* out) {              \
    if constexpr (KIND == SYMX_SNH_TET4) snh_tet4_##LEVEL<T>(in, out);            \
    else if constexpr (KIND == SYMX_STVK_TRI3) stvk_tri3_##LEVEL<T>(in, out);     \
    else if constexpr (KIND == SYMX_HINGE4) hinge4_##LEVEL<T>(in, out);           \
    else if constexpr (KIND == SYMX_NH_TET4) nh_tet4_##LEVEL<T>(in, out);         \
    else if constexpr (KIND == SYMX_STVK_TET4) stvk_tet4_##LEVEL<T>(in, out);     \
    else if constexpr (KIND == SYMX_FCR_TET4) fcr_tet4_##LEVEL<T>(in, out);       \
    else arap_tet4_##LEVEL<T>(in, out);                                           \
  }
SYMX_GEN_DISPATCH(s_E)
SYMX_GEN_DISPATCH(s_EgH)
SYMX_GEN_DISPATCH(row0_g)
SYMX_GEN_DISPATCH(row0_gHoff)
#undef SYMX_GEN_DISPATCH

// Kinds compiled into a kernel that meets elements of several sets: bit k
// set for kind k.  f(std::integral_constant<int, KIND>) runs for the
// element's kind.
constexpr uint32_t kKindsAll = 0x7Fu;
constexpr uint32_t kKindsSnh = 1u << SYMX_SNH_TET4;
constexpr uint32_t kKindsShell = (1u << SYMX_SNH_TET4) | (1u << SYMX_STVK_TRI3) | (1u << SYMX_HINGE4);
template <uint32_t KMASK, int KIND = 0, typename F>
__device__ __forceinline__ void with_kind(int kind, F&& f) {
  if constexpr (KIND < 7) {
    if constexpr ((KMASK >> KIND) & 1u) {
      if (kind == KIND) {
        f(std::integral_constant<int, KIND>{});
        return;
      }
    }
    with_kind<KMASK, KIND + 1>(kind, f);
  }
}
// [valu-hash-end row_inputs]

// ---------------------------------------------------------------------------
// lagged rotations (fixed co-rotational and ARAP tets)
// ---------------------------------------------------------------------------

// One Jacobi rotation of the symmetric 3x3 matrix a in the (P, Q) plane,
// accumulated into the columns of v: tan(phi) = t is the root of smaller
// magnitude of t^2 + 2 t cot(2 phi) - 1 = 0, cot(2 phi) = (a_QQ - a_PP) / 2a_PQ.
template <int P, int Q, typename R>
__device__ __forceinline__ void jacobi3_rotate(R (&a)[3][3], R (&v)[3][3]) {
  constexpr int Rr = 3 - P - Q;  // the third index
  const R apq = a[P][Q];
  if (apq == R(0)) return;
  const R d = a[Q][Q] - a[P][P];
  const R t = (d >= R(0) ? R(2) : R(-2)) * apq * rot_rcp(fabs(d) + rot_sqrt(d * d + R(4) * apq * apq));
  const R c = rot_rsq(R(1) + t * t), s = t * c;
  a[P][P] -= t * apq;
  a[Q][Q] += t * apq;
  a[P][Q] = a[Q][P] = R(0);
  const R arp = a[Rr][P], arq = a[Rr][Q];
  a[Rr][P] = a[P][Rr] = c * arp - s * arq;
  a[Rr][Q] = a[Q][Rr] = s * arp + c * arq;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const R vp = v[r][P], vq = v[r][Q];
    v[r][P] = c * vp - s * vq;
    v[r][Q] = s * vp + c * vq;
  }
}

template <typename R>
__device__ __forceinline__ void cross3(const R* a, const R* b, R* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Cyclic Jacobi sweeps on a symmetric 3x3 matrix until the squared
// off-diagonal falls below tol times the squared diagonal (at most 16 sweeps).
template <typename R>
__device__ __forceinline__ void jacobi3(R (&a)[3][3], R (&v)[3][3]) {
  const R tol = sizeof(R) == 4 ? R(1e-12) : R(1e-34);
  for (int sweep = 0; sweep < 16; ++sweep) {
    const R off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const R dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > tol * dia)) break;
    jacobi3_rotate<0, 1>(a, v);
    jacobi3_rotate<0, 2>(a, v);
    jacobi3_rotate<1, 2>(a, v);
  }
}

// Rotation-variant SVD F = U diag(s) V^T with U, V proper rotations and s3
// carrying the sign of det F.  F^T F = V diag(s^2) V^T by cyclic Jacobi,
// columns sorted by decreasing s^2; u1 = F v1 / |F v1|, u2 = F v2 made
// orthogonal to u1 and normalised, u3 = u1 x u2, v3 = v1 x v2, and s_k =
// u_k . F v_k.  A rank-deficient F takes any completion; F = 0 gives U = V.
template <typename R>
__device__ void svd3(const R (&F)[3][3], R (&U)[3][3], R (&s)[3], R (&V)[3][3]) {
  R a[3][3], v[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      a[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
      v[i][j] = i == j ? R(1) : R(0);
    }
  jacobi3(a, v);
  int i1 = 0, i2 = 1, i3 = 2;
  auto swap_if = [&](int& p, int& q) {
    const R lp = p == 0 ? a[0][0] : p == 1 ? a[1][1] : a[2][2];
    const R lq = q == 0 ? a[0][0] : q == 1 ? a[1][1] : a[2][2];
    if (lq > lp) {
      const int t = p;
      p = q;
      q = t;
    }
  };
  swap_if(i1, i2);
  swap_if(i1, i3);
  swap_if(i2, i3);
  R v1[3], v2[3], v3[3], u1[3], u2[3], u3[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    v1[r] = i1 == 0 ? v[r][0] : i1 == 1 ? v[r][1] : v[r][2];
    v2[r] = i2 == 0 ? v[r][0] : i2 == 1 ? v[r][1] : v[r][2];
  }
  cross3(v1, v2, v3);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    u1[r] = F[r][0] * v1[0] + F[r][1] * v1[1] + F[r][2] * v1[2];
    u2[r] = F[r][0] * v2[0] + F[r][1] * v2[1] + F[r][2] * v2[2];
  }
  const R n1 = rot_sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (!(n1 > R(0))) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      U[r][0] = V[r][0] = v1[r];
      U[r][1] = V[r][1] = v2[r];
      U[r][2] = V[r][2] = v3[r];
      s[r] = R(0);
    }
    return;
  }
  const R in1 = rot_rcp(n1);
#pragma unroll
  for (int r = 0; r < 3; ++r) u1[r] *= in1;
  const R p = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) u2[r] -= p * u1[r];
  R n2 = rot_sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  if (!(n2 > (sizeof(R) == 4 ? R(1e-30) : R(1e-300)))) {
    // rank one: any unit vector orthogonal to u1
    const R ax = fabs(u1[0]), ay = fabs(u1[1]), az = fabs(u1[2]);
    const R e[3] = {R(ax <= ay && ax <= az ? 1 : 0), R(ay < ax && ay <= az ? 1 : 0),
                    R(az < ax && az < ay ? 1 : 0)};
    cross3(u1, e, u2);
    n2 = rot_sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) u2[r] *= rot_rcp(n2);
  cross3(u1, u2, u3);
  R fv[3][3];  // F v_k
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    fv[0][r] = n1 * u1[r];
    fv[1][r] = F[r][0] * v2[0] + F[r][1] * v2[1] + F[r][2] * v2[2];
    fv[2][r] = F[r][0] * v3[0] + F[r][1] * v3[1] + F[r][2] * v3[2];
  }
  s[0] = n1;
  s[1] = u2[0] * fv[1][0] + u2[1] * fv[1][1] + u2[2] * fv[1][2];
  s[2] = u3[0] * fv[2][0] + u3[1] * fv[2][1] + u3[2] * fv[2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    U[r][0] = u1[r];
    U[r][1] = u2[r];
    U[r][2] = u3[r];
    V[r][0] = v1[r];
    V[r][1] = v2[r];
    V[r][2] = v3[r];
  }
}

// R = argmax tr(R^T F) over rotations (the rotation factor of the polar
// decomposition, with the sign of det F put on the smallest singular value):
// R = U V^T of the rotation-variant SVD, which maximises tr(R^T F) because the
// sign of det F sits on the smallest singular value.  F = 0 gives R = I.
__device__ void closest_rotation3(const double (&F)[3][3], double (&R)[3][3]) {
  double U[3][3], sv[3], V[3][3];
  svd3(F, U, sv, V);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R[i][j] = U[i][0] * V[j][0] + U[i][1] * V[j][1] + U[i][2] * V[j][2];
}

// ---------------------------------------------------------------------------
// Stable Neo-Hookean tets with the density Hessian filtered to PSD through its
// analytic eigensystem (Smith et al. 2019, for energies of I2 = |F|^2 and
// I3 = det F): with the rotation-variant SVD F = U diag(s) V^T and
// perturbations D = U Dh V^T, the nine eigenvectors of d2psi/dF2 are
//  * for each pair (i, j), k the third index, the twist Dh_ij = -Dh_ji with
//    eigenvalue 2 psi_2 + psi_3 s_k and the flip Dh_ij = Dh_ji with
//    2 psi_2 - psi_3 s_k;
//  * three scaling modes (diagonal Dh), the eigenvectors of the 3x3 block
//    2 psi_2 I + 4 psi_22 s s^T + psi_33 c c^T + psi_3 s_k off the diagonal,
//    c = (s2 s3, s1 s3, s1 s2).
// Negative eigenvalues are set to zero.  With the shape gradients b_a and
// c_a = V^T b_a, the filtered block of nodes (a, b) is vol U K_ab U^T with
// K_ab = diag(c_a) A+ diag(c_b) plus, per pair, the twist/flip terms.
// ---------------------------------------------------------------------------
template <typename R>
struct SnhFilter {
  R vol;
  R U[3][3];
  R c[4][3];      // V^T b_a
  R Ap[3][3];     // filtered scaling block
  R sp[3], dp[3]; // per pair (0,1), (0,2), (1,2): (l_twist + l_flip)/2, (l_flip - l_twist)/2
  R g[4][3];      // gradient vol P b_a
};

// R: the compute type (float in the single-precision kernels, with the
// hardware reciprocal and square root in the rotations; double otherwise).
// Edge vectors, Dm^-1 and F are formed in double.
template <typename R>
__device__ void snh_filter(const SetDev& S, int64_t e, const double* __restrict__ x,
                           const double* __restrict__ X, SnhFilter<R>& f) {
  const int4 cn = S.conn[e];
  const int nd[4] = {cn.x, cn.y, cn.z, cn.w};
  double Ds[3][3], Dm[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      Ds[r][b] = x[3 * (int64_t)nd[b + 1] + r] - x[3 * (int64_t)nd[0] + r];
      Dm[r][b] = X[3 * (int64_t)nd[b + 1] + r] - X[3 * (int64_t)nd[0] + r];
    }
  double Mi[3][3];  // adj(Dm)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int j1 = (j + 1) % 3, j2 = (j + 2) % 3, i1 = (i + 1) % 3, i2 = (i + 2) % 3;
      Mi[i][j] = Dm[j1][i1] * Dm[j2][i2] - Dm[j1][i2] * Dm[j2][i1];
    }
  const double det = Dm[0][0] * Mi[0][0] + Dm[0][1] * Mi[1][0] + Dm[0][2] * Mi[2][0];
  const double idet = 1.0 / det;
  f.vol = R(fabs(det) / 6.0);
  R B[4][3];  // shape gradients: rows of Dm^-1, b_0 = -their sum
  R F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double Fi[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Fi[j] = (Ds[i][0] * Mi[0][j] + Ds[i][1] * Mi[1][j] + Ds[i][2] * Mi[2][j]) * idet;
#pragma unroll
    for (int j = 0; j < 3; ++j) F[i][j] = R(Fi[j]);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double b1 = Mi[0][j] * idet, b2 = Mi[1][j] * idet, b3 = Mi[2][j] * idet;
    B[1][j] = R(b1);
    B[2][j] = R(b2);
    B[3][j] = R(b3);
    B[0][j] = R(-(b1 + b2 + b3));
  }
  const int st = S.prm_stride;
  const double mu = ld_prm(S.prm64, st, e, 0), lam = ld_prm(S.prm64, st, e, 1);
  const double mu_d = mu * (4.0 / 3.0), lam_d = lam + mu * (5.0 / 6.0);
  const R mu_ = R(mu_d), lam_ = R(lam_d);
  const R alpha = R(1.0 + mu_d / lam_d - mu_d / (4.0 * lam_d));
  R V[3][3], sv[3];
  svd3(F, f.U, sv, V);
  const R I2 = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
  const R J = sv[0] * sv[1] * sv[2];
  const R q = rot_rcp(I2 + R(1));
  const R p2 = R(0.5) * mu_ * (R(1) - q);
  const R p22 = R(0.5) * mu_ * q * q;
  const R p3 = lam_ * (J - alpha);
  const R p33 = lam_;
  // gradient: P = 2 psi_2 F + psi_3 cof F
  R Pm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      Pm[i][j] = R(2) * p2 * F[i][j] + p3 * (F[i1][j1] * F[i2][j2] - F[i1][j2] * F[i2][j1]);
    }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      f.g[a][i] = f.vol * (Pm[i][0] * B[a][0] + Pm[i][1] * B[a][1] + Pm[i][2] * B[a][2]);
  // c_a = V^T b_a
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int m = 0; m < 3; ++m) f.c[a][m] = V[0][m] * B[a][0] + V[1][m] * B[a][1] + V[2][m] * B[a][2];
  // scaling block, its eigensystem, the filtered block
  const R cc[3] = {sv[1] * sv[2], sv[0] * sv[2], sv[0] * sv[1]};
  R A[3][3], W[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i][j] = R(4) * p22 * sv[i] * sv[j] + p33 * cc[i] * cc[j] +
                (i == j ? R(2) * p2 : p3 * sv[3 - i - j]);
      W[i][j] = i == j ? R(1) : R(0);
    }
  jacobi3(A, W);
  const R l0 = fmax(A[0][0], R(0)), l1 = fmax(A[1][1], R(0)), l2 = fmax(A[2][2], R(0));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      f.Ap[i][j] = l0 * W[i][0] * W[j][0] + l1 * W[i][1] * W[j][1] + l2 * W[i][2] * W[j][2];
  // twist / flip of the pairs (0,1), (0,2), (1,2); the third index is 2, 1, 0
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const R sk = sv[2 - p];
    const R lt = fmax(R(2) * p2 + p3 * sk, R(0)), lf = fmax(R(2) * p2 - p3 * sk, R(0));
    f.sp[p] = R(0.5) * (lt + lf);
    f.dp[p] = R(0.5) * (lf - lt);
  }
}

// Filtered Hessian block of nodes (a, b): vol U K_ab U^T, ca = c_a, cb = c_b.
template <typename R>
__device__ __forceinline__ void snh_filter_block(const SnhFilter<R>& f, const R (&ca)[3],
                                                 const R (&cb)[3], R (&H)[3][3]) {
  R K[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[i][j] = ca[i] * f.Ap[i][j] * cb[j];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = p == 2 ? 1 : 0, j = p == 0 ? 1 : 2;
    K[i][i] += f.sp[p] * ca[j] * cb[j];
    K[j][j] += f.sp[p] * ca[i] * cb[i];
    K[i][j] += f.dp[p] * ca[j] * cb[i];
    K[j][i] += f.dp[p] * ca[i] * cb[j];
  }
  R KU[3][3];  // K U^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      KU[i][k] = K[i][0] * f.U[k][0] + K[i][1] * f.U[k][1] + K[i][2] * f.U[k][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      H[i][k] = f.vol * (f.U[i][0] * KU[0][k] + f.U[i][1] * KU[1][k] + f.U[i][2] * KU[2][k]);
}

// Filtered rows of every incidence of a Stable Neo-Hookean set into the
// incidence-ordered records (the layout of k_elem_rows_projected*).
template <typename T>
__global__ __launch_bounds__(64) void k_elem_rows_filtered(SetDev S, const double* __restrict__ x,
                                                          const double* __restrict__ X,
                                                          const int* __restrict__ inc_pos,
                                                          T* __restrict__ rows) {
  for (int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 64) {
    SnhFilter<T> f;
    snh_filter(S, e, x, X, f);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      T* rec = rows + (int64_t)inc_pos[e * 4 + a] * kIncRec;
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[i] = T(f.g[a][i]);
#pragma unroll
      for (int bp = 1; bp < 4; ++bp) {
        const int b = bp <= a ? bp - 1 : bp;
        T H[3][3];
        snh_filter_block(f, f.c[a], f.c[b], H);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = 0; k < 3; ++k) rec[3 + 9 * i + 3 * (bp - 1) + k] = T(H[i][k]);
      }
    }
  }
}

// Element-major E, gradient (n x 12) and filtered Hessian (n x 12 x 12) of a
// Stable Neo-Hookean set (the per-element interface).
template <typename T>
__global__ __launch_bounds__(64) void k_elem_filtered(SetDev S, const double* __restrict__ x,
                                                     const double* __restrict__ X,
                                                     T* __restrict__ Eo, T* __restrict__ go,
                                                     T* __restrict__ Ho) {
  for (int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 64) {
    SnhFilter<T> f;
    snh_filter(S, e, x, X, f);
    if (Eo) {
      T in[kMaxIn], out[1];
      elem_inputs<T, SYMX_SNH_TET4>(S, e, identity_order(S.conn[e]), x, X, in);
      gen_s_E<T, SYMX_SNH_TET4>(in, out);
      Eo[e] = out[0];
    }
    if (go) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) go[e * 12 + 3 * a + i] = T(f.g[a][i]);
    }
    if (Ho) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          T H[3][3];
          snh_filter_block(f, f.c[a], f.c[b], H);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) Ho[e * 144 + (3 * a + i) * 12 + 3 * b + k] = T(H[i][k]);
        }
    }
  }
}

// One lane per element: F = Ds Dm^-1 at positions x (node order of the
// connectivity), R of F row-major into rot64 and its float copy into rot32.
__global__ __launch_bounds__(256) void k_lagged_rotations(int64_t n, const int4* __restrict__ conn,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ X,
                                                          double* __restrict__ rot64,
                                                          float* __restrict__ rot32) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const int4 c = conn[e];
    const int nd[4] = {c.x, c.y, c.z, c.w};
    double Ds[3][3], Dm[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Ds[r][b] = x[3 * (int64_t)nd[b + 1] + r] - x[3 * (int64_t)nd[0] + r];
        Dm[r][b] = X[3 * (int64_t)nd[b + 1] + r] - X[3 * (int64_t)nd[0] + r];
      }
    // Dm^-1 = adj(Dm) / det(Dm)
    double Mi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3, i1 = (i + 1) % 3, i2 = (i + 2) % 3;
        Mi[i][j] = Dm[j1][i1] * Dm[j2][i2] - Dm[j1][i2] * Dm[j2][i1];
      }
    const double det = Dm[0][0] * Mi[0][0] + Dm[0][1] * Mi[1][0] + Dm[0][2] * Mi[2][0];
    double F[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        F[i][j] = (Ds[i][0] * Mi[0][j] + Ds[i][1] * Mi[1][j] + Ds[i][2] * Mi[2][j]) / det;
    double R[3][3];
    closest_rotation3(F, R);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        rot64[9 * e + 3 * i + j] = R[i][j];
        rot32[9 * e + 3 * i + j] = float(R[i][j]);
      }
  }
}

// ---------------------------------------------------------------------------
// element-wise energy (line-search level) -> partial sums
// ---------------------------------------------------------------------------
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_energy_set(SetDev S, const double* __restrict__ x,
                                                    const double* __restrict__ X,
                                                    double* __restrict__ partials,
                                                    int* __restrict__ nonfinite) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 256) {
    const Relabel R = identity_order(S.conn[e]);
    T in[kMaxIn];
    T out[1];
    elem_inputs<T, KIND>(S, e, R, x, X, in);
    gen_s_E<T, KIND>(in, out);
    acc += double(out[0]);
  }
  double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s;
    if (!isfinite(s)) *nonfinite = 1;
  }
}

__global__ __launch_bounds__(256) void k_energy_inertia(int64_t N, const double* __restrict__ x,
                                                        const double* __restrict__ xt,
                                                        const double* __restrict__ mass, double dt,
                                                        double* __restrict__ partials,
                                                        int* __restrict__ nonfinite) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    double in[8] = {x[3 * i], x[3 * i + 1], x[3 * i + 2], xt[3 * i], xt[3 * i + 1], xt[3 * i + 2],
                    mass[i], dt};
    double out[1];
    inertia_E<double>(in, out);
    acc += out[0];
  }
  double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s;
    if (!isfinite(s)) *nonfinite = 1;
  }
}


// ---------------------------------------------------------------------------
// per-element E / gradient / Hessian (low-level element interface)
// ---------------------------------------------------------------------------
template <typename T, int KIND>
__global__ __launch_bounds__(128) void k_elem_eval(SetDev S, const double* __restrict__ x,
                                                   const double* __restrict__ X, T* __restrict__ Eo,
                                                   T* __restrict__ go, T* __restrict__ Ho) {
  constexpr int K = KIND == SYMX_STVK_TRI3 ? 3 : 4;
  constexpr int D = 3 * K;
  for (int64_t e = (int64_t)blockIdx.x * 128 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 128) {
    const Relabel R = identity_order(S.conn[e]);
    T in[kMaxIn];
    T out[1 + D + D * D];
    elem_inputs<T, KIND>(S, e, R, x, X, in);
    gen_s_EgH<T, KIND>(in, out);
    if (Eo) Eo[e] = out[0];
    if (go) {
#pragma unroll
      for (int v = 0; v < D; ++v) go[e * D + v] = out[1 + v];
    }
    if (Ho) {
#pragma unroll
      for (int v = 0; v < D * D; ++v) Ho[e * D * D + v] = out[1 + D + v];
    }
  }
}

// ---------------------------------------------------------------------------
// nearest-PSD projection of element Hessians (Sec. 5.2, projection to a
// positive semi-definite matrix): H <- H - sum over negative eigenvalues of
// lambda u u^T.  One element per lane, everything in registers.
//
// Every element energy here is translation invariant, so H (1 (x) t) = 0 for
// every t and H = Q M Q^T exactly, where the columns of Q = [h_i (x) I_3] are
// an orthonormal basis of the node-space vectors orthogonal to (1, ..., 1)
// (Helmert basis: h_i = (1, ..., 1, -(i+1), 0, ...) / sqrt((i+1)(i+2)),
// i = 0..K-2) and M = Q^T H Q is (3K-3) x (3K-3).  The spectrum of H is that
// of M plus three zeros (translations), with eigenvectors u = Q w, so
// projecting M projects H.  M's upper triangle is diagonalised by cyclic
// Jacobi rotations (Golub & Van Loan, Alg. 8.4.3: one sweep visits every pair
// p < q in row order), accumulated in V.  Indices are compile-time constants
// once a sweep is unrolled.
// ---------------------------------------------------------------------------
template <int R>
__device__ constexpr int up_idx(int i, int j) {
  return i <= j ? i * R - i * (i - 1) / 2 + (j - i) : j * R - j * (j - 1) / 2 + (i - j);
}

// Helmert basis vector i (i = 0..K-2) at node a.
template <typename T>
__device__ constexpr T helmert(int i, int a) {
  return a <= i ? T(1) / sqrt(T((i + 1) * (i + 2)))
                : (a == i + 1 ? -T(i + 1) / sqrt(T((i + 1) * (i + 2))) : T(0));
}

// Reciprocal, reciprocal square root and square root for the rotation
// parameters: the hardware approximations (about 1 ulp) in single precision,
// correctly rounded operations in double precision.

// Eigenvector matrix V (R x R, row-major) of one lane: in registers, or in
// LDS with the lanes of the workgroup interleaved (entry i at i * 64 + lane).
template <typename T, int STRIDE>
struct LaneMat {
  T* p;
  __device__ __forceinline__ T& operator[](int i) const { return p[i * STRIDE]; }
};

// One Jacobi rotation zeroing a(p,q) (Golub & Van Loan, Alg. 8.4.1): the
// smaller root t of t^2 + 2 tau t - 1 = 0 with tau = (a_qq - a_pp) / (2 a_pq),
// written as t = sign(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp
// (no division by a_pq, no overflow of tau^2); c = 1 / sqrt(1 + t^2), s = t c.
template <typename T>
struct JacobiRot {
  T t, c, s, apq;
};
template <typename T, int R, int P, int Q>
__device__ __forceinline__ JacobiRot<T> jacobi_params(const T* a) {
  const T apq = a[up_idx<R>(P, Q)];
  const T app = a[up_idx<R>(P, P)], aqq = a[up_idx<R>(Q, Q)];
  const T d = aqq - app;
  // float64 takes the root as disc rsq(disc): a zero discriminant gives NaN,
  // which only arises for a_pq = 0, where t = 0 is taken
  const T disc = d * d + T(4) * apq * apq;
  const T den = fabs(d) + (sizeof(T) == 8 ? disc * rot_rsq(disc) : rot_sqrt(disc));
  const T num = d < T(0) ? T(-2) * apq : T(2) * apq;
  const T t = (apq != T(0) && den > T(0)) ? num * rot_rcp(den) : T(0);
  const T c = rot_rsq(T(1) + t * t);
  return JacobiRot<T>{t, c, t * c, apq};
}
// A <- J^T A J, V <- V J for the rotation r of the (P, Q) plane.
template <typename T, int R, int P, int Q, typename VM>
__device__ __forceinline__ void jacobi_apply(T* a, VM v, const JacobiRot<T>& r) {
  a[up_idx<R>(P, P)] -= r.t * r.apq;
  a[up_idx<R>(Q, Q)] += r.t * r.apq;
  a[up_idx<R>(P, Q)] = T(0);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k == P || k == Q) continue;
    const T akp = a[up_idx<R>(k, P)], akq = a[up_idx<R>(k, Q)];
    a[up_idx<R>(k, P)] = r.c * akp - r.s * akq;
    a[up_idx<R>(k, Q)] = r.s * akp + r.c * akq;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const T vkp = v[k * R + P], vkq = v[k * R + Q];
    v[k * R + P] = r.c * vkp - r.s * vkq;
    v[k * R + Q] = r.s * vkp + r.c * vkq;
  }
}

// Parallel (round-robin) order of the R(R-1)/2 planes: rounds of disjoint
// planes.  R odd: round r holds the pairs i < j with i + j = r (mod R), one
// index idle; R even: index R-1 meets r, the others pair as for R-1 with
// i + j = 2r (mod R-1).  Every plane appears once per sweep.
template <int R>
struct JacobiRounds {
  static constexpr int kRounds = R % 2 ? R : R - 1;
  static constexpr int kPairs = R / 2;
  int p[kRounds][kPairs], q[kRounds][kPairs];
  constexpr JacobiRounds() : p(), q() {
    const int m = R % 2 ? R : R - 1;
    for (int r = 0; r < kRounds; ++r) {
      int n = 0;
      if (R % 2 == 0) {
        p[r][n] = r;
        q[r][n] = R - 1;
        ++n;
      }
      const int target = R % 2 ? r : (2 * r) % m;
      for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j)
          if ((i + j) % m == target) {
            p[r][n] = i;
            q[r][n] = j;
            ++n;
          }
    }
  }
};

// One round: the rotations of its disjoint planes are computed from the same
// A (a rotation of one plane leaves the other planes' 2 x 2 blocks alone, so
// their parameters are independent: instruction-level parallelism) and then
// applied one after another (disjoint rotations commute).
template <typename T, int R, int RI, typename VM, int... K>
__device__ __forceinline__ void jacobi_round(T* a, VM v, std::integer_sequence<int, K...>) {
  constexpr JacobiRounds<R> tab{};
  const JacobiRot<T> rot[] = {jacobi_params<T, R, tab.p[RI][K], tab.q[RI][K]>(a)...};
  (jacobi_apply<T, R, tab.p[RI][K], tab.q[RI][K]>(a, v, rot[K]), ...);
}

template <typename T, int R, typename VM, int... RI>
__device__ __forceinline__ void jacobi_sweep(T* a, VM v, std::integer_sequence<int, RI...>) {
  (jacobi_round<T, R, RI>(a, v, std::make_integer_sequence<int, JacobiRounds<R>::kPairs>{}), ...);
}

// Cyclic (row-order) sweep: one plane after another.
template <typename T, int R, int P, int Q, typename VM>
__device__ __forceinline__ void jacobi_sweep_cyclic(T* a, VM v) {
  if constexpr (P < R - 1) {
    jacobi_apply<T, R, P, Q>(a, v, jacobi_params<T, R, P, Q>(a));
    if constexpr (Q + 1 < R)
      jacobi_sweep_cyclic<T, R, P, Q + 1>(a, v);
    else
      jacobi_sweep_cyclic<T, R, P + 1, P + 2>(a, v);
  }
}

// M = Q^T H Q, upper triangle, reduced index 3i + c (basis vector i, coord
// c), of a K-node element Hessian given entry by entry by h(p, q).
template <typename T, int K, typename HF>
__device__ __forceinline__ void reduce_hessian(HF h, T* a) {
  constexpr int R = 3 * (K - 1);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T hb[K][K];  // node block (a, b) of H for coordinates (c, d)
#pragma unroll
      for (int na = 0; na < K; ++na)
#pragma unroll
        for (int nb = 0; nb < K; ++nb) hb[na][nb] = h(3 * na + c, 3 * nb + d);
#pragma unroll
      for (int i = 0; i < K - 1; ++i)
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
          if (3 * i + c > 3 * j + d) continue;
          T m = T(0);
#pragma unroll
          for (int na = 0; na <= i + 1; ++na)
#pragma unroll
            for (int nb = 0; nb <= j + 1; ++nb)
              m += helmert<T>(i, na) * helmert<T>(j, nb) * hb[na][nb];
          a[up_idx<R>(3 * i + c, 3 * j + d)] = m;
        }
    }
}

// Jacobi sweeps on the packed upper triangle a (R x R) with V accumulated;
// stops when the off-diagonal norm is below tol times the matrix norm.
// Returns whether an eigenvalue (diagonal of a) is negative.
template <typename T, int R, typename VM>
__device__ __forceinline__ bool jacobi_eigen(T* a, VM v, int max_sweeps, T tol) {
#pragma unroll
  for (int k = 0; k < R * R; ++k) v[k] = (k % (R + 1) == 0) ? T(1) : T(0);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    T off = T(0), dia = T(0);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      dia += a[up_idx<R>(i, i)] * a[up_idx<R>(i, i)];
#pragma unroll
      for (int j = i + 1; j < R; ++j) off += a[up_idx<R>(i, j)] * a[up_idx<R>(i, j)];
    }
    if (off <= tol * tol * (dia + T(2) * off)) break;
    // float64 (latency-bound at one wave per SIMD): the parallel order; float32
    // (issue-bound) keeps the cyclic order and its lower register count
    if constexpr (sizeof(T) == 8)
      jacobi_sweep<T, R>(a, v, std::make_integer_sequence<int, JacobiRounds<R>::kRounds>{});
    else
      jacobi_sweep_cyclic<T, R, 0, 1>(a, v);
  }
  bool neg = false;
#pragma unroll
  for (int k = 0; k < R; ++k) neg |= a[up_idx<R>(k, k)] < T(0);
  return neg;
}

// u = Q w_k, the full-space eigenvector of eigenpair k of M.
template <typename T, int K, int KV, typename VM>
__device__ __forceinline__ void lift_eigenvector(VM v, T* u) {
  constexpr int R = 3 * (K - 1);
#pragma unroll
  for (int na = 0; na < K; ++na)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T s = T(0);
#pragma unroll
      for (int i = 0; i < K - 1; ++i) s += helmert<T>(i, na) * v[(3 * i + c) * R + KV];
      u[3 * na + c] = s;
    }
}

// For each negative eigenvalue lambda_k (k = KV ... R-1): f(lambda_k, u_k).
template <typename T, int K, int KV, typename VM, typename F>
__device__ __forceinline__ void for_negative_pairs(const T* a, VM v, F f) {
  constexpr int R = 3 * (K - 1);
  if constexpr (KV < R) {
    const T lam = a[up_idx<R>(KV, KV)];
    if (lam < T(0)) {
      T u[3 * K];
      lift_eigenvector<T, K, KV>(v, u);
      f(lam, u);
    }
    for_negative_pairs<T, K, KV + 1>(a, v, f);
  }
}

// In-place projection of n element Hessians (D x D, row-major, one per lane).
// K nodes per element: H is D x D with D = 3K, M is R x R with R = 3K - 3.
// vstore: null keeps V in registers, else the workgroup's LDS array of R*R*64.
template <typename T, int K, int VSTRIDE>
__device__ __forceinline__ void project_psd_lane(T* __restrict__ H, int64_t n, int max_sweeps,
                                                 T tol, T* vstore) {
  constexpr int D = 3 * K, R = 3 * (K - 1), NU = R * (R + 1) / 2;
  T vreg[VSTRIDE == 1 ? R * R : 1];
  const LaneMat<T, VSTRIDE> v{VSTRIDE == 1 ? vreg : vstore + threadIdx.x};
  for (int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 64) {
    T* He = H + e * D * D;
    T a[NU];
    reduce_hessian<T, K>([&](int p, int q) { return He[p * D + q]; }, a);
    if (!jacobi_eigen<T, R>(a, v, max_sweeps, tol)) continue;  // PSD: H stays as it is
    // H <- H - sum_k min(lambda_k, 0) u_k u_k^T, one eigenpair at a time
    for_negative_pairs<T, K, 0>(a, v, [&](T lam, const T* u) {
#pragma unroll
      for (int p = 0; p < D; ++p)
#pragma unroll
        for (int q = 0; q < D; ++q) He[p * D + q] -= lam * u[p] * u[q];
    });
  }
}

// Projected path of the global assembly: one lane per element evaluates E's
// gradient and Hessian, writes each node's row (gradient and the three
// off-diagonal blocks, in the relabelled order that the row kernel uses) to
// that incidence's record of the incidence-ordered buffer (kIncRec values per
// record, so an element's records are whole cache lines and the row kernel
// reads them contiguously), then projects the Hessian as above and subtracts
// the negative eigenpairs from the records it wrote.  The diagonal blocks are
// not stored: the row kernel forms them from the off-diagonal ones.

template <typename T, int KIND, int VSTRIDE>
__device__ __forceinline__ void elem_rows_projected(SetDev S, const double* __restrict__ x,
                                                    const double* __restrict__ X,
                                                    const int* __restrict__ inc_pos,
                                                    T* __restrict__ rows, int max_sweeps, T tol,
                                                    T* vstore) {
  constexpr int K = KIND == SYMX_STVK_TRI3 ? 3 : 4;
  constexpr int D = 3 * K, R = 3 * (K - 1), NU = R * (R + 1) / 2;
  T vreg[VSTRIDE == 1 ? R * R : 1];
  const LaneMat<T, VSTRIDE> v{VSTRIDE == 1 ? vreg : vstore + threadIdx.x};
  for (int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 64) {
    const Relabel R0 = identity_order(S.conn[e]);
    T in[kMaxIn];
    T out[1 + D + D * D];
    elem_inputs<T, KIND>(S, e, R0, x, X, in);
    gen_s_EgH<T, KIND>(in, out);
    const T* g = out + 1;
    const T* h = out + 1 + D;
    // record of incidence (e, a): g_a, then H(a_i, b_k) for b = the other
    // nodes in ascending local order (zeros for a triangle's missing node)
    T* rec[K];
#pragma unroll
    for (int na = 0; na < K; ++na) {
      rec[na] = rows + (int64_t)inc_pos[e * K + na] * kIncRec;
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[na][i] = g[3 * na + i];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int bp = 1; bp < 4; ++bp) {
          const int nb = bp <= na ? bp - 1 : bp;  // bp-th node other than na
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            rec[na][3 + 9 * i + 3 * (bp - 1) + kk] =
                nb < K ? h[(3 * na + i) * D + 3 * nb + kk] : T(0);
        }
    }
    // A hinge Hessian k_b c (K K^T) (x) I_3 (c > 0) is positive semi-definite
    // by construction: the projection leaves it as it is.
    if (KIND == SYMX_HINGE4) continue;
    T a[NU];
    reduce_hessian<T, K>([&](int p, int q) { return h[p * D + q]; }, a);
    if (!jacobi_eigen<T, R>(a, v, max_sweeps, tol)) continue;
    for_negative_pairs<T, K, 0>(a, v, [&](T lam, const T* u) {
#pragma unroll
      for (int na = 0; na < K; ++na)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int bp = 1; bp < K; ++bp) {
            const int nb = bp <= na ? bp - 1 : bp;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
              rec[na][3 + 9 * i + 3 * (bp - 1) + kk] -= lam * u[3 * na + i] * u[3 * nb + kk];
          }
    });
  }
}

template <int KIND>
__global__ __launch_bounds__(64, 2) void k_elem_rows_projected32(SetDev S, const double* x,
                                                                 const double* X,
                                                                 const int* inc_pos, float* rows,
                                                                 int max_sweeps, float tol) {
  elem_rows_projected<float, KIND, 1>(S, x, X, inc_pos, rows, max_sweeps, tol, nullptr);
}
template <int KIND>
__global__ __launch_bounds__(64) void k_elem_rows_projected64(SetDev S, const double* x,
                                                              const double* X,
                                                              const int* inc_pos, double* rows,
                                                              int max_sweeps, double tol) {
  if constexpr (KIND == SYMX_STVK_TET4) {
    // the StVK Hessian's evaluation leaves too few registers: V in LDS
    __shared__ double vs[9 * 9 * 64];
    elem_rows_projected<double, KIND, 64>(S, x, X, inc_pos, rows, max_sweeps, tol, vs);
  } else {
    elem_rows_projected<double, KIND, 1>(S, x, X, inc_pos, rows, max_sweeps, tol, nullptr);
  }
}

// inc_pos[set_first[s] + e k + a] = position of incidence (s, e, a) in the
// incidence lists (inverse of the incidence codes).
struct SetOffsets {
  int64_t first[kMaxSets];
};
__global__ __launch_bounds__(256) void k_incidence_positions(int64_t n_inc,
                                                             const uint32_t* __restrict__ code,
                                                             SetsDev sets, SetOffsets off,
                                                             int* __restrict__ inc_pos) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n_inc;
       q += (int64_t)gridDim.x * 256) {
    const uint32_t c = code[q];
    const int si = inc_set(c);
    inc_pos[off.first[si] + (int64_t)inc_elem(c) * sets.s[si].k + inc_local(c)] = (int)q;
  }
}

// Single precision fits A and V in 256 registers: two waves per SIMD.  Double
// precision keeps them in registers too (VGPRs and AGPRs, no scratch) and runs
// one wave per SIMD; V in LDS (41 KiB per 64-lane workgroup) allows only
// three waves per CU and measured slower on the assembly path.
template <int K>
__global__ __launch_bounds__(64, 2) void k_project_psd32(float* __restrict__ H, int64_t n,
                                                         int max_sweeps, float tol) {
  project_psd_lane<float, K, 1>(H, n, max_sweeps, tol, nullptr);
}
// The element-major projection (per-element interface) updates H in memory
// and would spill with V in registers: V in LDS for four-node elements.
template <int K>
__global__ __launch_bounds__(64) void k_project_psd64(double* __restrict__ H, int64_t n,
                                                      int max_sweeps, double tol) {
  if constexpr (K == 4) {
    __shared__ double vs[9 * 9 * 64];
    project_psd_lane<double, K, 64>(H, n, max_sweeps, tol, vs);
  } else {
    project_psd_lane<double, K, 1>(H, n, max_sweeps, tol, nullptr);
  }
}

// ---------------------------------------------------------------------------
// row assembly: one workgroup per batch of consecutive block rows
// ---------------------------------------------------------------------------
template <typename T>
struct RowArgs {
  SetsDev sets;
  const double* x;
  const double* X;
  const double* xt;      // x_tilde or null (no inertia)
  const double* mass;
  double inv_dt2;
  const uint8_t* fixed;  // null: no Dirichlet treatment
  const int* batch_row;
  const int* row_ptr;
  const int* col_idx;
  const int* diag_pos;
  const int* inc_ptr;
  const uint32_t* inc_code;
  const uint32_t* blk_info;
  const uint16_t* centry;
  const int* batch_entry;
  int64_t nnzb;
  T* vals;               // component-major 9 x nnzb, or null
  T* dinv;               // N x kDinv inverses of the diagonal blocks, or null
  float* vals_lo;        // null, or the values rounded to float32 (as vals)
  float* dinv_lo;        // null, or the inverses rounded to float32 (as dinv)
  // the solver's half storage (blocks (i, j) with j <= i, nine values each,
  // row-major), or null; lvals_lo its float32 copy, or null
  const int* lrow_ptr;
  int64_t nnzl;
  T* lvals;
  float* lvals_lo;
  double* g;             // N x 3
  const T* inc_rows;     // projected path: incidence records (kIncRec per incidence)
  int* nonfinite;
  const int* inc_nodes;  // higher-order tets: relabelled element node ids per incidence
};

// Gradient row of one incidence (element e seen from its local node a).
template <typename T, uint32_t KMASK>
__device__ __forceinline__ void incidence_grad(const RowArgs<T>& A, uint32_t code, T* out) {
  const int si = inc_set(code);
  const int a = inc_local(code);
  const int64_t e = inc_elem(code);
  const SetDev& S = A.sets.s[si];
  const Relabel R = relabel(S.conn[e], a);
  with_kind<KMASK>(S.kind, [&](auto kc) {
    constexpr int KIND = decltype(kc)::value;
    T in[kMaxIn];
    elem_inputs<T, KIND>(S, e, R, A.x, A.X, in);
    gen_row0_g<T, KIND>(in, out);
  });
}

// Gradient-only row assembly: one lane per incidence of the batch's rows, then
// one lane per row sums its incidences in (set, element id) order and adds
// inertia and Dirichlet.
template <typename T, uint32_t KMASK>
__global__ __launch_bounds__(kRowWG) void k_row_gradient(RowArgs<T> A) {
  __shared__ T st[3][kRowWG];
  __shared__ int s_inc[kRowWG + 1];
  const int t = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int r0 = A.batch_row[b], r1 = A.batch_row[b + 1];
  const int nrows = r1 - r0;
  const int q0 = A.inc_ptr[r0];
  for (int r = t; r <= nrows; r += kRowWG) s_inc[r] = A.inc_ptr[r0 + r] - q0;
  __syncthreads();
  const int nq = s_inc[nrows];
  if (t < nq) {
    T out[3];
    incidence_grad<T, KMASK>(A, A.inc_code[q0 + t], out);
#pragma unroll
    for (int v = 0; v < 3; ++v) st[v][t] = out[v];
  }
  __syncthreads();
  if (t < nrows) {
    const int row = r0 + t;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int q = s_inc[t]; q < s_inc[t + 1]; ++q) {
      g0 += double(st[0][q]);
      g1 += double(st[1][q]);
      g2 += double(st[2][q]);
    }
    if (A.xt) {
      const double w = A.mass[row] * A.inv_dt2;
      g0 += w * (A.x[3 * row + 0] - A.xt[3 * row + 0]);
      g1 += w * (A.x[3 * row + 1] - A.xt[3 * row + 1]);
      g2 += w * (A.x[3 * row + 2] - A.xt[3 * row + 2]);
    }
    if (A.fixed && A.fixed[row]) g0 = g1 = g2 = 0.0;
    if (!(isfinite(g0) && isfinite(g1) && isfinite(g2))) *A.nonfinite = 1;
    A.g[3 * row + 0] = g0;
    A.g[3 * row + 1] = g1;
    A.g[3 * row + 2] = g2;
  }
}

// [valu-hash-begin row_assemble]
// Inverse of a 3x3 block in float64 (identity for a singular block); the
// block-Jacobi preconditioner of the PCG.
__device__ __forceinline__ void inverse3(const double a[9], double r[9]) {
  const double c00 = a[4] * a[8] - a[5] * a[7];
  const double c01 = a[5] * a[6] - a[3] * a[8];
  const double c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (det != 0.0 && isfinite(det)) {
    const double id = 1.0 / det;
    r[0] = c00 * id;
    r[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    r[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    r[3] = c01 * id;
    r[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    r[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    r[6] = c02 * id;
    r[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    r[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  } else {
#pragma unroll
    for (int c = 0; c < 9; ++c) r[c] = (c % 4 == 0) ? 1.0 : 0.0;
  }
}

// The block-Jacobi inverse of a node's diagonal block is symmetric (so is the
// block); it is stored as its upper triangle, kDinv values, each off-diagonal
// entry the mean of the computed inverse's two (equal up to rounding).
template <typename T>
__device__ __forceinline__ void store_dinv(T* d, const double r[9]) {
  d[0] = T(r[0]);
  d[1] = T(0.5 * (r[1] + r[3]));
  d[2] = T(0.5 * (r[2] + r[6]));
  d[3] = T(r[4]);
  d[4] = T(0.5 * (r[5] + r[7]));
  d[5] = T(r[8]);
}

// Off-diagonal part of one incidence's Hessian block row (recompute path):
// out[0..2] gradient of node a, out[3 + 9 i + 3 (b-1) + k] entry (a_i, node b
// of the relabelled order, coord k) for b = 1, 2, 3 (zero for a triangle's
// missing node).
template <typename T, uint32_t KMASK>
__device__ __forceinline__ void incidence_row_off(const RowArgs<T>& A, uint32_t code, T* out) {
  const int si = inc_set(code);
  const int a = inc_local(code);
  const int64_t e = inc_elem(code);
  const SetDev& S = A.sets.s[si];
  const Relabel R = relabel(S.conn[e], a);
  with_kind<KMASK>(S.kind, [&](auto kc) {
    constexpr int KIND = decltype(kc)::value;
    T in[kMaxIn];
    elem_inputs<T, KIND>(S, e, R, A.x, A.X, in);
    if constexpr (KIND == SYMX_STVK_TRI3) {
      T o[21];
      gen_row0_gHoff<T, KIND>(in, o);
      out[0] = o[0];
      out[1] = o[1];
      out[2] = o[2];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int v = 0; v < 6; ++v) out[3 + 9 * i + v] = o[3 + 6 * i + v];
#pragma unroll
        for (int v = 6; v < 9; ++v) out[3 + 9 * i + v] = T(0);
      }
    } else {
      gen_row0_gHoff<T, KIND>(in, out);
    }
  });
}

constexpr int kRowEval = 0, kRowRecords = 1, kRowFilter = 2;

// Filtered Stable Neo-Hookean row of one incidence, in the layout of
// incidence_row_off.
template <typename T>
__device__ __forceinline__ void incidence_row_filtered(const RowArgs<T>& A, uint32_t code, T* out) {
  const int a = inc_local(code);
  SnhFilter<T> f;
  snh_filter(A.sets.s[inc_set(code)], inc_elem(code), A.x, A.X, f);
  // the lane's node first, then the others in ascending order: selected with
  // constant indices (indexing f's arrays by a would place them in scratch)
  T cr[4][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const T c0 = f.c[0][m], c1 = f.c[1][m], c2 = f.c[2][m], c3 = f.c[3][m];
    cr[0][m] = a == 0 ? c0 : a == 1 ? c1 : a == 2 ? c2 : c3;
    cr[1][m] = a == 0 ? c1 : c0;
    cr[2][m] = a <= 1 ? c2 : c1;
    cr[3][m] = a <= 2 ? c3 : c2;
    out[m] = a == 0 ? f.g[0][m] : a == 1 ? f.g[1][m] : a == 2 ? f.g[2][m] : f.g[3][m];
  }
#pragma unroll
  for (int bp = 1; bp < 4; ++bp) {
    T H[3][3];
    snh_filter_block(f, cr[0], cr[bp], H);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) out[3 + 9 * i + 3 * (bp - 1) + k] = T(H[i][k]);
  }
}

// Layout of the solver's half storage: value c of half block l.  Component-
// major (nine arrays of nnzl values) when kHalfSoA, else nine consecutive
// values per block.
constexpr bool kHalfSoA = false;
__host__ __device__ __forceinline__ int64_t half_at(int64_t l, int c, int64_t nnzl) {
  return kHalfSoA ? (int64_t)c * nnzl + l : 9 * l + c;
}

// Store the final block of row `row`, column `col` at slot `slot` of the row
// (pattern position row_ptr[row] + slot): into the component-major block
// arrays and their float32 copy, and into the solver's half storage (when
// col <= row) and its float32 copy, each when present.
template <typename T>
__device__ __forceinline__ void store_block(const RowArgs<T>& A, int row, int col, int slot,
                                            const T (&acc)[9]) {
  const int64_t p = (int64_t)A.row_ptr[row] + slot;
  if (A.vals) {
#pragma unroll
    for (int c = 0; c < 9; ++c) A.vals[(int64_t)c * A.nnzb + p] = acc[c];
  }
  if (A.vals_lo) {
#pragma unroll
    for (int c = 0; c < 9; ++c) A.vals_lo[(int64_t)c * A.nnzb + p] = float(acc[c]);
  }
  if (A.lvals && col <= row) {
    const int64_t l = (int64_t)A.lrow_ptr[row] + slot;
#pragma unroll
    for (int c = 0; c < 9; ++c) A.lvals[half_at(l, c, A.nnzl)] = acc[c];
    if (A.lvals_lo) {
#pragma unroll
      for (int c = 0; c < 9; ++c) A.lvals_lo[half_at(l, c, A.nnzl)] = float(acc[c]);
    }
  }
}

// Row assembly for translation-invariant element energies (all three kinds:
// each element Hessian row sums to zero over the nodes, and so does its
// nearest-PSD projection, which only removes directions orthogonal to the
// translations).
//  1. one lane per incidence evaluates the gradient and the off-diagonal
//     blocks of its Hessian row (in registers; the gradient to LDS);
//  2. in rounds of one or two component rows of the blocks: the incidence
//     lanes put those rows of their off-diagonal blocks in LDS, and one lane
//     per off-diagonal block sums its precomputed contribution list in
//     incidence order (the rounds keep a part of the values in LDS at a time,
//     which lets more waves share a CU);
//  3. the summed off-diagonal blocks are published to LDS;
//  4. one lane per (row, component): the elastic diagonal block is minus the
//     sum of the row's off-diagonal blocks (slot order), plus inertia; and
//     the gradient sums the row's incidences (float64, incidence order);
//  5. Dirichlet is applied and every block is written once, with the inverse
//     of each diagonal block when requested; with vals_lo, the block values
//     and inverses are also written rounded to float32 (the copy a float32
//     solve iterates on).
// SRC: where step 1 takes each incidence's row from -- kRowEval evaluates the
// generated row function, kRowRecords reads the incidence's record in the
// incidence-ordered buffer (projected path), kRowFilter evaluates the
// filtered Stable Neo-Hookean row (all sets of that kind).
// KMASK: the element kinds compiled in (kKindsSnh for the common single-
// material mesh keeps the kernel small).
// Occupancy: the float32 kernels are held to six waves per SIMD (at most 80
// VGPRs; a few values of the Stable Neo-Hookean row spill, which costs less
// than the wave lost at 83); the float64 ones run three, except the float64
// filtered kernel, held to four (128 VGPRs, a few values spilled, and the
// three-round LDS footprint), which is faster than three at 137 VGPRs.
template <typename T, bool WANT_G, int SRC, uint32_t KMASK>
__global__ __launch_bounds__(kRowWG, sizeof(T) == 8 ? (SRC == kRowFilter ? 4 : 3) : 6) void
k_row_assemble_fast(RowArgs<T> A) {
  constexpr int NV = 30;
  // Phase 2 stages two component rows of the blocks per round (two rounds)
  // where registers already hold occupancy down to what the larger LDS array
  // allows, and one row per round (three rounds) where more waves fit: the
  // records kernel (far fewer registers) and the float64 filtered one.
  constexpr int ROWS = SRC == kRowRecords || (SRC == kRowFilter && sizeof(T) == 8) ? 1 : 2;
  constexpr int ROUNDS = ROWS == 1 ? 3 : 2;
  // Component rows of the incidences' blocks, then the sums; and the
  // incidences' gradient rows.  Rows are padded by one value so that lanes
  // reading several components of one incidence (or one slot) hit distinct
  // LDS banks.
  __shared__ T st[9 * ROWS][kRowWG + 1];
  __shared__ T sg[3][kRowWG + 1];
  // batch-relative offsets (at most kRowWG) in 16 bits
  __shared__ uint16_t s_blk[kRowWG + 1];
  __shared__ uint16_t s_inc[kRowWG + 1];
  __shared__ uint16_t s_dslot[kRowWG];  // each row's diagonal block slot in the batch
  const int t = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int r0 = A.batch_row[b], r1 = A.batch_row[b + 1];
  const int nrows = r1 - r0;
  const int q0 = A.inc_ptr[r0];
  const int p0 = A.row_ptr[r0];
  for (int r = t; r <= nrows; r += kRowWG) {
    s_blk[r] = (uint16_t)(A.row_ptr[r0 + r] - p0);
    s_inc[r] = (uint16_t)(A.inc_ptr[r0 + r] - q0);
  }
  __syncthreads();
  const int nq = s_inc[nrows];
  const int np = s_blk[nrows];
  T out[NV];
  if (t < nq) {
    if constexpr (SRC == kRowRecords) {
      const T* rec = A.inc_rows + (int64_t)(q0 + t) * kIncRec;
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = rec[v];
    } else if constexpr (SRC == kRowFilter) {
      incidence_row_filtered<T>(A, A.inc_code[q0 + t], out);
    } else {
      incidence_row_off<T, KMASK>(A, A.inc_code[q0 + t], out);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) sg[v][t] = out[v];
  }
  // block lanes: row, column and the first eight contribution-list entries
  int r = 0, col = 0, cnt = 0;
  bool diag = false;
  const uint16_t* ce = nullptr;
  uint32_t w0[8];
  T acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = T(0);
  if (t < np) {
    while (s_blk[r + 1] <= t) ++r;
    col = A.col_idx[p0 + t];
    diag = (col == r0 + r);
    const uint32_t info = A.blk_info[p0 + t];
    ce = A.centry + A.batch_entry[b] + (info >> 8);
    cnt = int(info & 0xFFu);
#pragma unroll
    for (int k = 0; k < 8; ++k) w0[k] = k < cnt ? uint32_t(ce[k]) : 0u;
  }
  // The loads of phases 4 and 5 (masses, positions, x_tilde and Dirichlet
  // flags for the lane's first phase-4 item; the Dirichlet flags of the
  // lane's block) are issued now, so that they arrive during phase 2 instead
  // of after the barriers that precede their use.
  const int n4 = (WANT_G ? 12 : 9) * nrows;
  double pf_m = 0.0, pf_x = 0.0, pf_xt = 0.0;
  bool pf_fixed = false;
  if (t < n4) {
    if (t < 9 * nrows) {
      const int rr = t / 9, c = t - 9 * rr;
      if (A.xt && (c % 4) == 0) pf_m = A.mass[r0 + rr];
    } else {
      const int jj = t - 9 * nrows;
      const int rr = jj / 3, c = jj - 3 * rr;
      const int row = r0 + rr;
      if (A.xt) {
        pf_m = A.mass[row];
        pf_x = A.x[3 * row + c];
        pf_xt = A.xt[3 * row + c];
      }
      pf_fixed = A.fixed && A.fixed[row];
    }
  }
  const bool blk_fixed = t < np && A.fixed && (A.fixed[r0 + r] | A.fixed[col]);
  // phase 2: component rows [i0, i1) of the blocks per round
#pragma unroll
  for (int round = 0; round < ROUNDS; ++round) {
    const int i0 = ROWS * round, i1 = i0 + ROWS < 3 ? i0 + ROWS : 3;
    if (t < nq) {
#pragma unroll
      for (int i = i0; i < i1; ++i)
#pragma unroll
        for (int v = 0; v < 9; ++v) st[9 * (i - i0) + v][t] = out[3 + 9 * i + v];
    }
    __syncthreads();
    if (t < np) {
      // up to eight list entries are summed from registers, later ones are
      // loaded eight at a time; all in list order
      for (int j0 = 0; j0 < cnt; j0 += 8) {
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          w[k] = j0 == 0 ? w0[k] : (j0 + k < cnt ? uint32_t(ce[j0 + k]) : 0u);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (j0 + k < cnt) {
            const int q = int(w[k] >> 2);
            const int bb = int(w[k] & 3u) - 1;
#pragma unroll
            for (int i = i0; i < i1; ++i)
#pragma unroll
              for (int kk = 0; kk < 3; ++kk)
                acc[3 * i + kk] += st[9 * (i - i0) + 3 * bb + kk][q];
          }
        }
      }
    }
    __syncthreads();
  }
  // phase 3: publish the off-diagonal blocks (and each row's diagonal slot)
  if (t < np) {
#pragma unroll
    for (int c = 0; c < 9; ++c) st[c][t] = acc[c];
    if (diag) s_dslot[r] = (uint16_t)t;
  }
  __syncthreads();
  // phase 4: one lane per (row, component) of the elastic diagonal blocks
  // (minus the sum of the row's off-diagonal blocks, in slot order; the
  // diagonal slot still holds zero) and per (row, component) of the
  // gradient (incidences in order, float64)
  for (int j = t; j < n4; j += kRowWG) {
    const bool first = j == t;  // the item whose loads were issued before phase 2
    if (j < 9 * nrows) {
      const int rr = j / 9, c = j - 9 * rr;
      // LDS reads in groups of eight, added in slot order
      T sum = T(0);
      const int sl1 = s_blk[rr + 1];
      for (int sl = s_blk[rr]; sl < sl1; sl += 8) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = sl + k < sl1 ? st[c][sl + k] : T(0);
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (sl + k < sl1) sum += v[k];
      }
      T dv = -sum;
      if (A.xt && (c % 4) == 0) dv += T((first ? pf_m : A.mass[r0 + rr]) * A.inv_dt2);
      st[c][s_dslot[rr]] = dv;
    } else {
      const int jj = j - 9 * nrows;
      const int rr = jj / 3, c = jj - 3 * rr;
      const int row = r0 + rr;
      double g = 0.0;
      const int q1 = s_inc[rr + 1];
      for (int q = s_inc[rr]; q < q1; q += 8) {  // as above, incidence order
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = q + k < q1 ? sg[c][q + k] : T(0);
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (q + k < q1) g += double(v[k]);
      }
      if (A.xt) {
        if (first)
          g += pf_m * A.inv_dt2 * (pf_x - pf_xt);
        else
          g += A.mass[row] * A.inv_dt2 * (A.x[3 * row + c] - A.xt[3 * row + c]);
      }
      if (first ? pf_fixed : (A.fixed && A.fixed[row])) g = 0.0;
      if (!isfinite(g)) *A.nonfinite = 1;
      A.g[3 * row + c] = g;
    }
  }
  __syncthreads();
  // phase 5: Dirichlet, write every block once, block-Jacobi inverses
  if (t < np) {
    const int row = r0 + r;
    if (diag) {
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] = st[c][t];
    }
    if (blk_fixed) {
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] = (diag && (c % 4) == 0) ? T(1) : T(0);
    }
    store_block(A, row, col, t - s_blk[r], acc);
    if (diag && A.dinv) {
      double a[9], ri[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) a[c] = double(acc[c]);
      inverse3(a, ri);
      store_dinv(A.dinv + kDinv * (int64_t)row, ri);
      if (A.dinv_lo) store_dinv(A.dinv_lo + kDinv * (int64_t)row, ri);
    }
  }
}

// [valu-hash-end row_assemble]

// ---------------------------------------------------------------------------
// higher-order tets (Eq. 12): the element energy is a sum over quadrature
// points of one generated function, called with each point's weight and
// reference coordinates (Sec. 5.2, fixed value summation)
// ---------------------------------------------------------------------------
// Quadratic tets: the symmetric 4-point rule of degree 2 (Hammer, Marlowe and
// Stroud 1956); point q has barycentric coordinate a at corner q and b at the
// others, a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20, weight 1/24.
// Cubic tets: Keast's symmetric 11-point rule of degree 4: the centroid with
// weight -74/5625; four points with 11/14 at one corner and 1/14 at the
// others, weight 343/45000; six points with c at two corners and d at the
// other two, c, d = (1 +- sqrt(5/14))/4, weight 56/2250.  The weights of both
// rules sum to the reference volume 1/6; xi = (L1, L2, L3).
constexpr double kSqrt5 = 2.2360679774997896964;
constexpr double kQuadA = (5.0 + 3.0 * kSqrt5) / 20.0;
constexpr double kQuadB = (5.0 - kSqrt5) / 20.0;
constexpr double kSqrt5over14 = 0.59761430466719681998;
constexpr double kKeastC = (1.0 + kSqrt5over14) / 4.0;
constexpr double kKeastD = (1.0 - kSqrt5over14) / 4.0;

struct QuadRule {
  double w[11];
  double xi[11][3];
};
constexpr QuadRule make_rule(int K) {
  QuadRule r{};
  auto put = [&r](int q, double w, const double L[4]) {
    r.w[q] = w;
    for (int k = 0; k < 3; ++k) r.xi[q][k] = L[k + 1];
  };
  if (K == 10) {
    for (int q = 0; q < 4; ++q) {
      double L[4] = {kQuadB, kQuadB, kQuadB, kQuadB};
      L[q] = kQuadA;
      put(q, 1.0 / 24.0, L);
    }
    return r;
  }
  const double Lc[4] = {0.25, 0.25, 0.25, 0.25};
  put(0, -74.0 / 5625.0, Lc);
  for (int i = 0; i < 4; ++i) {
    double L[4] = {1.0 / 14.0, 1.0 / 14.0, 1.0 / 14.0, 1.0 / 14.0};
    L[i] = 11.0 / 14.0;
    put(1 + i, 343.0 / 45000.0, L);
  }
  int q = 5;
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      double L[4] = {kKeastD, kKeastD, kKeastD, kKeastD};
      L[i] = L[j] = kKeastC;
      put(q++, 56.0 / 2250.0, L);
    }
  return r;
}

__constant__ HoPerm<10> c_perm10 = make_ho_perm<10>();
__constant__ HoPerm<20> c_perm20 = make_ho_perm<20>();
__constant__ QuadRule c_rule10 = make_rule(10);
__constant__ QuadRule c_rule20 = make_rule(20);

// Per-order data: quadrature points, incidences per row batch, the shift of
// the incidence in a contribution entry, the number of LDS accumulators the
// row kernel sums the points into (two for the 11-point rule: half the
// rounds), and the generated functions (one row function per node class:
// corner, edge node, face node).
template <int K>
struct HoTet;
template <>
struct HoTet<10> {
  static constexpr int kPts = 4, kCap = kQuadInc, kShift = 4, kAcc = 1;
  __device__ static const int8_t* perm(int a) { return c_perm10.p[a]; }
  __device__ static const QuadRule& rule() { return c_rule10; }
  template <typename T>
  __device__ static void energy(const T* in, T* out) { snh_tet10_s_E<T>(in, out); }
  template <typename T, bool H>
  __device__ static void row(int a, const T* in, T* out) {
    if (H) {
      if (a < 4) snh_tet10_row0_gHoff<T>(in, out);
      else snh_tet10_row4_gHoff<T>(in, out);
    } else {
      if (a < 4) snh_tet10_row0_g<T>(in, out);
      else snh_tet10_row4_g<T>(in, out);
    }
  }
  // the row in one part
  template <typename T>
  static constexpr int parts() { return 1; }
  static constexpr int part_lo(int k) { return k == 0 ? 0 : 9; }
  template <typename T, int PART>
  __device__ static void row_part(int a, const T* in, T* out) { row<T, true>(a, in, out); }
};
template <>
struct HoTet<20> {
  static constexpr int kPts = 11, kCap = kCubicInc, kShift = 5, kAcc = 2;
  __device__ static const int8_t* perm(int a) { return c_perm20.p[a]; }
  __device__ static const QuadRule& rule() { return c_rule20; }
  template <typename T>
  __device__ static void energy(const T* in, T* out) { snh_tet20_s_E<T>(in, out); }
  template <typename T, bool H>
  __device__ static void row(int a, const T* in, T* out) {
    if (H) {
      if (a < 4) snh_tet20_row0_gHoff<T>(in, out);
      else if (a < 16) snh_tet20_row4_gHoff<T>(in, out);
      else snh_tet20_row19_gHoff<T>(in, out);
    } else {
      if (a < 4) snh_tet20_row0_g<T>(in, out);
      else if (a < 16) snh_tet20_row4_g<T>(in, out);
      else snh_tet20_row19_g<T>(in, out);
    }
  }
  // float64: the row in three parts (gradient and the blocks of the other
  // nodes 0-6; 7-12; 13-18), each generated on its own, so that no lane
  // holds the 174 values of a whole row (which spilled 740 B per lane to
  // scratch: 2.40 -> 2.13 ms on the cubic box).  Float32 keeps the whole row
  // (the parts repeat the row's common part three times: 0.86 -> 1.12 ms).
  template <typename T>
  static constexpr int parts() { return sizeof(T) == 8 ? 3 : 1; }
  static constexpr int part_lo(int k) { return k == 0 ? 0 : k == 1 ? 7 : k == 2 ? 13 : 19; }
  template <typename T, int PART>
  __device__ static void row_part(int a, const T* in, T* out) {
    if constexpr (PART == 0) {
      if (a < 4) snh_tet20_row0_gHoff_p0<T>(in, out);
      else if (a < 16) snh_tet20_row4_gHoff_p0<T>(in, out);
      else snh_tet20_row19_gHoff_p0<T>(in, out);
    } else if constexpr (PART == 1) {
      if (a < 4) snh_tet20_row0_gHoff_p1<T>(in, out);
      else if (a < 16) snh_tet20_row4_gHoff_p1<T>(in, out);
      else snh_tet20_row19_gHoff_p1<T>(in, out);
    } else {
      if (a < 4) snh_tet20_row0_gHoff_p2<T>(in, out);
      else if (a < 16) snh_tet20_row4_gHoff_p2<T>(in, out);
      else snh_tet20_row19_gHoff_p2<T>(in, out);
    }
  }
};

// Inputs 0..6K+1 of the per-point function for element e whose node ids, in
// the evaluation order, are ids[0..K): positions and rest positions relative
// to the first node (a corner), then mu and lambda.  All positions are loaded
// before they are used, so the loads are in flight together.
template <int K, typename T>
__device__ __forceinline__ void fill_ho_ids(const SetDev& S, int64_t e, const int* ids,
                                            const double* __restrict__ x,
                                            const double* __restrict__ X, T* in) {
  double px[3 * K], pX[3 * K];
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int64_t n = ids[b];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      px[3 * b + i] = x[3 * n + i];
      pX[3 * b + i] = X[3 * n + i];
    }
  }
  // a compiler barrier: every position load above is issued before the first
  // use below (otherwise the loads are interleaved with their uses and each
  // node costs a memory round trip)
  __asm__ volatile("" ::: "memory");
#pragma unroll
  for (int b = 0; b < K; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      in[3 * b + i] = T(px[3 * b + i] - px[i]);
      in[3 * K + 3 * b + i] = T(pX[3 * b + i] - pX[i]);
    }
  const T* P = prm_ptr<T>(S);
  in[6 * K] = ld_prm(P, S.prm_stride, e, 0);
  in[6 * K + 1] = ld_prm(P, S.prm_stride, e, 1);
}

// The same for the element's node ids c[0..K) taken in the order perm.
template <int K, typename T>
__device__ __forceinline__ void fill_ho(const SetDev& S, int64_t e, const int* c,
                                        const int8_t* perm, const double* __restrict__ x,
                                        const double* __restrict__ X, T* in) {
  int ids[K];
#pragma unroll
  for (int b = 0; b < K; ++b) ids[b] = c[perm[b]];
  fill_ho_ids<K, T>(S, e, ids, x, X, in);
}

// Inputs 6K+2..6K+5: weight and reference coordinates of quadrature point q
// of rule r.
template <int K, typename T>
__device__ __forceinline__ void set_point(const QuadRule& r, int q, T* in) {
  in[6 * K + 2] = T(r.w[q]);
  in[6 * K + 3] = T(r.xi[q][0]);
  in[6 * K + 4] = T(r.xi[q][1]);
  in[6 * K + 5] = T(r.xi[q][2]);
}

// Energy of element e: its points summed in order (float64).
template <int K, typename T>
__device__ __forceinline__ double ho_energy(const SetDev& S, int64_t e, const double* x,
                                            const double* X) {
  T in[6 * K + 6];
  // the relabelling of corner 0 leaves every node in place
  fill_ho<K, T>(S, e, S.conn_ho + (int64_t)K * e, HoTet<K>::perm(0), x, X, in);
  double Ee = 0.0;
  for (int q = 0; q < HoTet<K>::kPts; ++q) {
    T out[1];
    set_point<K, T>(HoTet<K>::rule(), q, in);
    HoTet<K>::template energy<T>(in, out);
    Ee += double(out[0]);
  }
  return Ee;
}

// Element energies of a higher-order tet set -> one partial sum per workgroup.
template <int K, typename T>
__global__ __launch_bounds__(256) void k_energy_ho(SetDev S, const double* __restrict__ x,
                                                  const double* __restrict__ X,
                                                  double* __restrict__ partials,
                                                  int* __restrict__ nonfinite) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 256)
    acc += ho_energy<K, T>(S, e, x, X);
  double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s;
    if (!isfinite(s)) *nonfinite = 1;
  }
}

// Row of local node a of element e (node ids in a's relabelled order) at
// point q of rule r: out[0..2] gradient, out[3 + 3(K-1) i + 3 j + k] the
// off-diagonal block entries of the K - 1 other nodes in the row function's
// order (WANT_H), or the gradient only.
template <int K, typename T, bool WANT_H>
__device__ __forceinline__ void ho_row_point(const SetDev& S, int64_t e, const int* ids, int a,
                                             const QuadRule& r, int q, const double* x,
                                             const double* X, T* out) {
  T in[6 * K + 6];
  fill_ho_ids<K, T>(S, e, ids, x, X, in);
  set_point<K, T>(r, q, in);
  HoTet<K>::template row<T, WANT_H>(a, in, out);
}

// Part PART of the Hessian row (as HoTet<K>::row_part).
template <int K, typename T, int PART>
__device__ __forceinline__ void ho_row_point_part(const SetDev& S, int64_t e, const int* ids,
                                                  int a, const QuadRule& r, int q,
                                                  const double* x, const double* X, T* out) {
  T in[6 * K + 6];
  fill_ho_ids<K, T>(S, e, ids, x, X, in);
  set_point<K, T>(r, q, in);
  HoTet<K>::template row_part<T, PART>(a, in, out);
}

// Per-element E, gradient (n x 3K) and Hessian (n x 3K x 3K, row-major) of a
// higher-order tet set: one lane per (local node a, element) writes node a's
// gradient and Hessian rows; the diagonal block is minus the sum of the row's
// off-diagonal blocks (translation invariance).  Lanes run node-major so that
// the lanes of a wave take the same row function.
template <int K, typename T>
__global__ __launch_bounds__(64) void k_elem_eval_ho(SetDev S, const double* __restrict__ x,
                                                    const double* __restrict__ X,
                                                    T* __restrict__ Eo, T* __restrict__ go,
                                                    T* __restrict__ Ho) {
  constexpr int NO = 3 * (K - 1);
  constexpr int NV = 3 + 3 * NO;
  const int64_t n = S.n_elem * K;
  for (int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 64) {
    const int a = int(t / S.n_elem);
    const int64_t e = t - a * S.n_elem;
    const int8_t* perm = HoTet<K>::perm(a);
    const int r = ho_row_pos(K, a);
    T acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = T(0);
    int ids[K];
#pragma unroll
    for (int b = 0; b < K; ++b) ids[b] = S.conn_ho[(int64_t)K * e + perm[b]];
    for (int q = 0; q < HoTet<K>::kPts; ++q) {
      T out[NV];
      ho_row_point<K, T, true>(S, e, ids, a, HoTet<K>::rule(), q, x, X, out);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += out[v];
    }
    if (go) {
#pragma unroll
      for (int i = 0; i < 3; ++i) go[e * 3 * K + 3 * a + i] = acc[i];
    }
    if (Ho) {
      T* Hr = Ho + e * 9 * K * K + (int64_t)(3 * a) * 3 * K;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T d0 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
          const int b = perm[j < r ? j : j + 1];
          const T h0 = acc[3 + NO * i + 3 * j], h1 = acc[4 + NO * i + 3 * j],
                  h2 = acc[5 + NO * i + 3 * j];
          Hr[3 * K * i + 3 * b + 0] = h0;
          Hr[3 * K * i + 3 * b + 1] = h1;
          Hr[3 * K * i + 3 * b + 2] = h2;
          d0 += h0;
          d1 += h1;
          d2 += h2;
        }
        Hr[3 * K * i + 3 * a + 0] = -d0;
        Hr[3 * K * i + 3 * a + 1] = -d1;
        Hr[3 * K * i + 3 * a + 2] = -d2;
      }
    }
    if (Eo && a == 0) Eo[e] = T(ho_energy<K, T>(S, e, x, X));
  }
}

// Row assembly of a higher-order tet mesh (the steps of k_row_assemble_fast
// with the evaluation split over quadrature points).  A batch holds at most
// HoTet<K>::kCap incidences.  Step 1 runs the evaluation items (point p,
// incidence qi) = (item / nq, item % nq) in passes of kRowWG lanes; each pass
// adds its items into LDS one point at a time, or for the cubic rule two at a
// time (even points into one accumulator, odd points into another), so every
// incidence sums its points (its even and its odd points) in point order.  The batch's incidence codes, the incidences'
// relabelled element node ids (contiguous per batch) and the rule are staged
// in LDS first (in the space the block sums use later), so an item's position
// loads depend on LDS reads only; the contribution entries are staged too,
// and the block metadata of steps 2 and 5 is loaded before the evaluation.
// Contribution entries are (incidence << kShift) | j, j the other node's
// index in the row function's order.  WANT_H = false: gradient only.
template <int K>
struct HoStage {
  uint32_t code[HoTet<K>::kCap];
  int ids[HoTet<K>::kCap][K];
  QuadRule rule;
};

// Waves per SIMD the row kernel is compiled for (registers capped at 512 /
// waves, the rest spilled), so that several workgroups share a CU and one's
// memory waits overlap another's arithmetic.  Measured on the 137K-DoF boxes:
// FP32 g+H 0.24 -> 0.20 ms (quadratic, 3 waves) and 1.51 -> 0.98 ms (cubic, 2
// waves); the FP64 kernels spill too much for it to pay (cubic 3.0 -> 5.8 ms).
template <int K, typename T, bool WANT_H>
constexpr int ho_row_waves() {
  if (sizeof(T) == 8) return 1;
  return K == 10 ? (WANT_H ? 3 : 1) : 2;
}

template <int K, typename T, bool WANT_G, bool WANT_H>
__global__ __launch_bounds__(kRowWG, (ho_row_waves<K, T, WANT_H>())) void k_row_assemble_ho(
    RowArgs<T> A) {
  using P = HoTet<K>;
  constexpr int NO = 3 * (K - 1);
  constexpr int NV = WANT_H ? 3 + 3 * NO : 3;
  // rows padded by one value: lanes reading several components of one
  // incidence (or one slot) hit distinct LDS banks
  __shared__ T st[NV][P::kCap + 1];
  __shared__ T st2[P::kAcc == 2 ? NV : 1][P::kAcc == 2 ? P::kCap + 1 : 1];  // odd points
  __shared__ union {
    T blk[WANT_H ? 9 : 1][kRowWG + 1];
    HoStage<K> stg;
  } sh;
  auto& blk = sh.blk;
  __shared__ uint16_t s_ce[WANT_H ? P::kCap * (K - 1) : 1];
  __shared__ uint16_t s_blk[kRowWG + 1];
  __shared__ uint16_t s_inc[kRowWG + 1];
  const int t = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int r0 = A.batch_row[b], r1 = A.batch_row[b + 1];
  const int nrows = r1 - r0;
  const int q0 = A.inc_ptr[r0];
  const int p0 = A.row_ptr[r0];
  for (int r = t; r <= nrows; r += kRowWG) {
    s_blk[r] = (uint16_t)(A.row_ptr[r0 + r] - p0);
    s_inc[r] = (uint16_t)(A.inc_ptr[r0 + r] - q0);
  }
  __syncthreads();
  const int nq = s_inc[nrows];
  const int np = s_blk[nrows];
  // block metadata for steps 2 and 5, in flight during the evaluation
  int r = 0, col = 0;
  uint32_t info = 0;
  if (WANT_H && t < np) {
    while (s_blk[r + 1] <= t) ++r;
    col = A.col_idx[p0 + t];
    info = A.blk_info[p0 + t];
  }
  // step 0: staging
  for (int j = t; j < nq; j += kRowWG) sh.stg.code[j] = A.inc_code[q0 + j];
  for (int j = t; j < nq * K; j += kRowWG)
    sh.stg.ids[j / K][j % K] = A.inc_nodes[(int64_t)q0 * K + j];
  for (int j = t; j < 4 * P::kPts; j += kRowWG) {
    const int q = j >> 2, c = j & 3;
    if (c == 0) sh.stg.rule.w[q] = P::rule().w[q];
    else sh.stg.rule.xi[q][c - 1] = P::rule().xi[q][c - 1];
  }
  if (WANT_H) {
    const int e0 = A.batch_entry[b];
    for (int j = t; j < (K - 1) * nq; j += kRowWG) s_ce[j] = A.centry[e0 + j];
  }
  __syncthreads();
  uint8_t fixed_rc = 0;  // Dirichlet flags of the block's row and column
  if (WANT_H && t < np && A.fixed) fixed_rc = A.fixed[r0 + r] | A.fixed[col];
  // step 1: evaluation passes (with the Hessian, once per part of the row:
  // part k accumulates its values v = part_v(k, u) only)
  const int n_items = nq * P::kPts;
  auto eval_part = [&](auto part_c) {
    constexpr int PART = decltype(part_c)::value;
    constexpr int NP = WANT_H ? P::template parts<T>() : 1;
    constexpr int J0 = WANT_H ? P::part_lo(PART) : 0, J1 = WANT_H ? P::part_lo(PART + 1) : 0;
    constexpr int NG = PART == 0 ? 3 : 0;                   // gradient values in this part
    constexpr int NVP = NP == 1 ? NV : NG + 9 * (J1 - J0);  // values of this part
    // value u of the part -> its row entry v (NP == 1: the identity)
    auto part_v = [](int u) {
      if (NP == 1 || u < NG) return u;
      const int w = u - NG, per_i = 3 * (J1 - J0);
      const int i = w / per_i, jm = w - i * per_i;
      return 3 + NO * i + 3 * J0 + jm;
    };
    for (int i0 = 0; i0 < n_items; i0 += kRowWG) {
      const int item = i0 + t;
      const bool act = item < n_items;
      const int p = act ? item / nq : 0;
      const int qi = act ? item - p * nq : 0;
      T out[NVP];
      if (act) {
        const uint32_t code = sh.stg.code[qi];
        if constexpr (NP == 1)
          ho_row_point<K, T, WANT_H>(A.sets.s[inc_set(code)], inc_elem(code), sh.stg.ids[qi],
                                     inc_local(code), sh.stg.rule, p, A.x, A.X, out);
        else
          ho_row_point_part<K, T, PART>(A.sets.s[inc_set(code)], inc_elem(code), sh.stg.ids[qi],
                                        inc_local(code), sh.stg.rule, p, A.x, A.X, out);
      }
      // With two accumulators, even points accumulate in st and odd points in
      // st2, a pair of points per round.  Round k is uniform: the first round
      // stores, the others add in chunks of 64 values (their LDS reads in
      // flight together, then the adds and stores).
      const int k_lo = (i0 / nq) / P::kAcc, k_hi = ((min(n_items, i0 + kRowWG) - 1) / nq) / P::kAcc;
      T(*acc_st)[P::kCap + 1] = st;
      if constexpr (P::kAcc == 2) acc_st = (p & 1) ? st2 : st;
      for (int k = k_lo; k <= k_hi; ++k) {
        if (act && p / P::kAcc == k) {
          if (k == 0) {
#pragma unroll
            for (int u = 0; u < NVP; ++u) acc_st[part_v(u)][qi] = out[u];
          } else {
            constexpr int C = 64;
#pragma unroll
            for (int u0 = 0; u0 < NVP; u0 += C) {
              T cur[C];
#pragma unroll
              for (int u = 0; u < C; ++u)
                if (u0 + u < NVP) cur[u] = acc_st[part_v(u0 + u)][qi];
#pragma unroll
              for (int u = 0; u < C; ++u)
                if (u0 + u < NVP) acc_st[part_v(u0 + u)][qi] = cur[u] + out[u0 + u];
            }
          }
        }
        __syncthreads();
      }
    }
  };
  eval_part(std::integral_constant<int, 0>{});
  if constexpr (WANT_H && P::template parts<T>() > 1) eval_part(std::integral_constant<int, 1>{});
  if constexpr (WANT_H && P::template parts<T>() > 2) eval_part(std::integral_constant<int, 2>{});
  if constexpr (P::kAcc == 2) {
    // sum of the even and the odd points
    for (int j = t; j < NV * nq; j += kRowWG) {
      const int v = j / nq, qi = j - v * nq;
      st[v][qi] += st2[v][qi];
    }
    __syncthreads();
  }
  const bool diag = WANT_H && t < np && col == r0 + r;
  T acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = T(0);
  if constexpr (WANT_H) {
    // step 2: off-diagonal blocks from their contribution lists
    if (t < np) {
      const uint16_t* ce = s_ce + (info >> 8);
      const int cnt = int(info & 0xFFu);
      for (int j = 0; j < cnt; ++j) {
        const uint32_t wv = ce[j];
        const int q = int(wv >> P::kShift);
        const int jj = int(wv & ((1u << P::kShift) - 1u));
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            acc[3 * i + kk] += st[3 + NO * i + 3 * jj + kk][q];
      }
      // step 3: publish
#pragma unroll
      for (int c = 0; c < 9; ++c) blk[c][t] = acc[c];
    }
    __syncthreads();
  }
  // step 4: diagonal blocks (minus the sum of the row's off-diagonal blocks,
  // plus inertia) and the gradient (incidences in order, float64)
  const int nd = WANT_H ? 9 * nrows : 0;
  for (int j = t; j < nd + (WANT_G ? 3 * nrows : 0); j += kRowWG) {
    if (j < nd) {
      const int rr = j / 9, c = j - 9 * rr;
      T sum = T(0);
      for (int sl = s_blk[rr]; sl < s_blk[rr + 1]; ++sl) sum += blk[WANT_H ? c : 0][sl];
      T dv = -sum;
      if (A.xt && (c % 4) == 0) dv += T(A.mass[r0 + rr] * A.inv_dt2);
      blk[WANT_H ? c : 0][A.diag_pos[r0 + rr] - p0] = dv;
    } else {
      const int jj = j - nd;
      const int rr = jj / 3, c = jj - 3 * rr;
      const int row = r0 + rr;
      double g = 0.0;
      for (int q = s_inc[rr]; q < s_inc[rr + 1]; ++q) g += double(st[c][q]);
      if (A.xt) g += A.mass[row] * A.inv_dt2 * (A.x[3 * row + c] - A.xt[3 * row + c]);
      if (A.fixed && A.fixed[row]) g = 0.0;
      if (!isfinite(g)) *A.nonfinite = 1;
      A.g[3 * row + c] = g;
    }
  }
  if (!WANT_H) return;
  __syncthreads();
  // step 5: Dirichlet, write every block once, block-Jacobi inverses
  if (t < np) {
    const int row = r0 + r;
    if (diag) {
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] = blk[WANT_H ? c : 0][t];
    }
    if (fixed_rc) {
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] = (diag && (c % 4) == 0) ? T(1) : T(0);
    }
    store_block(A, row, col, t - s_blk[r], acc);
    if (diag && A.dinv) {
      double a9[9], ri[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) a9[c] = double(acc[c]);
      inverse3(a9, ri);
      store_dinv(A.dinv + kDinv * (int64_t)row, ri);
    }
  }
}

// ---------------------------------------------------------------------------
// solver kernels
// ---------------------------------------------------------------------------

// [traffic-hash-begin pcg_spmv]
// Lanes per block row of the solver's SpMV kernels (a row of a tet mesh has
// about 15 blocks).
constexpr int kSpmvLanes = 16;
constexpr int kSpmvRows = 256 / kSpmvLanes;  // block rows per 256-lane workgroup pass

// Sum of v over the kSpmvLanes lanes of a row group (same order on every row).
template <typename TY>
__device__ __forceinline__ TY row_lane_sum(TY v) {
#pragma unroll
  for (int m = kSpmvLanes / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kSpmvLanes);
  return v;
}

// y = A x (BSR, component-major values; kSpmvLanes lanes per block row,
// lane l takes blocks l, l + kSpmvLanes, ...)
template <typename TA, typename TX, typename TY>
__device__ __forceinline__ void spmv_row(int row, int lane, const int* __restrict__ row_ptr,
                                         const int* __restrict__ col, const TA* __restrict__ vals,
                                         int64_t nnzb, const TX* __restrict__ x, TY* acc) {
  acc[0] = acc[1] = acc[2] = TY(0);
  const int pe = row_ptr[row + 1];
  for (int p = row_ptr[row] + lane; p < pe; p += kSpmvLanes) {
    const int j = col[p];
    // the nine value loads are issued together, ahead of the gather of x
    TY v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = TY(vals[c * nnzb + p]);
    const TY x0 = TY(x[3 * j]), x1 = TY(x[3 * j + 1]), x2 = TY(x[3 * j + 2]);
    acc[0] += v[0] * x0 + v[1] * x1 + v[2] * x2;
    acc[1] += v[3] * x0 + v[4] * x1 + v[5] * x2;
    acc[2] += v[6] * x0 + v[7] * x1 + v[8] * x2;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = row_lane_sum(acc[c]);
}

// The solver's matrix in half storage: row i holds its blocks (i, j), j <= i,
// at half positions lrow_ptr[i] ... (values at half_at); cv[p] pairs pattern
// slot p's column with the half position to read (bitwise complement: the
// stored block is the transpose (j, i) of slot (i, j)).
template <typename T>
struct HalfBsr {
  const int* row_ptr;
  const int2* cv;
  const T* vals;
  int64_t nnzl;
};

// y = A x for one block row of a half-stored symmetric matrix (kSpmvLanes
// lanes per block row, lane l takes pattern slots l, l + kSpmvLanes, ...;
// same lane order and reduction as spmv_row).
template <typename TA, typename TX, typename TY>
__device__ __forceinline__ void spmv_row_half(int row, int lane, const HalfBsr<TA>& H,
                                              const TX* __restrict__ x, TY* acc) {
  acc[0] = acc[1] = acc[2] = TY(0);
  const int pe = H.row_ptr[row + 1];
  for (int p = H.row_ptr[row] + lane; p < pe; p += kSpmvLanes) {
    const int2 e = H.cv[p];
    const bool tr = e.y < 0;  // the stored block is read by columns
    const int64_t l = tr ? ~e.y : e.y;
    TY v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = TY(H.vals[half_at(l, c, H.nnzl)]);
    const TY x0 = TY(x[3 * (int64_t)e.x]), x1 = TY(x[3 * (int64_t)e.x + 1]),
             x2 = TY(x[3 * (int64_t)e.x + 2]);
    const TY a01 = tr ? v[3] : v[1], a02 = tr ? v[6] : v[2];
    const TY a10 = tr ? v[1] : v[3], a12 = tr ? v[7] : v[5];
    const TY a20 = tr ? v[2] : v[6], a21 = tr ? v[5] : v[7];
    acc[0] += v[0] * x0 + a01 * x1 + a02 * x2;
    acc[1] += a10 * x0 + v[4] * x1 + a12 * x2;
    acc[2] += a20 * x0 + a21 * x1 + v[8] * x2;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = row_lane_sum(acc[c]);
}

// The contact matrix beside the mesh's (DYN): a second BSR over the same rows.
template <typename T>
struct DynBsr {
  const int* row_ptr;
  const int* col;
  const T* vals;
  int64_t nnzb;
};

// r = b - A x  (float64 residual of the Newton system, A promoted)
template <typename TA, bool DYN>
__global__ __launch_bounds__(256) void k_residual64(int64_t N, HalfBsr<TA> H,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ r, DynBsr<TA> C) {
  const int lane = threadIdx.x % kSpmvLanes;
  for (int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kSpmvLanes; row < N;
       row += (int64_t)gridDim.x * kSpmvRows) {
    double acc[3];
    spmv_row_half<TA, double, double>((int)row, lane, H, x, acc);
    if (DYN) {
      double ac[3];
      spmv_row<TA, double, double>((int)row, lane, C.row_ptr, C.col, C.vals, C.nnzb, x, ac);
      acc[0] += ac[0];
      acc[1] += ac[1];
      acc[2] += ac[2];
    }
    if (lane == 0) {
      r[3 * row + 0] = b[3 * row + 0] - acc[0];
      r[3 * row + 1] = b[3 * row + 1] - acc[1];
      r[3 * row + 2] = b[3 * row + 2] - acc[2];
    }
  }
}

// PCG state.  Partial sums (one per workgroup) are written
// by one kernel and reduced, redundantly and in the same order, by every
// workgroup of the next kernel.  Scalars live in a small device array; rz of
// iteration k is kept in slot S_RZ + (k & 1) so that readers of the previous
// value never race with the writer of the new one.
// Grid sizes: the SpMV kernel streams the matrix and runs best with up to
// 2048 workgroups; the node-wise kernels use up to 256 (every SpMV workgroup
// first sums their partials, so fewer of them make that preamble cheaper at
// no cost to the node-wise kernels themselves).  Small meshes get
// grids sized to their rows (gs a multiple of 8), so that no launch is made
// of workgroups with nothing to do.  Each partial array holds up to kPcgP
// entries.
constexpr int kPcgGs = 2048, kPcgGu = 256, kPcgP = 4096;
static int pcg_gs(int64_t N) {
  const int64_t g = (N + kSpmvRows - 1) / kSpmvRows;
  return (int)std::min<int64_t>(kPcgGs, std::max<int64_t>(8, (g + 7) / 8 * 8));
}
static int pcg_gu(int64_t N) {
  return (int)std::min<int64_t>(kPcgGu, std::max<int64_t>(1, (N + 255) / 256));
}
enum { S_DONE = 0, S_ITERS, S_TOL2, S_BB, S_RZ, S_RZ1, S_MAXIT, S_NSCALARS };
enum { P_RZ = 0, P_RR = 1, P_BB = 2, P_PQ = 3 };  // partial arrays, kPcgP each

// r = b, z = M^-1 r, x = p = q = 0; partials of rz, rr, bb
template <typename T, typename TB>
__global__ __launch_bounds__(256) void k_pcg_init(int64_t N, const TB* __restrict__ b,
                                                  const T* __restrict__ Dinv, T* __restrict__ xs,
                                                  T* __restrict__ r, T* __restrict__ z,
                                                  T* __restrict__ p, T* __restrict__ q,
                                                  double* __restrict__ P, double* __restrict__ S,
                                                  double tol2, int max_iter) {
  __shared__ double sh[4];
  double rz = 0.0, rr = 0.0, bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    T rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rv[c] = T(b[3 * i + c]);
      r[3 * i + c] = rv[c];
      xs[3 * i + c] = T(0);
      p[3 * i + c] = T(0);
      q[3 * i + c] = T(0);
      const double bc = double(b[3 * i + c]);
      bb += bc * bc;
      rr += double(rv[c]) * double(rv[c]);
    }
    const T* d = Dinv + kDinv * i;  // upper triangle of the symmetric inverse
    const T d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4], d5 = d[5];
    const T zv[3] = {d0 * rv[0] + d1 * rv[1] + d2 * rv[2], d1 * rv[0] + d3 * rv[1] + d4 * rv[2],
                     d2 * rv[0] + d4 * rv[1] + d5 * rv[2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[3 * i + c] = zv[c];
      rz += double(rv[c]) * double(zv[c]);
    }
  }
  const double s0 = block_sum_256(rz, sh);
  const double s1 = block_sum_256(rr, sh);
  const double s2 = block_sum_256(bb, sh);
  if (threadIdx.x == 0) {
    P[P_RZ * kPcgP + blockIdx.x] = s0;
    P[P_RR * kPcgP + blockIdx.x] = s1;
    P[P_BB * kPcgP + blockIdx.x] = s2;
    if (blockIdx.x == 0) {
      S[S_DONE] = 0.0;
      S[S_ITERS] = 0.0;
      S[S_TOL2] = tol2;
      S[S_MAXIT] = double(max_iter);
    }
  }
}

// Iteration k: reduce rz, rr of the previous update; stop on convergence or
// at the iteration limit; beta = rz_k / rz_(k-1); w = A z; p = z + beta p;
// q = w + beta q; partials of p.q.
// Rows: workgroup b runs on XCD b % 8 and takes, in steps of kSpmvRows rows,
// the rows of the XCD's contiguous eighth of the matrix (gridDim.x is a
// multiple of 8).
// The body takes the workgroup index and count as arguments: a launch of one
// mesh passes blockIdx.x and gridDim.x, a launch over several meshes each
// mesh's own index and count (so each mesh computes exactly what it would
// alone).
template <typename T, bool DYN>
__device__ __forceinline__ void pcg_spmv_body(int bid, int nblk, int k, int64_t N,
                                              const HalfBsr<T>& H,
                                              const T* __restrict__ z, T* __restrict__ p,
                                              T* __restrict__ q, double* __restrict__ P,
                                              double* __restrict__ S, int gu, DynBsr<T> C) {
  if (S[S_DONE] != 0.0) return;
  __shared__ double sh[4];
  const double rz = sum_partials(P + P_RZ * kPcgP, gu, sh);
  const double rr = sum_partials(P + P_RR * kPcgP, gu, sh);
  const double bb = k == 0 ? sum_partials(P + P_BB * kPcgP, gu, sh) : S[S_BB];
  const bool first = bid == 0 && threadIdx.x == 0;
  if (bb == 0.0 || rr <= S[S_TOL2] * bb || k >= int(S[S_MAXIT]) || !isfinite(rr)) {
    if (first) {
      S[S_DONE] = isfinite(rr) ? 1.0 : 3.0;
      S[S_ITERS] = double(k);
    }
    return;
  }
  const T beta = k == 0 ? T(0) : T(rz / S[S_RZ + ((k - 1) & 1)]);
  if (first) {
    S[S_RZ + (k & 1)] = rz;
    if (k == 0) S[S_BB] = bb;
  }
  const int lane = threadIdx.x % kSpmvLanes;
  // XCD-aware row ranges: XCD x takes the x-th contiguous eighth of the rows,
  // so that the gathered entries of z and the transposed blocks (read from
  // rows a few thousand rows away) are met again in that XCD's L2.  (Over
  // several meshes, each mesh's first workgroup is a multiple of 8, so bid & 7
  // is still the workgroup's XCD.)
  const int xcd = bid & 7;
  const int64_t lo = N * xcd / 8, hi = N * (xcd + 1) / 8;
  const int64_t stride = (int64_t)(nblk >> 3) * kSpmvRows;
  const int64_t first_row = (int64_t)(bid >> 3) * kSpmvRows;
  double pq = 0.0;
  for (int64_t row = lo + first_row + threadIdx.x / kSpmvLanes; row < hi; row += stride) {
    T acc[3];
    spmv_row_half<T, T, T>((int)row, lane, H, z, acc);
    if (DYN) {
      T ac[3];
      spmv_row<T, T, T>((int)row, lane, C.row_ptr, C.col, C.vals, C.nnzb, z, ac);
      acc[0] += ac[0];
      acc[1] += ac[1];
      acc[2] += ac[2];
    }
    if (lane < 3) {  // lane c writes component c of the row
      const T a = lane == 0 ? acc[0] : lane == 1 ? acc[1] : acc[2];
      const T pn = z[3 * row + lane] + beta * p[3 * row + lane];
      const T qn = a + beta * q[3 * row + lane];
      p[3 * row + lane] = pn;
      q[3 * row + lane] = qn;
      pq += double(pn) * double(qn);
    }
  }
  const double s = block_sum_256(pq, sh);
  if (threadIdx.x == 0) P[P_PQ * kPcgP + bid] = s;
}

template <typename T, bool DYN>
__global__ __launch_bounds__(256) void k_pcg_spmv(int k, int64_t N, HalfBsr<T> H,
                                                  const T* __restrict__ z, T* __restrict__ p,
                                                  T* __restrict__ q, double* __restrict__ P,
                                                  double* __restrict__ S, int gu, DynBsr<T> C) {
  pcg_spmv_body<T, DYN>(blockIdx.x, gridDim.x, k, N, H, z, p, q, P, S, gu, C);
}

// [traffic-hash-end pcg_spmv]

// Iteration k: alpha = rz_k / p.q; x += alpha p; r -= alpha q; z = M^-1 r;
// partials of rz, rr.
template <typename T>
__device__ __forceinline__ void pcg_update_body(int bid, int nblk, int k, int64_t N,
                                                const T* __restrict__ Dinv, T* __restrict__ xs,
                                                T* __restrict__ r, T* __restrict__ z,
                                                const T* __restrict__ p, const T* __restrict__ q,
                                                double* __restrict__ P, double* __restrict__ S,
                                                int gs) {
  if (S[S_DONE] != 0.0) return;
  __shared__ double sh[4];
  const double pq = sum_partials(P + P_PQ * kPcgP, gs, sh);
  if (!(pq > 0.0)) {  // direction of non-positive curvature: stop
    if (bid == 0 && threadIdx.x == 0) {
      S[S_DONE] = 2.0;
      S[S_ITERS] = double(k);
    }
    return;
  }
  const T alpha = T(S[S_RZ + (k & 1)] / pq);
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)bid * 256 + threadIdx.x; i < N; i += (int64_t)nblk * 256) {
    T rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xs[3 * i + c] += alpha * p[3 * i + c];
      rv[c] = r[3 * i + c] - alpha * q[3 * i + c];
      r[3 * i + c] = rv[c];
      rr += double(rv[c]) * double(rv[c]);
    }
    const T* d = Dinv + kDinv * i;  // upper triangle of the symmetric inverse
    const T d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4], d5 = d[5];
    const T zv[3] = {d0 * rv[0] + d1 * rv[1] + d2 * rv[2], d1 * rv[0] + d3 * rv[1] + d4 * rv[2],
                     d2 * rv[0] + d4 * rv[1] + d5 * rv[2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[3 * i + c] = zv[c];
      rz += double(rv[c]) * double(zv[c]);
    }
  }
  const double s0 = block_sum_256(rz, sh);
  const double s1 = block_sum_256(rr, sh);
  if (threadIdx.x == 0) {
    P[P_RZ * kPcgP + bid] = s0;
    P[P_RR * kPcgP + bid] = s1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pcg_update(int k, int64_t N, const T* __restrict__ Dinv,
                                                    T* __restrict__ xs, T* __restrict__ r,
                                                    T* __restrict__ z, const T* __restrict__ p,
                                                    const T* __restrict__ q,
                                                    double* __restrict__ P,
                                                    double* __restrict__ S, int gs) {
  pcg_update_body<T>(blockIdx.x, gridDim.x, k, N, Dinv, xs, r, z, p, q, P, S, gs);
}

// PCG iterations of several meshes in one launch (the serving loop's batch):
// workgroups [blk, blk + g) of the launch run mesh s's iteration k0 + j with
// that mesh's own grid g, so every mesh computes what it would alone.
template <typename T>
struct PcgScene {
  int64_t N;
  HalfBsr<T> H;
  DynBsr<T> C;
  const T* Dinv;
  T *xs, *r, *z, *p, *q;
  double* P;
  double* S;
  int gs, gu;        // the mesh's SpMV and update grids
  int k0, n;         // first iteration of this chunk, iterations wanted
  int blk_s, blk_u;  // first workgroup in the SpMV launch (a multiple of 8) and the update launch
};

template <typename T>
__device__ __forceinline__ int pcg_scene_of(const PcgScene<T>* __restrict__ tab, int ns,
                                            bool spmv) {
  int s = 0;
  while (s + 1 < ns && (spmv ? tab[s + 1].blk_s : tab[s + 1].blk_u) <= (int)blockIdx.x) ++s;
  return s;
}

template <typename T, bool DYN>
__global__ __launch_bounds__(256) void k_pcg_spmv_multi(int j, const PcgScene<T>* __restrict__ tab,
                                                        int ns) {
  const PcgScene<T>& sc = tab[pcg_scene_of(tab, ns, true)];
  const int bid = (int)blockIdx.x - sc.blk_s;
  if (j >= sc.n || bid >= sc.gs) return;
  pcg_spmv_body<T, DYN>(bid, sc.gs, sc.k0 + j, sc.N, sc.H, sc.z, sc.p, sc.q, sc.P, sc.S, sc.gu,
                        sc.C);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pcg_update_multi(int j, const PcgScene<T>* __restrict__ tab,
                                                          int ns) {
  const PcgScene<T>& sc = tab[pcg_scene_of(tab, ns, false)];
  const int bid = (int)blockIdx.x - sc.blk_u;
  if (j >= sc.n || bid >= sc.gu) return;
  pcg_update_body<T>(bid, sc.gu, sc.k0 + j, sc.N, sc.Dinv, sc.xs, sc.r, sc.z, sc.p, sc.q, sc.P,
                     sc.S, sc.gs);
}

__global__ __launch_bounds__(256) void k_dot64(int64_t n, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ partials) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += a[i] * b[i];
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_reduce_checked(const double* __restrict__ partials, int n,
                                                        double* __restrict__ out,
                                                        int* __restrict__ nonfinite) {
  __shared__ double sh[4];
  const double s = sum_partials(partials, n, sh);
  if (threadIdx.x == 0) {
    *out = s;
    if (!isfinite(s)) *nonfinite = 1;
  }
}

__global__ __launch_bounds__(256) void k_x_tilde(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ v, double dt, double g0,
                                                 double g1, double g2, double* __restrict__ xt) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int c = int(i % 3);
    const double g = c == 0 ? g0 : c == 1 ? g1 : g2;
    xt[i] = x[i] + dt * v[i] + dt * dt * g;
  }
}

// out = a + beta b
__global__ __launch_bounds__(256) void k_lincomb64(int64_t n, double* __restrict__ out,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ b, double beta) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = a[i] + beta * b[i];
}

__global__ __launch_bounds__(256) void k_velocity(int64_t n, double* __restrict__ v,
                                                  const double* __restrict__ xn,
                                                  const double* __restrict__ xo, double inv_dt) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    v[i] = (xn[i] - xo[i]) * inv_dt;
}

// dst = float(src), round to nearest (the float32 copy of float64 data)
__global__ __launch_bounds__(256) void k_round_f64(int64_t n, const double* __restrict__ src,
                                                   float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i] = float(src[i]);
}

// dx (float64) += x_pcg (T)
template <typename T>
__global__ __launch_bounds__(256) void k_accumulate(int64_t n, double* __restrict__ dx,
                                                    const T* __restrict__ xs) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dx[i] += double(xs[i]);
}

__global__ __launch_bounds__(256) void k_check_finite(int64_t n, const double* __restrict__ a,
                                                      int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    bad |= !isfinite(a[i]);
  if (bad) *flag = 1;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// conditional contact barrier: node p against the plane of nodes t0, t1, t2
// (Eq. 9: elements whose activation c_e = d_hat - d is positive are gathered
// and evaluated, the others add nothing)
// ---------------------------------------------------------------------------
// Inputs of the generated functions: positions relative to p, k_c, d_hat.
template <typename T>
__device__ __forceinline__ void fill_contact(const int* __restrict__ tup,
                                             const double* __restrict__ x, double kc, double dhat,
                                             T* in) {
  const int64_t p = tup[0];
  const double x0 = x[3 * p], x1 = x[3 * p + 1], x2 = x[3 * p + 2];
  in[0] = in[1] = in[2] = T(0);
#pragma unroll
  for (int a = 1; a < 4; ++a) {
    const int64_t n = tup[a];
    in[3 * a + 0] = T(x[3 * n + 0] - x0);
    in[3 * a + 1] = T(x[3 * n + 1] - x1);
    in[3 * a + 2] = T(x[3 * n + 2] - x2);
  }
  in[12] = T(kc);
  in[13] = T(dhat);
}

// Activation of every candidate (float64), counted per chunk of
// kContactChunk candidates (one workgroup per chunk).  A degenerate triangle
// gives a NaN activation: inactive.
__global__ __launch_bounds__(256) void k_contact_activate(int64_t n, const int* __restrict__ tuples,
                                                         const double* __restrict__ x, double kc,
                                                         double dhat, uint8_t* __restrict__ flag,
                                                         int* __restrict__ chunk_count) {
  __shared__ int sh[4];
  const int64_t c0 = (int64_t)blockIdx.x * kContactChunk;
  const int64_t c1 = c0 + kContactChunk < n ? c0 + kContactChunk : n;
  int cnt = 0;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
    double in[14], a[1];
    fill_contact<double>(tuples + 4 * c, x, kc, dhat, in);
    ipc_point_plane_act_s_E<double>(in, a);
    const int f = a[0] > 0.0 ? 1 : 0;
    flag[c] = (uint8_t)f;
    cnt += f;
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) cnt += __shfl_xor(cnt, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) chunk_count[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Exclusive scan of the chunk counts (in place) and the total.
__global__ void k_contact_scan(int n_chunks, int* __restrict__ chunk_count, int* __restrict__ total) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int acc = 0;
  for (int i = 0; i < n_chunks; ++i) {
    const int v = chunk_count[i];
    chunk_count[i] = acc;
    acc += v;
  }
  *total = acc;
}

// Compaction in candidate order: act[k] = the k-th active candidate, slot[c]
// = its k, or -1 for an inactive candidate.
__global__ __launch_bounds__(256) void k_contact_compact(int64_t n, const uint8_t* __restrict__ flag,
                                                        const int* __restrict__ chunk_off,
                                                        int* __restrict__ slot, int* __restrict__ act) {
  __shared__ int wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kContactChunk;
  int base = chunk_off[blockIdx.x];
  for (int r = 0; r < kContactChunk / 256; ++r) {
    const int64_t c = c0 + r * 256 + threadIdx.x;
    const int f = c < n ? flag[c] : 0;
    const unsigned long long mask = __ballot(f);
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[w] = __popcll(mask);
    __syncthreads();
    int off = base;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (c < n) {
      if (f) {
        slot[c] = off + pre;
        act[off + pre] = (int)c;
      } else {
        slot[c] = -1;
      }
    }
    base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

// Gradients (eg, n x 12) and Hessians (eH, n x 144) of the active elements,
// in compacted order.
template <typename T>
__global__ __launch_bounds__(128) void k_contact_eval(const int* __restrict__ act,
                                                     const int* __restrict__ n_active,
                                                     const int* __restrict__ tuples,
                                                     const double* __restrict__ x, double kc,
                                                     double dhat, T* __restrict__ eg,
                                                     T* __restrict__ eH) {
  const int na = *n_active;
  for (int k = blockIdx.x * 128 + threadIdx.x; k < na; k += gridDim.x * 128) {
    T in[14], o[157];
    fill_contact<T>(tuples + 4 * (int64_t)act[k], x, kc, dhat, in);
    ipc_point_plane_s_EgH<T>(in, o);
#pragma unroll
    for (int v = 0; v < 12; ++v) eg[(int64_t)k * 12 + v] = o[1 + v];
#pragma unroll
    for (int v = 0; v < 144; ++v) eH[(int64_t)k * 144 + v] = o[13 + v];
  }
}

// Branch mode: every candidate through the barrier whose activation is a
// branch of its expression (inactive candidates take the zero arm, which
// skips the barrier's operations); the element arrays are indexed by
// candidate, slot[c] = c, and the "active" count is n.
template <typename T>
__global__ __launch_bounds__(128) void k_contact_eval_branch(int64_t n, const int* __restrict__ tuples,
                                                            const double* __restrict__ x, double kc,
                                                            double dhat, T* __restrict__ eg,
                                                            T* __restrict__ eH,
                                                            int* __restrict__ slot,
                                                            int* __restrict__ n_active) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_active = (int)n;
  for (int64_t k = (int64_t)blockIdx.x * 128 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 128) {
    T in[14], o[157];
    fill_contact<T>(tuples + 4 * k, x, kc, dhat, in);
    ipc_point_plane_cond_s_EgH<T>(in, o);
#pragma unroll
    for (int v = 0; v < 12; ++v) eg[k * 12 + v] = o[1 + v];
#pragma unroll
    for (int v = 0; v < 144; ++v) eH[k * 144 + v] = o[13 + v];
    slot[k] = (int)k;
  }
}

// Dynamic element set: every element's gradient and Hessian (generated
// s_EgH of its kind) in element order, slot[e] = e and the "active" count n;
// the contact block, gradient and inverse kernels then assemble them.
template <typename T, int KIND>
__global__ __launch_bounds__(128) void k_dyn_eval(SetDev S, const double* __restrict__ x,
                                                  const double* __restrict__ X,
                                                  T* __restrict__ eg, T* __restrict__ eH,
                                                  int* __restrict__ slot, int* __restrict__ n_active) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_active = (int)S.n_elem;
  for (int64_t e = (int64_t)blockIdx.x * 128 + threadIdx.x; e < S.n_elem;
       e += (int64_t)gridDim.x * 128) {
    const Relabel R = identity_order(S.conn[e]);
    T in[kMaxIn];
    T out[157];
    elem_inputs<T, KIND>(S, e, R, x, X, in);
    gen_s_EgH<T, KIND>(in, out);
#pragma unroll
    for (int v = 0; v < 12; ++v) eg[e * 12 + v] = out[1 + v];
#pragma unroll
    for (int v = 0; v < 144; ++v) eH[e * 144 + v] = out[13 + v];
    slot[e] = (int)e;
  }
}

// Nearest-PSD projection of the active elements' Hessians (the element
// projection of the mesh's energies; the count is read on the device).
__global__ __launch_bounds__(64, 2) void k_contact_project32(float* __restrict__ H,
                                                            const int* __restrict__ n_active) {
  project_psd_lane<float, 4, 1>(H, *n_active, 30, 2e-7f, nullptr);
}
__global__ __launch_bounds__(64) void k_contact_project64(double* __restrict__ H,
                                                         const int* __restrict__ n_active) {
  __shared__ double vs[9 * 9 * 64];
  project_psd_lane<double, 4, 64>(H, *n_active, 30, 1e-15, vs);
}

// Contact blocks: each block sums its (candidate, a, b) contributions of the
// active candidates in candidate order; Dirichlet rows and columns are zero.
template <typename T>
__global__ __launch_bounds__(256) void k_contact_blocks(
    int64_t nnzb, const int* __restrict__ blk_row, const int* __restrict__ col,
    const int* __restrict__ blk_ptr, const int* __restrict__ blk_src, const int* __restrict__ slot,
    const T* __restrict__ eH, const uint8_t* __restrict__ fixed, T* __restrict__ vals) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnzb;
       p += (int64_t)gridDim.x * 256) {
    T acc[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) acc[v] = T(0);
    for (int j = blk_ptr[p]; j < blk_ptr[p + 1]; ++j) {
      const int src = blk_src[j];
      const int k = slot[src >> 4];
      if (k < 0) continue;
      const int a = (src >> 2) & 3, b = src & 3;
      const T* H = eH + (int64_t)k * 144;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) acc[3 * i + kk] += H[(3 * a + i) * 12 + 3 * b + kk];
    }
    if (fixed && (fixed[blk_row[p]] | fixed[col[p]])) {
#pragma unroll
      for (int v = 0; v < 9; ++v) acc[v] = T(0);
    }
#pragma unroll
    for (int v = 0; v < 9; ++v) vals[(int64_t)v * nnzb + p] = acc[v];
  }
}

// Contact gradient rows added to g (float64, candidate order per node);
// Dirichlet nodes keep their zero row.
template <typename T>
__global__ __launch_bounds__(256) void k_contact_grad(int64_t n_gnode, const int* __restrict__ gnode,
                                                     const int* __restrict__ gptr,
                                                     const int* __restrict__ gsrc,
                                                     const int* __restrict__ slot,
                                                     const T* __restrict__ eg,
                                                     const uint8_t* __restrict__ fixed,
                                                     double* __restrict__ g,
                                                     int* __restrict__ nonfinite) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_gnode;
       i += (int64_t)gridDim.x * 256) {
    const int64_t v = gnode[i];
    if (fixed && fixed[v]) continue;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = gptr[i]; j < gptr[i + 1]; ++j) {
      const int src = gsrc[j];
      const int k = slot[src >> 2];
      if (k < 0) continue;
      const int a = src & 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += double(eg[(int64_t)k * 12 + 3 * a + c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double gv = g[3 * v + c] + acc[c];
      if (!isfinite(gv)) *nonfinite = 1;
      g[3 * v + c] = gv;
    }
  }
}

// Block-Jacobi inverses of the nodes with contact blocks, from the sum of the
// mesh's and the contact diagonal block.
template <typename T>
__global__ __launch_bounds__(256) void k_contact_dinv(int64_t n_gnode, const int* __restrict__ gnode,
                                                     const int* __restrict__ gdiag,
                                                     const int* __restrict__ row_ptr,
                                                     const int* __restrict__ diag_pos,
                                                     const int* __restrict__ lrow_ptr,
                                                     const T* __restrict__ lvals, int64_t nnzl,
                                                     const T* __restrict__ cvals, int64_t cnnzb,
                                                     T* __restrict__ dinv) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_gnode;
       i += (int64_t)gridDim.x * 256) {
    const int64_t v = gnode[i];
    // the mesh's diagonal block: the last block of row v's half
    const int64_t l = (int64_t)lrow_ptr[v] + diag_pos[v] - row_ptr[v];
    const int64_t q = gdiag[i];
    double a[9], r[9];
#pragma unroll
    for (int c = 0; c < 9; ++c)
      a[c] = double(lvals[half_at(l, c, nnzl)]) + double(cvals[c * cnnzb + q]);
    inverse3(a, r);
    store_dinv(dinv + kDinv * v, r);
  }
}

// Contact energy of every candidate at x (float64): zero when inactive, +inf
// when the point is on or behind the plane.
// BRANCH: the energy comes from the branched barrier for every candidate
// (zero arm when inactive) instead of the activation test and the plain
// barrier; the domain end (d <= 0) is +inf in both.
template <bool BRANCH>
__global__ __launch_bounds__(256) void k_contact_energy(int64_t n, const int* __restrict__ tuples,
                                                       const double* __restrict__ x, double kc,
                                                       double dhat, double* __restrict__ partials,
                                                       int* __restrict__ nonfinite) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
    double in[14], a[1];
    fill_contact<double>(tuples + 4 * c, x, kc, dhat, in);
    ipc_point_plane_act_s_E<double>(in, a);
    if (!BRANCH && !(a[0] > 0.0)) continue;
    if (!(a[0] < dhat)) {
      acc = INFINITY;
      continue;
    }
    double e[1];
    if (BRANCH)
      ipc_point_plane_cond_s_E<double>(in, e);
    else
      ipc_point_plane_s_E<double>(in, e);
    acc += e[0];
  }
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s;
    if (!isfinite(s)) *nonfinite = 1;
  }
}

// Host side of the kind dispatch: f(std::integral_constant<int, KIND>) for a
// set of kind `kind` (validated at mesh creation); higher-order tets have
// kernels of their own (host_with_order) and are not dispatched here.
template <typename F>
static void host_with_kind(int kind, F&& f) {
  switch (kind) {
    case SYMX_SNH_TET4: f(std::integral_constant<int, SYMX_SNH_TET4>{}); break;
    case SYMX_STVK_TRI3: f(std::integral_constant<int, SYMX_STVK_TRI3>{}); break;
    case SYMX_HINGE4: f(std::integral_constant<int, SYMX_HINGE4>{}); break;
    case SYMX_NH_TET4: f(std::integral_constant<int, SYMX_NH_TET4>{}); break;
    case SYMX_STVK_TET4: f(std::integral_constant<int, SYMX_STVK_TET4>{}); break;
    case SYMX_FCR_TET4: f(std::integral_constant<int, SYMX_FCR_TET4>{}); break;
    case SYMX_ARAP_TET4: f(std::integral_constant<int, SYMX_ARAP_TET4>{}); break;
    default: break;
  }
}

// f(std::integral_constant<int, K>) for a set of quadratic (K = 10) or cubic
// (K = 20) tets; nothing for any other kind.
template <typename F>
static void host_with_order(int kind, F&& f) {
  if (kind == SYMX_SNH_TET10) f(std::integral_constant<int, 10>{});
  if (kind == SYMX_SNH_TET20) f(std::integral_constant<int, 20>{});
}

static int grid_for(int64_t work, int per_block, int cap = 16384) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

#define LAUNCH_CHECK(what)                                          \
  do {                                                              \
    hipError_t e_ = hipGetLastError();                              \
    if (e_ != hipSuccess) return hip_check(e_, what);              \
  } while (0)

#define TRY(expr)                     \
  do {                                \
    symx_status s_ = (expr);          \
    if (s_ != SYMX_OK) return s_;     \
  } while (0)

symx_status launch_energy(Mesh& m, const double* x, const double* xt, double dt, int precision,
                          double* E_dev) {
  const char* PNAME = "energy";
  const SetsDev sd = m.sets_dev();
  int off = 0;
  for (int s = 0; s < sd.n; ++s) {
    const int G = grid_for(sd.s[s].n_elem, 256, 8192);
    host_with_order(sd.s[s].kind, [&](auto kc) {
      constexpr int K = decltype(kc)::value;
      if (precision == SYMX_F32)
        SYMX_LAUNCH(m, PNAME, (k_energy_ho<K, float>), dim3(G), dim3(256), 0, sd.s[s], x, m.X,
                    m.partials + off, m.nonfinite);
      else
        SYMX_LAUNCH(m, PNAME, (k_energy_ho<K, double>), dim3(G), dim3(256), 0, sd.s[s], x, m.X,
                    m.partials + off, m.nonfinite);
    });
    host_with_kind(sd.s[s].kind, [&](auto kc) {
      constexpr int KIND = decltype(kc)::value;
      if (precision == SYMX_F32)
        SYMX_LAUNCH(m, PNAME, (k_energy_set<float, KIND>), dim3(G), dim3(256), 0, sd.s[s], x,
                    m.X, m.partials + off, m.nonfinite);
      else
        SYMX_LAUNCH(m, PNAME, (k_energy_set<double, KIND>), dim3(G), dim3(256), 0, sd.s[s], x,
                    m.X, m.partials + off, m.nonfinite);
    });
    LAUNCH_CHECK("k_energy_set");
    off += G;
  }
  if (m.contacts && m.contacts->kind >= 0) {
    // the dynamic element set, after the static sets
    const SetDev S = m.dyn_dev();
    const int G = grid_for(S.n_elem, 256, 8192);
    host_with_kind(S.kind, [&](auto kc) {
      constexpr int KIND = decltype(kc)::value;
      if (precision == SYMX_F32)
        SYMX_LAUNCH(m, PNAME, (k_energy_set<float, KIND>), dim3(G), dim3(256), 0, S, x, m.X,
                    m.partials + off, m.nonfinite);
      else
        SYMX_LAUNCH(m, PNAME, (k_energy_set<double, KIND>), dim3(G), dim3(256), 0, S, x, m.X,
                    m.partials + off, m.nonfinite);
    });
    LAUNCH_CHECK("k_energy_set");
    off += G;
  } else if (m.contacts) {
    const Contacts& c = *m.contacts;
    const int G = grid_for(c.n, 256, 8192);
    if (m.contact_mode == SYMX_CONTACT_BRANCH)
      SYMX_LAUNCH(m, "contact_energy", k_contact_energy<true>, dim3(G), dim3(256), 0, c.n,
                  c.tuples, x, c.kc, c.dhat, m.partials + off, m.nonfinite);
    else
      SYMX_LAUNCH(m, "contact_energy", k_contact_energy<false>, dim3(G), dim3(256), 0, c.n,
                  c.tuples, x, c.kc, c.dhat, m.partials + off, m.nonfinite);
    LAUNCH_CHECK("k_contact_energy");
    off += G;
  }
  if (xt) {
    const int G = grid_for(m.N, 256, 8192);
    SYMX_LAUNCH(m, PNAME, k_energy_inertia, dim3(G), dim3(256), 0, m.N, x, xt, m.mass, dt,
                       m.partials + off, m.nonfinite);
    LAUNCH_CHECK("k_energy_inertia");
    off += G;
  }
  SYMX_LAUNCH(m, "reduce", k_reduce_checked, dim3(1), dim3(256), 0, m.partials, off, E_dev,
                     m.nonfinite);
  LAUNCH_CHECK("k_reduce_checked");
  return SYMX_OK;
}

template <typename T>
static symx_status elem_eval_t(Mesh& m, int set, const double* x, void* E, void* g, void* H) {
  const char* PNAME = "elem_eval";
  const SetsDev sd = m.sets_dev();
  const SetDev& S = sd.s[set];
  const int G = grid_for(S.n_elem, 128, 65535);
  if (S.n_elem == 0) return SYMX_OK;
  host_with_order(S.kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    SYMX_LAUNCH(m, PNAME, (k_elem_eval_ho<K, T>), dim3(grid_for(K * S.n_elem, 64, 65535)),
                dim3(64), 0, S, x, m.X, (T*)E, (T*)g, (T*)H);
  });
  host_with_kind(S.kind, [&](auto kc) {
    constexpr int KIND = decltype(kc)::value;
    SYMX_LAUNCH(m, PNAME, (k_elem_eval<T, KIND>), dim3(G), dim3(128), 0, S, x, m.X, (T*)E,
                (T*)g, (T*)H);
  });
  LAUNCH_CHECK("k_elem_eval");
  return SYMX_OK;
}

symx_status launch_elem_eval(Mesh& m, int set, const double* x, int want, int precision, void* E,
                             void* g, void* H) {
  (void)want;
  if (precision == SYMX_F32) return elem_eval_t<float>(m, set, x, E, g, H);
  return elem_eval_t<double>(m, set, x, E, g, H);
}

symx_status launch_lagged_rotations(Mesh& m, const double* x) {
  const char* PNAME = "lagged_rotations";
  const SetsDev sd = m.sets_dev();
  for (int s = 0; s < sd.n; ++s) {
    const SetDev& S = sd.s[s];
    if (!kind_has_rotation(S.kind) || S.n_elem == 0) continue;
    SYMX_LAUNCH(m, PNAME, k_lagged_rotations, dim3(grid_for(S.n_elem, 256)), dim3(256), 0,
                S.n_elem, S.conn, x, m.X, m.sets[s].d_rot64, m.sets[s].d_rot32);
    LAUNCH_CHECK("k_lagged_rotations");
  }
  return SYMX_OK;
}

symx_status launch_incidence_positions(Mesh& m, int* inc_pos) {
  const char* PNAME = "incidence_positions";
  SetOffsets off{};
  int64_t acc = 0;
  for (size_t s = 0; s < m.sets.size(); ++s) {
    off.first[s] = acc;
    acc += m.sets[s].n_elem * m.sets[s].k;
  }
  SYMX_LAUNCH(m, PNAME, k_incidence_positions, dim3(grid_for(m.n_inc, 256)), dim3(256), 0,
              m.n_inc, m.inc_code, m.sets_dev(), off, inc_pos);
  LAUNCH_CHECK("k_incidence_positions");
  return SYMX_OK;
}

symx_status launch_incidence_rows_projected(Mesh& m, const double* x, int precision, int mode,
                                            const int* inc_pos, void* rows) {
  const char* PNAME = "elem_rows_projected";
  const SetsDev sd = m.sets_dev();
  int64_t first = 0;
  for (int s = 0; s < sd.n; ++s) {
    const SetDev& S = sd.s[s];
    const int* ip = inc_pos + first;
    first += S.n_elem * S.k;
    if (S.n_elem == 0) continue;
    const int G = grid_for(S.n_elem, 64, 65535);
    if (mode == 2 && S.kind == SYMX_SNH_TET4) {
      if (precision == SYMX_F32)
        SYMX_LAUNCH(m, "elem_rows_filtered", k_elem_rows_filtered<float>, dim3(G), dim3(64), 0, S,
                    x, m.X, ip, (float*)rows);
      else
        SYMX_LAUNCH(m, "elem_rows_filtered", k_elem_rows_filtered<double>, dim3(G), dim3(64), 0,
                    S, x, m.X, ip, (double*)rows);
      LAUNCH_CHECK("k_elem_rows_filtered");
      continue;
    }
    host_with_kind(S.kind, [&](auto kc) {
      constexpr int KIND = decltype(kc)::value;
      if (precision == SYMX_F32)
        SYMX_LAUNCH(m, PNAME, k_elem_rows_projected32<KIND>, dim3(G), dim3(64), 0, S, x, m.X, ip,
                    (float*)rows, 30, 2e-7f);
      else
        SYMX_LAUNCH(m, PNAME, k_elem_rows_projected64<KIND>, dim3(G), dim3(64), 0, S, x, m.X, ip,
                    (double*)rows, 30, 1e-15);
    });
    LAUNCH_CHECK("k_elem_rows_projected");
  }
  return SYMX_OK;
}

symx_status launch_elem_filtered(Mesh& m, int set, const double* x, int precision, void* E,
                                 void* g, void* H) {
  const char* PNAME = "elem_filtered";
  const SetDev S = m.sets_dev().s[set];
  if (S.n_elem == 0) return SYMX_OK;
  const int G = grid_for(S.n_elem, 64, 65535);
  if (precision == SYMX_F32)
    SYMX_LAUNCH(m, PNAME, k_elem_filtered<float>, dim3(G), dim3(64), 0, S, x, m.X, (float*)E,
                (float*)g, (float*)H);
  else
    SYMX_LAUNCH(m, PNAME, k_elem_filtered<double>, dim3(G), dim3(64), 0, S, x, m.X, (double*)E,
                (double*)g, (double*)H);
  LAUNCH_CHECK("k_elem_filtered");
  return SYMX_OK;
}

symx_status launch_project(Mesh& m, int precision, void* H, int64_t n, int dim) {
  const char* PNAME = "project_psd";
  if (n == 0) return SYMX_OK;
  if (dim != 9 && dim != 12) {
    set_error("projection supports 9x9 and 12x12 element Hessians");
    return SYMX_ERR_INVALID_ARG;
  }
  // stop when the off-diagonal norm is below tol times the matrix norm
  const int G = grid_for(n, 64, 65535);
  if (precision == SYMX_F32) {
    if (dim == 12)
      SYMX_LAUNCH(m, PNAME, k_project_psd32<4>, dim3(G), dim3(64), 0, (float*)H, n, 30,
                  2e-7f);
    else
      SYMX_LAUNCH(m, PNAME, k_project_psd32<3>, dim3(G), dim3(64), 0, (float*)H, n, 30,
                  2e-7f);
  } else {
    if (dim == 12)
      SYMX_LAUNCH(m, PNAME, k_project_psd64<4>, dim3(G), dim3(64), 0, (double*)H, n, 30,
                  1e-15);
    else
      SYMX_LAUNCH(m, PNAME, k_project_psd64<3>, dim3(G), dim3(64), 0, (double*)H, n, 30,
                  1e-15);
  }
  LAUNCH_CHECK("k_project_psd");
  return SYMX_OK;
}

template <typename T, uint32_t KMASK>
static void row_assemble_launch(Mesh& m, const char* PNAME, dim3 grid, dim3 block,
                                const RowArgs<T>& A, bool want_g, bool want_H) {
  if (want_H && want_g) {
    SYMX_LAUNCH(m, PNAME, (k_row_assemble_fast<T, true, kRowEval, KMASK>), grid, block, 0, A);
  } else if (want_H) {
    SYMX_LAUNCH(m, PNAME, (k_row_assemble_fast<T, false, kRowEval, KMASK>), grid, block, 0, A);
  } else {
    SYMX_LAUNCH(m, PNAME, (k_row_gradient<T, KMASK>), grid, block, 0, A);
  }
}

template <typename T>
static symx_status row_assemble_t(Mesh& m, const double* x, const double* xt, double dt,
                                  bool want_g, bool want_H, bool dirichlet,
                                  const void* inc_rows, bool filter, double* g_out, void* dinv,
                                  float* dinv_lo, bool half) {
  RowArgs<T> A;
  A.sets = m.sets_dev();
  A.x = x;
  A.X = m.X;
  A.xt = xt;
  A.mass = m.mass;
  A.inv_dt2 = xt ? 1.0 / (dt * dt) : 0.0;
  A.fixed = dirichlet ? m.fixed : nullptr;
  A.batch_row = m.batch_row;
  A.row_ptr = m.row_ptr;
  A.col_idx = m.col_idx;
  A.diag_pos = m.diag_pos;
  A.inc_ptr = m.inc_ptr;
  A.inc_code = m.inc_code;
  A.blk_info = m.blk_info;
  A.centry = m.centry;
  A.batch_entry = m.batch_entry;
  A.nnzb = m.nnzb;
  T* const v = (T*)(sizeof(T) == 4 ? (half ? (void*)m.lvals32 : (void*)m.vals32)
                                    : (half ? (void*)m.lvals64 : (void*)m.vals64));
  // float32 copies written by the float64 kernel itself (not by the
  // higher-order kernels, whose copies are rounded afterwards)
  float* const v_lo = want_H && dinv_lo && !m.ho ? (half ? m.lvals32 : m.vals32) : nullptr;
  A.vals = want_H && !half ? v : nullptr;
  A.vals_lo = half ? nullptr : v_lo;
  A.lrow_ptr = m.lrow_ptr;
  A.nnzl = m.nnzl;
  A.lvals = want_H && half ? v : nullptr;
  A.lvals_lo = half ? v_lo : nullptr;
  A.g = g_out;
  A.dinv = (T*)dinv;
  A.dinv_lo = want_H && !m.ho ? dinv_lo : nullptr;
  A.nonfinite = m.nonfinite;
  A.inc_rows = (const T*)inc_rows;
  A.inc_nodes = m.inc_nodes;
  if ((want_g && !g_out) || (!want_g && !want_H) || (want_H && !v) ||
      (want_H && dinv_lo && !m.ho && !v_lo)) {
    set_error("row assembly without an output");
    return SYMX_ERR_INVALID_ARG;
  }
  const dim3 grid(m.n_batch), block(kRowWG);
  const char* PNAME = want_H ? (want_g ? "row_assemble_gH" : "row_assemble_H") : "row_assemble_g";
  // Kernels compiled for the kinds the mesh holds keep their register count
  // (and occupancy) at that of the heaviest kind present: one kind alone, the
  // solid + shell kinds, or all kinds for any other mix.  The projected path
  // reads records and evaluates no element.
  uint32_t kinds = 0;
  for (const SetHost& s : m.sets) kinds |= 1u << s.kind;
  if (m.ho) {
    host_with_order(m.sets[0].kind, [&](auto kc) {
      constexpr int K = decltype(kc)::value;
      if (want_H && want_g)
        SYMX_LAUNCH(m, PNAME, (k_row_assemble_ho<K, T, true, true>), grid, block, 0, A);
      else if (want_H)
        SYMX_LAUNCH(m, PNAME, (k_row_assemble_ho<K, T, false, true>), grid, block, 0, A);
      else
        SYMX_LAUNCH(m, PNAME, (k_row_assemble_ho<K, T, true, false>), grid, block, 0, A);
    });
  } else if (filter && want_H) {
    if (want_g)
      SYMX_LAUNCH(m, PNAME, (k_row_assemble_fast<T, true, kRowFilter, 0u>), grid, block, 0, A);
    else
      SYMX_LAUNCH(m, PNAME, (k_row_assemble_fast<T, false, kRowFilter, 0u>), grid, block, 0, A);
  } else if (inc_rows && want_H) {
    if (want_g)
      SYMX_LAUNCH(m, PNAME, (k_row_assemble_fast<T, true, kRowRecords, 0u>), grid, block, 0, A);
    else
      SYMX_LAUNCH(m, PNAME, (k_row_assemble_fast<T, false, kRowRecords, 0u>), grid, block, 0, A);
  } else if (kinds == kKindsSnh)
    row_assemble_launch<T, kKindsSnh>(m, PNAME, grid, block, A, want_g, want_H);
  else if ((kinds & ~kKindsShell) == 0)
    row_assemble_launch<T, kKindsShell>(m, PNAME, grid, block, A, want_g, want_H);
  else if (kinds == 1u << SYMX_NH_TET4)
    row_assemble_launch<T, 1u << SYMX_NH_TET4>(m, PNAME, grid, block, A, want_g, want_H);
  else if (kinds == 1u << SYMX_STVK_TET4)
    row_assemble_launch<T, 1u << SYMX_STVK_TET4>(m, PNAME, grid, block, A, want_g, want_H);
  else if (kinds == 1u << SYMX_FCR_TET4)
    row_assemble_launch<T, 1u << SYMX_FCR_TET4>(m, PNAME, grid, block, A, want_g, want_H);
  else if (kinds == 1u << SYMX_ARAP_TET4)
    row_assemble_launch<T, 1u << SYMX_ARAP_TET4>(m, PNAME, grid, block, A, want_g, want_H);
  else
    row_assemble_launch<T, kKindsAll>(m, PNAME, grid, block, A, want_g, want_H);
  LAUNCH_CHECK("k_row_assemble");
  return SYMX_OK;
}

symx_status launch_row_assemble(Mesh& m, const double* x, const double* xt, double dt, bool want_g,
                                bool want_H, int precision, bool dirichlet,
                                const void* inc_rows, bool filter, double* g_out, void* dinv,
                                float* dinv_lo, bool half) {
  if (precision == SYMX_F32)
    return row_assemble_t<float>(m, x, xt, dt, want_g, want_H, dirichlet, inc_rows, filter, g_out,
                                 dinv, nullptr, half);
  if (dinv_lo && !dinv) {
    set_error("row assembly: float32 copies need the inverses");
    return SYMX_ERR_INVALID_ARG;
  }
  return row_assemble_t<double>(m, x, xt, dt, want_g, want_H, dirichlet, inc_rows, filter, g_out,
                                dinv, dinv_lo, half);
}

symx_status launch_x_tilde(Mesh& m, const double* x, const double* v, double dt, const double g[3],
                           double* xt) {
  const char* PNAME = "x_tilde";
  const int64_t n = 3 * m.N;
  SYMX_LAUNCH(m, PNAME, k_x_tilde, dim3(grid_for(n, 256)), dim3(256), 0, n, x, v, dt, g[0],
                     g[1], g[2], xt);
  LAUNCH_CHECK("k_x_tilde");
  return SYMX_OK;
}

symx_status launch_dot64(Mesh& m, const double* a, const double* b, int64_t n, double* out_dev) {
  const char* PNAME = "dot64";
  const int G = grid_for(n, 256, 1024);
  SYMX_LAUNCH(m, PNAME, k_dot64, dim3(G), dim3(256), 0, n, a, b, m.partials);
  SYMX_LAUNCH(m, "reduce", k_reduce_checked, dim3(1), dim3(256), 0, m.partials, G, out_dev,
                     m.nonfinite);
  LAUNCH_CHECK("k_dot64");
  return SYMX_OK;
}

symx_status launch_lincomb64(Mesh& m, double* out, const double* a, const double* b, double beta,
                             int64_t n) {
  const char* PNAME = "lincomb64";
  SYMX_LAUNCH(m, PNAME, k_lincomb64, dim3(grid_for(n, 256)), dim3(256), 0, n, out, a, b,
                     beta);
  LAUNCH_CHECK("k_lincomb64");
  return SYMX_OK;
}

symx_status launch_velocity(Mesh& m, double* v, const double* xn, const double* xo, double inv_dt,
                            int64_t n) {
  const char* PNAME = "velocity";
  SYMX_LAUNCH(m, PNAME, k_velocity, dim3(grid_for(n, 256)), dim3(256), 0, n, v, xn, xo,
                     inv_dt);
  LAUNCH_CHECK("k_velocity");
  return SYMX_OK;
}

symx_status launch_round_values(Mesh& m, bool mesh_vals, const double* dinv64, float* dinv32,
                                int64_t n_inv) {
  const char* PNAME = "round_values";
  if (mesh_vals && (!m.lvals64 || !m.lvals32)) {
    set_error("round_values: the float64 and float32 value arrays must exist");
    return SYMX_ERR_INVALID_ARG;
  }
  const int64_t nv = 9 * m.nnzl;
  if (mesh_vals)
    SYMX_LAUNCH(m, PNAME, k_round_f64, dim3(grid_for(nv, 256, 8192)), dim3(256), 0, nv,
                (const double*)m.lvals64, m.lvals32);
  if (m.contacts && m.contacts->nnzb > 0) {
    Contacts& c = *m.contacts;
    if (c.vals_cap32 < c.nnzb) {
      dev_free(m.pool, c.vals32);
      c.vals32 = nullptr;
      c.vals_cap32 = 0;
      TRY(dev_alloc(m.pool, (void**)&c.vals32, 9 * c.nnzb * sizeof(float)));
      c.vals_cap32 = c.nnzb;
    }
    const int64_t nc = 9 * c.nnzb;
    SYMX_LAUNCH(m, PNAME, k_round_f64, dim3(grid_for(nc, 256, 8192)), dim3(256), 0, nc,
                (const double*)c.vals64, c.vals32);
  }
  if (dinv64 && dinv32)
    SYMX_LAUNCH(m, PNAME, k_round_f64, dim3(grid_for(n_inv, 256, 8192)), dim3(256), 0, n_inv,
                dinv64, dinv32);
  LAUNCH_CHECK("k_round_f64");
  return SYMX_OK;
}

symx_status launch_check_finite(Mesh& m, const double* a, int64_t n) {
  const char* PNAME = "check_finite";
  SYMX_LAUNCH(m, PNAME, k_check_finite, dim3(grid_for(n, 256, 4096)), dim3(256), 0, n, a,
                     m.nonfinite);
  LAUNCH_CHECK("k_check_finite");
  return SYMX_OK;
}

// ---------------------------------------------------------------------------
// PCG driver pieces (called from symx_newton.cpp)
// ---------------------------------------------------------------------------
symx_status launch_pcg_init(Mesh& m, int precision, const PcgBuffers& B, const double* b,
                            double tol2, int max_iter) {
  const char* PNAME = "pcg_init";
  const int gu = pcg_gu(m.N);
  if (precision == SYMX_F64)
    SYMX_LAUNCH(m, PNAME, (k_pcg_init<double, double>), dim3(gu), dim3(256), 0, m.N, b,
                       (const double*)B.Dinv, (double*)B.xs, (double*)B.r, (double*)B.z,
                       (double*)B.p, (double*)B.q, m.partials, m.scalars, tol2, max_iter);
  else
    SYMX_LAUNCH(m, PNAME, (k_pcg_init<float, double>), dim3(gu), dim3(256), 0, m.N, b,
                       (const float*)B.Dinv, (float*)B.xs, (float*)B.r, (float*)B.z, (float*)B.p,
                       (float*)B.q, m.partials, m.scalars, tol2, max_iter);
  LAUNCH_CHECK("k_pcg_init");
  return SYMX_OK;
}

// The mesh's half-stored solver matrix in precision T.
template <typename T>
static HalfBsr<T> half_bsr(const Mesh& m) {
  return HalfBsr<T>{m.row_ptr, m.cv,
                    (const T*)(sizeof(T) == 4 ? (const void*)m.lvals32 : (const void*)m.lvals64),
                    m.nnzl};
}

// Enqueue iterations k0 .. k0+n_iter-1 (each: SpMV kernel, update kernel).
symx_status launch_pcg_iters(Mesh& m, int precision, const PcgBuffers& B, int k0, int n_iter) {
  const int gs = pcg_gs(m.N), gu = pcg_gu(m.N);
  const Contacts* cs = m.contacts;
  const DynBsr<double> C64{cs ? cs->row_ptr : nullptr, cs ? cs->col_idx : nullptr,
                           cs ? cs->vals64 : nullptr, cs ? cs->nnzb : 0};
  const DynBsr<float> C32{cs ? cs->row_ptr : nullptr, cs ? cs->col_idx : nullptr,
                          cs ? cs->vals32 : nullptr, cs ? cs->nnzb : 0};
  const HalfBsr<double> H64 = half_bsr<double>(m);
  const HalfBsr<float> H32 = half_bsr<float>(m);
  for (int it = k0; it < k0 + n_iter; ++it) {
    {
      const char* PNAME = "pcg_spmv";
      if (precision == SYMX_F64) {
        if (cs)
          SYMX_LAUNCH(m, PNAME, (k_pcg_spmv<double, true>), dim3(gs), dim3(256), 0, it, m.N, H64,
                      (const double*)B.z, (double*)B.p, (double*)B.q, m.partials, m.scalars, gu,
                      C64);
        else
          SYMX_LAUNCH(m, PNAME, (k_pcg_spmv<double, false>), dim3(gs), dim3(256), 0, it, m.N, H64,
                      (const double*)B.z, (double*)B.p, (double*)B.q, m.partials, m.scalars, gu,
                      C64);
      } else {
        if (cs)
          SYMX_LAUNCH(m, PNAME, (k_pcg_spmv<float, true>), dim3(gs), dim3(256), 0, it, m.N, H32,
                      (const float*)B.z, (float*)B.p, (float*)B.q, m.partials, m.scalars, gu, C32);
        else
          SYMX_LAUNCH(m, PNAME, (k_pcg_spmv<float, false>), dim3(gs), dim3(256), 0, it, m.N, H32,
                      (const float*)B.z, (float*)B.p, (float*)B.q, m.partials, m.scalars, gu, C32);
      }
    }
    {
      const char* PNAME = "pcg_update";
      if (precision == SYMX_F64)
        SYMX_LAUNCH(m, PNAME, k_pcg_update<double>, dim3(gu), dim3(256), 0, it, m.N,
                           (const double*)B.Dinv, (double*)B.xs, (double*)B.r, (double*)B.z,
                           (const double*)B.p, (const double*)B.q, m.partials, m.scalars, gs);
      else
        SYMX_LAUNCH(m, PNAME, k_pcg_update<float>, dim3(gu), dim3(256), 0, it, m.N,
                           (const float*)B.Dinv, (float*)B.xs, (float*)B.r, (float*)B.z,
                           (const float*)B.p, (const float*)B.q, m.partials, m.scalars, gs);
    }
  }
  LAUNCH_CHECK("k_pcg");
  return SYMX_OK;
}

// Batched PCG chunks of several meshes (the serving loop): the items are
// grouped by precision and by whether the mesh has contacts; per iteration,
// one SpMV and one update launch per group.  Each item's workgroups keep the
// mesh's own grids (SpMV ranges start at multiples of 8).
constexpr int kBatchGroups = 4;  // (float, double) x (no contacts, contacts)
symx_status pcg_batch_tables_alloc(PcgBatchTables& t, int cap) {
  const size_t bytes = size_t(kBatchGroups) * cap * sizeof(PcgScene<double>);
  TRY(hip_check(hipMalloc(&t.dev, bytes), "hipMalloc(batch tables)"));
  TRY(hip_check(hipHostMalloc(&t.host, bytes), "hipHostMalloc(batch tables)"));
  t.cap = cap;
  return SYMX_OK;
}

void pcg_batch_tables_free(PcgBatchTables& t) {
  if (t.dev) (void)hipFree(t.dev);
  if (t.host) (void)hipHostFree(t.host);
  t = PcgBatchTables();
}

template <typename T>
static PcgScene<T> pcg_scene(const PcgBatchItem& it) {
  const Mesh& m = *it.m;
  const Contacts* cs = m.contacts;
  PcgScene<T> sc;
  sc.N = m.N;
  sc.H = half_bsr<T>(m);
  sc.C = DynBsr<T>{cs ? cs->row_ptr : nullptr, cs ? cs->col_idx : nullptr,
                   cs ? (const T*)(sizeof(T) == 4 ? (const void*)cs->vals32 : (const void*)cs->vals64)
                      : nullptr,
                   cs ? cs->nnzb : 0};
  sc.Dinv = (const T*)it.B.Dinv;
  sc.xs = (T*)it.B.xs;
  sc.r = (T*)it.B.r;
  sc.z = (T*)it.B.z;
  sc.p = (T*)it.B.p;
  sc.q = (T*)it.B.q;
  sc.P = m.partials;
  sc.S = m.scalars;
  sc.gs = pcg_gs(m.N);
  sc.gu = pcg_gu(m.N);
  sc.k0 = it.k0;
  sc.n = it.n;
  sc.blk_s = sc.blk_u = 0;
  return sc;
}

template <typename T, bool DYN>
static symx_status pcg_batch_group(hipStream_t stream, PcgBatchTables& t, int group,
                                   const std::vector<const PcgBatchItem*>& items, int* n_max,
                                   const PcgScene<T>** dev_tab, int* gs_total, int* gu_total) {
  PcgScene<T>* host = (PcgScene<T>*)((char*)t.host + size_t(group) * t.cap * sizeof(PcgScene<double>));
  PcgScene<T>* dev = (PcgScene<T>*)((char*)t.dev + size_t(group) * t.cap * sizeof(PcgScene<double>));
  int bs = 0, bu = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    host[i] = pcg_scene<T>(*items[i]);
    host[i].blk_s = bs;
    host[i].blk_u = bu;
    bs += host[i].gs;  // pcg_gs is a multiple of 8
    bu += host[i].gu;
    *n_max = std::max(*n_max, host[i].n);
  }
  TRY(hip_check(hipMemcpyAsync(dev, host, items.size() * sizeof(PcgScene<T>),
                               hipMemcpyHostToDevice, stream),
                "hipMemcpyAsync(batch table)"));
  *dev_tab = dev;
  *gs_total = bs;
  *gu_total = bu;
  return SYMX_OK;
}

symx_status launch_pcg_batch(hipStream_t stream, PcgBatchTables& t, const PcgBatchItem* items,
                             int n_items) {
  if (n_items > t.cap) {
    set_error("batched PCG: more meshes than the batch tables hold");
    return SYMX_ERR_INVALID_ARG;
  }
  std::vector<const PcgBatchItem*> grp[kBatchGroups];
  for (int i = 0; i < n_items; ++i) {
    const bool f64 = items[i].precision == SYMX_F64;
    const bool dyn = items[i].m->contacts != nullptr;
    grp[(f64 ? 2 : 0) + (dyn ? 1 : 0)].push_back(&items[i]);
  }
  int n_max = 0;
  const PcgScene<float>* tf[2] = {nullptr, nullptr};
  const PcgScene<double>* td[2] = {nullptr, nullptr};
  int gs[kBatchGroups] = {}, gu[kBatchGroups] = {};
  if (!grp[0].empty()) TRY((pcg_batch_group<float, false>(stream, t, 0, grp[0], &n_max, &tf[0], &gs[0], &gu[0])));
  if (!grp[1].empty()) TRY((pcg_batch_group<float, true>(stream, t, 1, grp[1], &n_max, &tf[1], &gs[1], &gu[1])));
  if (!grp[2].empty()) TRY((pcg_batch_group<double, false>(stream, t, 2, grp[2], &n_max, &td[0], &gs[2], &gu[2])));
  if (!grp[3].empty()) TRY((pcg_batch_group<double, true>(stream, t, 3, grp[3], &n_max, &td[1], &gs[3], &gu[3])));
  for (int j = 0; j < n_max; ++j) {
    if (tf[0]) hipLaunchKernelGGL((k_pcg_spmv_multi<float, false>), dim3(gs[0]), dim3(256), 0, stream, j, tf[0], (int)grp[0].size());
    if (tf[1]) hipLaunchKernelGGL((k_pcg_spmv_multi<float, true>), dim3(gs[1]), dim3(256), 0, stream, j, tf[1], (int)grp[1].size());
    if (td[0]) hipLaunchKernelGGL((k_pcg_spmv_multi<double, false>), dim3(gs[2]), dim3(256), 0, stream, j, td[0], (int)grp[2].size());
    if (td[1]) hipLaunchKernelGGL((k_pcg_spmv_multi<double, true>), dim3(gs[3]), dim3(256), 0, stream, j, td[1], (int)grp[3].size());
    if (tf[0]) hipLaunchKernelGGL((k_pcg_update_multi<float>), dim3(gu[0]), dim3(256), 0, stream, j, tf[0], (int)grp[0].size());
    if (tf[1]) hipLaunchKernelGGL((k_pcg_update_multi<float>), dim3(gu[1]), dim3(256), 0, stream, j, tf[1], (int)grp[1].size());
    if (td[0]) hipLaunchKernelGGL((k_pcg_update_multi<double>), dim3(gu[2]), dim3(256), 0, stream, j, td[0], (int)grp[2].size());
    if (td[1]) hipLaunchKernelGGL((k_pcg_update_multi<double>), dim3(gu[3]), dim3(256), 0, stream, j, td[1], (int)grp[3].size());
  }
  LAUNCH_CHECK("k_pcg_multi");
  return SYMX_OK;
}

symx_status launch_accumulate(Mesh& m, int precision, double* dx, const void* xs) {
  const char* PNAME = "accumulate";
  const int64_t n = 3 * m.N;
  if (precision == SYMX_F64)
    SYMX_LAUNCH(m, PNAME, k_accumulate<double>, dim3(grid_for(n, 256)), dim3(256), 0, n, dx,
                       (const double*)xs);
  else
    SYMX_LAUNCH(m, PNAME, k_accumulate<float>, dim3(grid_for(n, 256)), dim3(256), 0, n, dx,
                       (const float*)xs);
  LAUNCH_CHECK("k_accumulate");
  return SYMX_OK;
}

template <typename T>
static symx_status contact_assemble_t(Mesh& m, const double* x, bool want_g, bool want_H,
                                      bool project, bool dirichlet, double* g, T* dinv) {
  Contacts& c = *m.contacts;
  const bool branch = m.contact_mode == SYMX_CONTACT_BRANCH;
  if (!branch && c.kind < 0) {
    const int n_chunks = (int)((c.n + kContactChunk - 1) / kContactChunk);
    SYMX_LAUNCH(m, "contact_activate", k_contact_activate, dim3(n_chunks), dim3(256), 0, c.n,
                c.tuples, x, c.kc, c.dhat, c.flag, c.chunk_count);
    SYMX_LAUNCH(m, "contact_scan", k_contact_scan, dim3(1), dim3(64), 0, n_chunks, c.chunk_count,
                c.n_active);
    SYMX_LAUNCH(m, "contact_compact", k_contact_compact, dim3(n_chunks), dim3(256), 0, c.n,
                c.flag, c.chunk_count, c.slot, c.act);
  }
  const size_t eb = size_t(c.n) * kContactVals * sizeof(T);
  if (c.eval_bytes < eb) {
    dev_free(m.pool, c.eval);
    c.eval = nullptr;
    c.eval_bytes = 0;
    TRY(dev_alloc(m.pool, &c.eval, eb));
    c.eval_bytes = eb;
  }
  T* eg = (T*)c.eval;
  T* eH = eg + 12 * c.n;
  if (c.kind >= 0) {
    const SetDev S = m.dyn_dev();
    host_with_kind(c.kind, [&](auto kc) {
      constexpr int KIND = decltype(kc)::value;
      if constexpr (KIND == SYMX_SNH_TET4 || KIND == SYMX_NH_TET4 || KIND == SYMX_STVK_TET4 ||
                    KIND == SYMX_HINGE4)
        SYMX_LAUNCH(m, "dyn_eval", (k_dyn_eval<T, KIND>), dim3(grid_for(c.n, 128, 8192)),
                    dim3(128), 0, S, x, m.X, eg, eH, c.slot, c.n_active);
    });
  } else if (branch)
    SYMX_LAUNCH(m, "contact_eval", k_contact_eval_branch<T>, dim3(grid_for(c.n, 128, 8192)),
                dim3(128), 0, c.n, c.tuples, x, c.kc, c.dhat, eg, eH, c.slot, c.n_active);
  else
    SYMX_LAUNCH(m, "contact_eval", k_contact_eval<T>, dim3(grid_for(c.n, 128, 8192)), dim3(128),
                0, c.act, c.n_active, c.tuples, x, c.kc, c.dhat, eg, eH);
  if (want_H && project) {
    const int G = grid_for(c.n, 64, 65535);
    if (sizeof(T) == 4)
      SYMX_LAUNCH(m, "contact_project", k_contact_project32, dim3(G), dim3(64), 0, (float*)eH,
                  c.n_active);
    else
      SYMX_LAUNCH(m, "contact_project", k_contact_project64, dim3(G), dim3(64), 0, (double*)eH,
                  c.n_active);
  }
  const uint8_t* fixed = dirichlet ? m.fixed : nullptr;
  if (want_H) {
    T*& vals = *(T**)(sizeof(T) == 4 ? (void*)&c.vals32 : (void*)&c.vals64);
    int64_t& vcap = sizeof(T) == 4 ? c.vals_cap32 : c.vals_cap64;
    if (vcap < c.nnzb) {  // a new candidate list may have more blocks
      dev_free(m.pool, vals);
      vals = nullptr;
      vcap = 0;
      TRY(dev_alloc(m.pool, (void**)&vals, 9 * c.nnzb * sizeof(T)));
      vcap = c.nnzb;
    }
    SYMX_LAUNCH(m, "contact_blocks", k_contact_blocks<T>, dim3(grid_for(c.nnzb, 256)), dim3(256),
                0, c.nnzb, c.blk_row, c.col_idx, c.blk_ptr, c.blk_src, c.slot, eH, fixed, vals);
    if (dinv) {
      // with the inverses, the mesh's blocks are in the solver's half storage
      const T* mv = (const T*)(sizeof(T) == 4 ? (void*)m.lvals32 : (void*)m.lvals64);
      SYMX_LAUNCH(m, "contact_dinv", k_contact_dinv<T>, dim3(grid_for(c.n_gnode, 256)), dim3(256),
                  0, c.n_gnode, c.gnode, c.gdiag, m.row_ptr, m.diag_pos, m.lrow_ptr, mv, m.nnzl,
                  vals, c.nnzb, dinv);
    }
  }
  if (want_g)
    SYMX_LAUNCH(m, "contact_grad", k_contact_grad<T>, dim3(grid_for(c.n_gnode, 256)), dim3(256), 0,
                c.n_gnode, c.gnode, c.gptr, c.gsrc, c.slot, eg, fixed, g, m.nonfinite);
  LAUNCH_CHECK("k_contact");
  return SYMX_OK;
}

symx_status launch_contact_assemble(Mesh& m, const double* x, bool want_g, bool want_H,
                                    bool project, int precision, bool dirichlet, double* g,
                                    void* dinv) {
  if (!m.contacts || (!want_g && !want_H)) return SYMX_OK;
  if (precision == SYMX_F32)
    return contact_assemble_t<float>(m, x, want_g, want_H, project, dirichlet, g, (float*)dinv);
  return contact_assemble_t<double>(m, x, want_g, want_H, project, dirichlet, g, (double*)dinv);
}

symx_status launch_residual64(Mesh& m, int precision, const double* x, const double* b,
                              double* r) {
  const char* PNAME = "residual64";
  const int G = grid_for(m.N * kSpmvLanes, 256, 16384);
  const Contacts* cs = m.contacts;
  const DynBsr<double> C64{cs ? cs->row_ptr : nullptr, cs ? cs->col_idx : nullptr,
                           cs ? cs->vals64 : nullptr, cs ? cs->nnzb : 0};
  const DynBsr<float> C32{cs ? cs->row_ptr : nullptr, cs ? cs->col_idx : nullptr,
                          cs ? cs->vals32 : nullptr, cs ? cs->nnzb : 0};
  if (precision == SYMX_F64) {
    if (cs)
      SYMX_LAUNCH(m, PNAME, (k_residual64<double, true>), dim3(G), dim3(256), 0, m.N,
                  half_bsr<double>(m), x, b, r, C64);
    else
      SYMX_LAUNCH(m, PNAME, (k_residual64<double, false>), dim3(G), dim3(256), 0, m.N,
                  half_bsr<double>(m), x, b, r, C64);
  } else {
    if (cs)
      SYMX_LAUNCH(m, PNAME, (k_residual64<float, true>), dim3(G), dim3(256), 0, m.N,
                  half_bsr<float>(m), x, b, r, C32);
    else
      SYMX_LAUNCH(m, PNAME, (k_residual64<float, false>), dim3(G), dim3(256), 0, m.N,
                  half_bsr<float>(m), x, b, r, C32);
  }
  LAUNCH_CHECK("k_residual64");
  return SYMX_OK;
}

}  // namespace symxi
