// symx_gen: build-time generator of element functions.
//
// Each energy is written once for a single representative element with the
// symbolic scalar type (Sec. 5.1-5.2: energies defined per element on fixed-size
// local inputs, Eq. 5).  The generator differentiates it symbolically, removes
// common subexpressions and emits straight-line code, one line per graph node
// (Sec. 5.2, code generation), as
//   * HIP device templates (float / double) for the library, and
//   * plain C (double) for a test-only CPU library that checks the generator
//     against the hand-derived FP64 oracle.
//
// Variants per energy (the paper's three evaluation levels, Sec. 5.2):
//   NAME_E, NAME_Eg, NAME_EgH      energy / + gradient / + full Hessian, with the
//                                  paper's input layout (e.g. 26 inputs for tet4)
//   NAME_s_E, NAME_s_EgH           same with node 0 at the origin (x0 = X0 = 0):
//                                  the library passes coordinates relative to
//                                  node 0, so single precision keeps the digits
//                                  of the element's edge vectors
//   NAME_row0_g, NAME_row0_gH      gradient of node 0 and Hessian block row 0
//                                  (node 0 at the origin); node a's row is
//                                  obtained by relabelling node a as node 0
//   NAME_rowR_g, NAME_rowR_gHoff   the same for node R (R = 0, and 4 for the
//                                  quadratic tet, whose edge nodes cannot be
//                                  relabelled into a corner)
//
// Usage: symx_gen <output directory>
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "expr.h"

using namespace symx;

namespace {

struct EnergySpec {
  std::string name;
  int n_nodes;        // element nodes (3 coordinates each are the DoFs)
  int n_in;           // total inputs
  int rest_slot;      // first slot of node-0 rest coordinates, or -1
  std::function<S(Graph&, const std::vector<S>&)> energy;
  // linear tets: the density psi(F, inputs) of energy = V psi(F); when set,
  // the Hessian row functions are generated through F (fewer operations
  // than differentiating the energy with respect to the positions)
  std::function<S(const symx::Mat&, const std::vector<S>&)> density = nullptr;
};

Mat cols_minus_first(Graph& g, const std::vector<S>& in, int base, int n_nodes) {
  // columns p_a - p_0 for a = 1..n_nodes-1 of the 3D points in[base + 3a + i]
  Mat M(3, n_nodes - 1, &g);
  for (int a = 1; a < n_nodes; ++a)
    for (int i = 0; i < 3; ++i) M(i, a - 1) = in[base + 3 * a + i] - in[base + i];
  return M;
}

// Stable Neo-Hookean tet4 (App. B, Stable Neo-Hookean branch) with the Lame
// re-parametrisation mu' = 4/3 mu, lambda' = lambda + 5/6 mu; E = V psi(F),
// F = Ds Dm^-1, V = |det Dm| / 6 (Sec. 3.1).
S snh_tet4(Graph& g, const std::vector<S>& in) {
  Mat Ds = cols_minus_first(g, in, 0, 4);
  Mat Dm = cols_minus_first(g, in, 12, 4);
  S mu = in[24], lam = in[25];
  S detDm = det3(Dm);
  S V = abs(detDm) / 6.0;
  Mat F = matmul(Ds, inv3(Dm));
  S mu_ = mu * (4.0 / 3.0);
  S lam_ = lam + mu * (5.0 / 6.0);
  S Ic = frob2(F);
  S J = det3(F);
  S alpha = 1.0 + mu_ / lam_ - mu_ / (4.0 * lam_);
  S psi = 0.5 * mu_ * (Ic - 3.0) + 0.5 * lam_ * pown(J - alpha, 2) - 0.5 * mu_ * log(Ic + 1.0);
  return V * psi;
}

// Deformation gradient and rest volume of a tet4 with inputs x (0..11), X
// (12..23): F = Ds Dm^-1, V = |det Dm| / 6 (Sec. 3.1).
struct TetKinematics {
  Mat F;
  S V;
};
TetKinematics tet_kinematics(Graph& g, const std::vector<S>& in) {
  Mat Ds = cols_minus_first(g, in, 0, 4);
  Mat Dm = cols_minus_first(g, in, 12, 4);
  return {matmul(Ds, inv3(Dm)), abs(det3(Dm)) / 6.0};
}

// Rotation R (row-major, inputs 26..34) of the lagged-rotation materials.
Mat lagged_rotation(Graph& g, const std::vector<S>& in) {
  Mat R(3, 3, &g);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R(i, j) = in[26 + 3 * i + j];
  return R;
}

// Classic Neo-Hookean (App. B, Neo-Hookean branch; Eq. 6 with the sign of
// the log term that makes the rest state stress free):
// psi = mu/2 (Ic - 3) - mu log J + lambda/2 log^2 J.
S nh_density(const Mat& F, const std::vector<S>& in) {
  S mu = in[24], lam = in[25];
  S logJ = log(det3(F));
  return 0.5 * mu * (frob2(F) - 3.0) - mu * logJ + 0.5 * lam * pown(logJ, 2);
}
S nh_tet4(Graph& g, const std::vector<S>& in) {
  TetKinematics k = tet_kinematics(g, in);
  return k.V * nh_density(k.F, in);
}

// Fixed co-rotational (App. B, fixed co-rotational branch) with the rotation
// R held constant over a time step (lagged):
// psi = mu |F - R|^2 + lambda/2 (J - 1)^2.
S fcr_density(const Mat& F, const std::vector<S>& in) {
  Graph& g = *F.v[0].g;
  Mat R = lagged_rotation(g, in);
  S mu = in[24], lam = in[25];
  Mat D(3, 3, &g);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D(i, j) = F(i, j) - R(i, j);
  return mu * frob2(D) + 0.5 * lam * pown(det3(F) - 1.0, 2);
}
S fcr_tet4(Graph& g, const std::vector<S>& in) {
  TetKinematics k = tet_kinematics(g, in);
  return k.V * fcr_density(k.F, in);
}

// As-rigid-as-possible with a volume term (App. B, ARAP branch), R lagged:
// psi = mu/2 (Ic - 2 tr(F^T R) + 3) + lambda/2 (J - 1)^2.
S arap_density(const Mat& F, const std::vector<S>& in) {
  Graph& g = *F.v[0].g;
  Mat R = lagged_rotation(g, in);
  S mu = in[24], lam = in[25];
  S trFR = trace(matmul(transpose(F), R));
  return 0.5 * mu * (frob2(F) - 2.0 * trFR + 3.0) + 0.5 * lam * pown(det3(F) - 1.0, 2);
}
S arap_tet4(Graph& g, const std::vector<S>& in) {
  TetKinematics k = tet_kinematics(g, in);
  return k.V * arap_density(k.F, in);
}

// StVK membrane triangle (App. B, Saint Venant-Kirchhoff branch, on the 3x2
// deformation gradient of a triangle).  Written frame-free: with the rest
// metric G = Dm^T Dm and the current metric C = Ds^T Ds of the two edge
// vectors, F^T F in any orthonormal rest frame is similar to G^-1 C, so
// tr(E) = (tr(G^-1 C) - 2)/2 and |E|^2 = tr((G^-1 C - I)^2)/4; the rest area
// is sqrt(det G)/2 and the energy is thickness * area * psi.
S stvk_tri3(Graph& g, const std::vector<S>& in) {
  Mat Ds = cols_minus_first(g, in, 0, 3);
  Mat Dm = cols_minus_first(g, in, 9, 3);
  S mu = in[18], lam = in[19], h = in[20];
  Mat Gm = matmul(transpose(Dm), Dm);
  Mat Cm = matmul(transpose(Ds), Ds);
  Mat M = matmul(inv2(Gm), Cm);
  S trM = trace(M);
  Mat D(2, 2, &g);
  D(0, 0) = M(0, 0) - 1.0;
  D(0, 1) = M(0, 1);
  D(1, 0) = M(1, 0);
  D(1, 1) = M(1, 1) - 1.0;
  S trD2 = D(0, 0) * D(0, 0) + 2.0 * (D(0, 1) * D(1, 0)) + D(1, 1) * D(1, 1);
  S trE = 0.5 * (trM - 2.0);
  S psi = mu * (0.25 * trD2) + 0.5 * lam * (trE * trE);
  S area = 0.5 * sqrt(det2(Gm));
  return h * area * psi;
}

// Stable Neo-Hookean density (App. B, Stable Neo-Hookean branch) with the Lame
// re-parametrisation mu' = 4/3 mu, lambda' = lambda + 5/6 mu.
S snh_density(const Mat& F, S mu, S lam) {
  S mu_ = mu * (4.0 / 3.0);
  S lam_ = lam + mu * (5.0 / 6.0);
  S Ic = frob2(F);
  S J = det3(F);
  S alpha = 1.0 + mu_ / lam_ - mu_ / (4.0 * lam_);
  return 0.5 * mu_ * (Ic - 3.0) + 0.5 * lam_ * pown(J - alpha, 2) - 0.5 * mu_ * log(Ic + 1.0);
}

// Signed distance of node p (inputs 0..2) to the plane through t0, t1, t2
// (3..11), positive on the side of N = (t1 - t0) x (t2 - t0).
S point_plane_distance(Graph& g, const std::vector<S>& in) {
  (void)g;
  Vec u(3), e1(3), e2(3);
  for (int i = 0; i < 3; ++i) {
    u[i] = in[i] - in[3 + i];
    e1[i] = in[6 + i] - in[3 + i];
    e2[i] = in[9 + i] - in[3 + i];
  }
  Vec N = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
           e1[0] * e2[1] - e1[1] * e2[0]};
  return dot(u, N) / sqrt(dot(N, N));
}

// Contact barrier between a point and a plane (Sec. 5.4, the contact
// potential): -k_c (d - d_hat)^2 ln(d / d_hat), k_c (input 12), d_hat (13).
// It is evaluated only where its activation is positive (Eq. 9).
S ipc_point_plane(Graph& g, const std::vector<S>& in) {
  S d = point_plane_distance(g, in);
  S kc = in[12], dh = in[13];
  return -kc * pown(d - dh, 2) * log(d / dh);
}

// The same barrier with its activation inside the expression: a branch on
// c_e = d_hat - d (Eq. 9; Sec. 5.2, branching) selects the barrier where the
// candidate is active and zero elsewhere.  Differentiation keeps the branch,
// and the generated code takes it with an if/else, so an inactive candidate
// costs the distance and nothing more.
S ipc_point_plane_cond(Graph& g, const std::vector<S>& in) {
  S d = point_plane_distance(g, in);
  S kc = in[12], dh = in[13];
  return branch(dh - d, -kc * pown(d - dh, 2) * log(d / dh), S(&g, g.cst(0.0)));
}

// Its activation c_e = d_hat - d (Eq. 9), compiled as a function of its own.
S ipc_point_plane_act(Graph& g, const std::vector<S>& in) {
  return in[13] - point_plane_distance(g, in);
}

// Quadratic bending (Eq. 13, Bergou et al. 2006): E = k_b/2 x^T Q x with the
// constant Q = c (K K^T) (x) I3; inputs are the per-node weights K_a and the
// scale c = 3/(A0 + A1), precomputed from the rest hinge.
S hinge4(Graph& g, const std::vector<S>& in) {
  (void)g;
  std::vector<S> s(3);
  for (int i = 0; i < 3; ++i) {
    S acc = in[12] * in[i];
    for (int a = 1; a < 4; ++a) acc = acc + in[12 + a] * in[3 * a + i];
    s[i] = acc;
  }
  S kb = in[17], c = in[16];
  return 0.5 * kb * c * dot(s, s);
}

// Inertia of one node (Eq. 2 and the inertia energy of the paper's listing):
// m / (2 dt^2) |x - x_tilde|^2.
S inertia(Graph& g, const std::vector<S>& in) {
  (void)g;
  std::vector<S> d = {in[0] - in[3], in[1] - in[4], in[2] - in[5]};
  S m = in[6], dt = in[7];
  return m / (2.0 * (dt * dt)) * dot(d, d);
}

// ---------------------------------------------------------------------------
// Higher-order tets (App. A, Eq. 12).  Node order: corners 0-3; the edges are
// k = (0,1), (1,2), (2,0), (0,3), (1,3), (2,3).  Quadratic: node 4 + k at the
// middle of edge k, N = L_c (2 L_c - 1) at a corner and 4 L_i L_j on an edge.
// Cubic: on edge k = (i, j) node 4 + 2k a third of the way from i and 5 + 2k a
// third from j, N = 9/2 L_i L_j (3 L_i - 1) (resp. 3 L_j - 1); node 16 + c at
// the centroid of the face opposite corner c, N = 27 L_i L_j L_k; corners
// N = L (3L - 1)(3L - 2) / 2.  L = (1 - xi0 - xi1 - xi2, xi0, xi1, xi2).
// ---------------------------------------------------------------------------
std::vector<S> tet10_shape(const std::vector<S>& L) {
  const int edge[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
  std::vector<S> N;
  for (int c = 0; c < 4; ++c) N.push_back(L[c] * (2.0 * L[c] - 1.0));
  for (const auto& e : edge) N.push_back(4.0 * L[e[0]] * L[e[1]]);
  return N;
}

std::vector<S> tet20_shape(const std::vector<S>& L) {
  const int edge[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
  std::vector<S> N;
  for (int c = 0; c < 4; ++c) N.push_back(0.5 * L[c] * (3.0 * L[c] - 1.0) * (3.0 * L[c] - 2.0));
  for (const auto& e : edge) {
    N.push_back(4.5 * L[e[0]] * L[e[1]] * (3.0 * L[e[0]] - 1.0));
    N.push_back(4.5 * L[e[0]] * L[e[1]] * (3.0 * L[e[1]] - 1.0));
  }
  for (int c = 0; c < 4; ++c) {
    S p = 27.0 * L[c == 0 ? 1 : 0];
    for (int k = (c == 0 ? 2 : 1); k < 4; ++k)
      if (k != c) p = p * L[k];
    N.push_back(p);
  }
  return N;
}

// Energies c * psi(F) whose deformation gradient is linear in the positions,
// F = sum_b x_b g_b^T with constant (position-free) vectors g_b:
// - linear tets: F = Ds Dm^-1, g_b the rows of Dm^-1 for b = 1..3 and
//   g_0 = -(g_1 + g_2 + g_3), c = V = |det Dm| / 6 (Sec. 3.1);
// - one quadrature point of a higher-order tet (Eq. 12): F = J_x J_X^-1,
//   g_b = J_X^-T dN_b/dxi (the shape functions differentiated symbolically
//   with respect to xi, as in App. A), c = w |det J_X(xi)|; the element
//   energy is the sum over the rule's points of this one function (Sec. 5.2,
//   fixed value summation).
// The density is differentiated with respect to the nine entries of F and
// the chain rule gives the element derivatives (struct ThroughF below).
struct Kinematics {
  Mat F;
  S c;
  std::vector<std::vector<S>> G;  // g_b, 3 entries per node
};

struct ThroughFSpec {
  std::string name;
  int n_nodes;
  int n_in;
  int rest_slot;  // first slot of node-0 rest coordinates
  std::function<Kinematics(Graph&, const std::vector<S>&)> kin;
  std::function<S(const Mat& F, const std::vector<S>& in)> psi;
  std::vector<int> row_nodes;  // nodes with row functions (one per node class)
  bool full;                   // also the full element E, g, H
  // also each row in parts: part k holds (gradient, for k = 0, and) the
  // off-diagonal blocks of the other nodes j in [part_lo[k], part_lo[k+1])
  // of the row's order, so that a kernel never holds the whole row
  std::vector<int> part_lo = {};
};

// Linear tet: inputs x (0..11), X (12..23).
Kinematics tet4_kin(Graph& g, const std::vector<S>& in) {
  Mat Ds = cols_minus_first(g, in, 0, 4);
  Mat Dm = cols_minus_first(g, in, 12, 4);
  Mat Dmi = inv3(Dm);
  Kinematics k{matmul(Ds, Dmi), abs(det3(Dm)) / 6.0, std::vector<std::vector<S>>(4, Vec(3))};
  for (int j = 0; j < 3; ++j) {
    k.G[0][j] = -(Dmi(0, j) + Dmi(1, j) + Dmi(2, j));
    for (int b = 1; b < 4; ++b) k.G[b][j] = Dmi(b - 1, j);
  }
  return k;
}

// One quadrature point of a higher-order tet with shape functions `shape`:
// inputs x (0..3K-1), X (3K..6K-1), mu, lambda, weight w, point xi
// (6K..6K+5).
Kinematics high_order_kin(Graph& g, const std::vector<S>& in, int K,
                          const std::function<std::vector<S>(const std::vector<S>&)>& shape) {
  std::vector<S> xi = {in[6 * K + 3], in[6 * K + 4], in[6 * K + 5]};
  for (const S& v : xi) g.set_dof(v.id);
  const std::vector<S> N = shape({1.0 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]});
  std::vector<std::vector<S>> dN(K, Vec(3));
  for (int a = 0; a < K; ++a)
    for (int k = 0; k < 3; ++k) dN[a][k] = S(&g, g.diff(N[a].id, xi[k].id));
  Mat JX(3, 3, &g), Jx(3, 3, &g);
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      S pX = in[3 * K + i] * dN[0][k], px = in[i] * dN[0][k];
      for (int a = 1; a < K; ++a) {
        pX = pX + in[3 * K + 3 * a + i] * dN[a][k];
        px = px + in[3 * a + i] * dN[a][k];
      }
      JX(i, k) = pX;
      Jx(i, k) = px;
    }
  const Mat JXi = inv3(JX);
  Kinematics kin{matmul(Jx, JXi), in[6 * K + 2] * abs(det3(JX)), std::vector<std::vector<S>>(K, Vec(3))};
  for (int a = 0; a < K; ++a)
    for (int j = 0; j < 3; ++j)
      kin.G[a][j] = JXi(0, j) * dN[a][0] + JXi(1, j) * dN[a][1] + JXi(2, j) * dN[a][2];
  return kin;
}

// Lame pair of the linear-tet materials.
S mu_of(const std::vector<S>& in) { return in[24]; }
S lam_of(const std::vector<S>& in) { return in[25]; }

// Saint Venant-Kirchhoff (App. B, Saint Venant branch):
// psi = mu |E|^2 + lambda/2 tr(E)^2, E = (F^T F - I) / 2.
S stvk_density(const Mat& F, const std::vector<S>& in) {
  Mat C = matmul(transpose(F), F);
  Mat E(3, 3, F.v[0].g);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) E(i, j) = i == j ? 0.5 * (C(i, j) - 1.0) : 0.5 * C(i, j);
  return mu_of(in) * frob2(E) + 0.5 * lam_of(in) * pown(trace(E), 2);
}

// Derivatives of c psi(F) through F (see above), built in graph g for the
// inputs `in` of a function with n_in inputs: nine placeholder symbols stand
// for F while psi is differentiated, then are replaced by F's expressions.
//   dE/dx_{a,i} = c sum_j P_ij g_a[j],  P = dpsi/dF;
//   d2E/dx_{a,i} dx_{b,m} = c sum_{j,l} D_{ij,ml} g_a[j] g_b[l],  D = d2psi/dF2.
// The contraction over j is the directional derivative of P along
// dF = c e_i g_a^T (forward mode through the graph of P, the zero entries of
// dF folded away), so D itself is never formed:
//   dP_i = d/deps P(F + eps c e_i g_a^T) at eps = 0,
//   entry (a_i, b_m) = sum_l dP_i[m][l] g_b[l].
struct ThroughF {
  Graph& g;
  const Kinematics& kin;
  Mat Fh;
  std::map<int, int> to_F;  // placeholder slot -> entry of F
  std::vector<int> Pph;     // P in terms of the placeholders
  std::vector<int> P;       // P in terms of the inputs
  S E;
  ThroughF(Graph& gr, const std::vector<S>& in, const Kinematics& k,
           const std::function<S(const Mat&, const std::vector<S>&)>& psi_of, int n_in)
      : g(gr), kin(k), Fh(3, 3, &gr), Pph(9) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        Fh(i, j) = S(&g, g.sym(n_in + 3 * i + j));
        g.set_dof(Fh(i, j).id);
        to_F[n_in + 3 * i + j] = kin.F(i, j).id;
      }
    const S psi = psi_of(Fh, in);
    for (int k2 = 0; k2 < 9; ++k2) Pph[k2] = g.diff(psi.id, Fh.v[k2].id);
    std::vector<int> dens = {psi.id};
    dens.insert(dens.end(), Pph.begin(), Pph.end());
    dens = g.substitute_nodes(dens, to_F);
    E = kin.c * S(&g, dens[0]);
    P.assign(dens.begin() + 1, dens.end());
  }
  S grad(int a, int i) const {
    const auto& G = kin.G;
    return kin.c * (S(&g, P[3 * i]) * G[a][0] + S(&g, P[3 * i + 1]) * G[a][1] +
                    S(&g, P[3 * i + 2]) * G[a][2]);
  }
  // Hessian row of node a: for i = 0..2 the blocks (a, b), b in order (the
  // diagonal block left out unless with_diag); only the blocks whose
  // position j in that order is in [j_lo, j_hi)
  std::vector<int> row_blocks(int a, bool with_diag, int j_lo = 0, int j_hi = 1 << 30) {
    const auto& G = kin.G;
    const int K = (int)G.size();
    std::vector<std::vector<int>> dP(3);
    for (int i = 0; i < 3; ++i) {
      std::map<int, int> dir;
      for (int q = 0; q < 3; ++q) dir[Fh(i, q).id] = (kin.c * G[a][q]).id;
      dP[i] = g.substitute_nodes(g.tangent(Pph, dir), to_F);
    }
    std::vector<int> ids;
    for (int i = 0; i < 3; ++i)
      for (int b = 0, j = 0; b < K; ++b) {
        if (b == a && !with_diag) continue;
        if (j >= j_lo && j < j_hi) {
          for (int m = 0; m < 3; ++m)
            ids.push_back((S(&g, dP[i][3 * m]) * G[b][0] + S(&g, dP[i][3 * m + 1]) * G[b][1] +
                           S(&g, dP[i][3 * m + 2]) * G[b][2]).id);
        }
        ++j;
      }
    return ids;
  }
};

struct Generated {
  std::string hip, c, meta;
};

void emit_all(Graph& g, const std::vector<Function>& fns, Generated& out);

void generate(const EnergySpec& spec, Generated& out) {
  Graph g;
  std::vector<S> in;
  for (int k = 0; k < spec.n_in; ++k) in.push_back(S(&g, g.sym(k)));
  int n_dof = 3 * spec.n_nodes;
  for (int k = 0; k < n_dof; ++k) g.set_dof(in[k].id);
  S E = spec.energy(g, in);
  std::vector<int> grad(n_dof);
  for (int k = 0; k < n_dof; ++k) grad[k] = g.diff(E.id, in[k].id);
  std::vector<int> hess(n_dof * n_dof);
  for (int k = 0; k < n_dof; ++k)
    for (int l = k; l < n_dof; ++l) hess[k * n_dof + l] = hess[l * n_dof + k] = g.diff(grad[k], in[l].id);

  std::vector<Function> fns;
  auto add_fn = [&](const std::string& suffix, std::vector<int> outs) {
    Function f;
    f.name = spec.name + suffix;
    f.n_in = spec.n_in;
    f.outputs = std::move(outs);
    fns.push_back(f);
  };
  std::vector<int> Eg = {E.id};
  Eg.insert(Eg.end(), grad.begin(), grad.end());
  std::vector<int> EgH = Eg;
  EgH.insert(EgH.end(), hess.begin(), hess.end());
  add_fn("_E", {E.id});
  add_fn("_Eg", Eg);
  add_fn("_EgH", EgH);

  // node 0 at the origin
  std::map<int, double> zero;
  for (int i = 0; i < 3; ++i) {
    zero[i] = 0.0;
    if (spec.rest_slot >= 0) zero[spec.rest_slot + i] = 0.0;
  }
  add_fn("_s_E", g.substitute({E.id}, zero));
  add_fn("_s_EgH", g.substitute(EgH, zero));
  // row of node 0: gradient and Hessian row; gradient only; gradient and the
  // off-diagonal blocks (the other nodes in ascending order), the diagonal
  // block following from translation invariance (each Hessian row sums to
  // zero over the nodes), so the kernel forms it as minus their sum
  std::vector<int> row_g(grad.begin(), grad.begin() + 3);
  add_fn("_row0_g", g.substitute(row_g, zero));
  std::vector<int> row_gH = row_g, row_gHoff = row_g;
  if (spec.density) {
    // linear tets: the Hessian rows (and the gradient row they carry) through F
    const Kinematics kin = tet4_kin(g, in);
    ThroughF tf(g, in, kin, spec.density, spec.n_in);
    for (int i = 0; i < 3; ++i) row_gH[i] = row_gHoff[i] = tf.grad(0, i).id;
    const std::vector<int> full = tf.row_blocks(0, true), off = tf.row_blocks(0, false);
    row_gH.insert(row_gH.end(), full.begin(), full.end());
    row_gHoff.insert(row_gHoff.end(), off.begin(), off.end());
  } else {
    for (int i = 0; i < 3; ++i)
      for (int l = 0; l < n_dof; ++l) {
        row_gH.push_back(hess[i * n_dof + l]);
        if (l >= 3) row_gHoff.push_back(hess[i * n_dof + l]);
      }
  }
  add_fn("_row0_gH", g.substitute(row_gH, zero));
  add_fn("_row0_gHoff", g.substitute(row_gHoff, zero));

  emit_all(g, fns, out);
}

void emit_all(Graph& g, const std::vector<Function>& fns, Generated& out) {
  for (const Function& f : fns) {
    Census ch, cc;
    out.hip += emit_hip(g, f, &ch);
    out.c += emit_c(g, f, &cc);
    std::ostringstream m;
    m << f.name << " " << f.n_in << " " << f.outputs.size() << " " << ch.add << " " << ch.sub << " "
      << ch.mul << " " << ch.div << " " << ch.neg << " " << ch.log << " " << ch.sqrt << " " << ch.abs
      << " " << ch.pown << " " << ch.total() << "\n";
    out.meta += m.str();
    std::printf("  %-24s in %3d out %4zu ops %6d\n", f.name.c_str(), f.n_in, f.outputs.size(),
                ch.total());
  }
}

void generate_through_F(const ThroughFSpec& spec, Generated& out) {
  Graph g;
  const int K = spec.n_nodes, n_in = spec.n_in;
  std::vector<S> in;
  for (int k = 0; k < n_in; ++k) in.push_back(S(&g, g.sym(k)));
  const Kinematics kin = spec.kin(g, in);
  ThroughF tf(g, in, kin, spec.psi, n_in);
  const S E = tf.E;
  auto grad = [&](int a, int i) { return tf.grad(a, i); };
  auto row_blocks = [&](int a, bool with_diag) { return tf.row_blocks(a, with_diag); };

  std::vector<Function> fns;
  auto add_fn = [&](const std::string& suffix, std::vector<int> outs) {
    Function f;
    f.name = spec.name + suffix;
    f.n_in = n_in;
    f.outputs = std::move(outs);
    fns.push_back(f);
  };
  // node 0 at the origin
  std::map<int, double> zero;
  for (int i = 0; i < 3; ++i) zero[i] = zero[spec.rest_slot + i] = 0.0;
  std::vector<int> EgH = {E.id};
  if (spec.full) {
    for (int a = 0; a < K; ++a)
      for (int i = 0; i < 3; ++i) EgH.push_back(grad(a, i).id);
  }
  add_fn("_E", {E.id});
  if (spec.full) add_fn("_Eg", EgH);
  if (spec.full) {
    // full Hessian, row-major (a, i) x (b, m)
    for (int a = 0; a < K; ++a) {
      const std::vector<int> row = row_blocks(a, true);
      EgH.insert(EgH.end(), row.begin(), row.end());
    }
    add_fn("_EgH", EgH);
  }
  add_fn("_s_E", g.substitute({E.id}, zero));
  if (spec.full) add_fn("_s_EgH", g.substitute(EgH, zero));
  for (int r : spec.row_nodes) {
    const std::string R = "_row" + std::to_string(r);
    std::vector<int> row_g;
    for (int i = 0; i < 3; ++i) row_g.push_back(grad(r, i).id);
    add_fn(R + "_g", g.substitute(row_g, zero));
    if (spec.full) {
      // gradient and the whole Hessian row (diagonal block included)
      std::vector<int> row_gH = row_g;
      const std::vector<int> blocks = row_blocks(r, true);
      row_gH.insert(row_gH.end(), blocks.begin(), blocks.end());
      add_fn(R + "_gH", g.substitute(row_gH, zero));
    }
    // gradient of node r and the off-diagonal blocks of its Hessian row (the
    // other nodes in ascending order); the kernels form the diagonal block as
    // minus their sum (translation invariance)
    std::vector<int> row_gHoff = row_g;
    const std::vector<int> blocks = row_blocks(r, false);
    row_gHoff.insert(row_gHoff.end(), blocks.begin(), blocks.end());
    add_fn(R + "_gHoff", g.substitute(row_gHoff, zero));
    for (size_t k = 0; k + 1 < spec.part_lo.size(); ++k) {
      std::vector<int> part = k == 0 ? row_g : std::vector<int>();
      const std::vector<int> pb = tf.row_blocks(r, false, spec.part_lo[k], spec.part_lo[k + 1]);
      part.insert(part.end(), pb.begin(), pb.end());
      add_fn(R + "_gHoff_p" + std::to_string(k), g.substitute(part, zero));
    }
  }
  emit_all(g, fns, out);
}

bool write_file(const std::string& path, const std::string& text) {
  std::ofstream f(path);
  if (!f) return false;
  f << text;
  return bool(f);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s <output directory>\n", argv[0]);
    return 2;
  }
  std::string dir = argv[1];
  // The linear-tet materials carry their density: their Hessian rows are
  // generated through F (SNH 680 operations per row against 795 by
  // differentiating the energy directly, NH 663 / 739, fixed co-rotational
  // 502 / 584, ARAP 512 / 597); energies, gradients and full element
  // Hessians are differentiated directly (fewer operations that way).
  auto snh_psi = [](const Mat& F, const std::vector<S>& in) { return snh_density(F, in[24], in[25]); };
  std::vector<EnergySpec> specs = {
      {"snh_tet4", 4, 26, 12, snh_tet4, snh_psi},
      {"stvk_tri3", 3, 21, 9, stvk_tri3},
      {"hinge4", 4, 18, -1, hinge4},
      {"inertia", 1, 8, -1, inertia},
      {"nh_tet4", 4, 26, 12, nh_tet4, nh_density},
      {"fcr_tet4", 4, 35, 12, fcr_tet4, fcr_density},
      {"arap_tet4", 4, 35, 12, arap_tet4, arap_density},
      {"ipc_point_plane", 4, 14, -1, ipc_point_plane},
      {"ipc_point_plane_act", 4, 14, -1, ipc_point_plane_act},
      {"ipc_point_plane_cond", 4, 14, -1, ipc_point_plane_cond},
  };
  // Energies differentiated through F throughout: StVK on linear tets (its
  // rows take 979 operations this way against 1,330 by direct
  // differentiation) and one quadrature point of the higher-order tets (2,214
  // against 4,661 for the cubic rows).
  auto tet4 = [](const std::string& name, int n_in,
                 std::function<S(const Mat&, const std::vector<S>&)> psi) {
    return ThroughFSpec{name, 4, n_in, 12, tet4_kin, std::move(psi), {0}, true};
  };
  auto high_order = [](const std::string& name, int K,
                       std::function<std::vector<S>(const std::vector<S>&)> shape,
                       std::vector<int> rows, bool full, std::vector<int> part_lo = {}) {
    return ThroughFSpec{name,
                        K,
                        6 * K + 6,
                        3 * K,
                        [K, shape](Graph& g, const std::vector<S>& in) {
                          return high_order_kin(g, in, K, shape);
                        },
                        [K](const Mat& F, const std::vector<S>& in) {
                          return snh_density(F, in[6 * K], in[6 * K + 1]);
                        },
                        std::move(rows),
                        full,
                        std::move(part_lo)};
  };
  const std::vector<ThroughFSpec> through_F = {
      tet4("stvk_tet4", 26, stvk_density),
      high_order("snh_tet10", 10, tet10_shape, {0, 4}, true),
      // the cubic rows also in three parts (7, 6 and 6 of the 19 other nodes)
      high_order("snh_tet20", 20, tet20_shape, {0, 4, 19}, false, {0, 7, 13, 19}),
  };
  Generated all;
  all.hip =
      "// Generated by symx_gen from the symbolic energy definitions; do not edit.\n"
      "#pragma once\n#include \"symx_math.h\"\n\n";
  all.c =
      "/* Generated by symx_gen (test-only CPU variant); do not edit. */\n"
      "#include <math.h>\n"
      "static double symx_pown(double a, int n) { double r = 1.0; for (int k = 0; k < n; ++k) r *= a; "
      "return r; }\n\n";
  all.meta = "# name n_in n_out add sub mul div neg log sqrt abs pown total\n";
  for (const auto& s : specs) {
    std::printf("%s\n", s.name.c_str());
    generate(s, all);
  }
  for (const auto& s : through_F) {
    std::printf("%s\n", s.name.c_str());
    generate_through_F(s, all);
  }
  if (!write_file(dir + "/symx_generated.h", all.hip) ||
      !write_file(dir + "/symx_generated_cpu.c", all.c) ||
      !write_file(dir + "/symx_generated_meta.txt", all.meta)) {
    std::fprintf(stderr, "symx_gen: cannot write to %s\n", dir.c_str());
    return 1;
  }
  return 0;
}
