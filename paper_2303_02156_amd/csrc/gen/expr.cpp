// Expression graph, hash-consing, differentiation and emitters (see expr.h).
#include "expr.h"

#include <cmath>
#include <cstdio>
#include <climits>
#include <functional>
#include <map>
#include <set>
#include <tuple>
#include <unordered_map>
#include <sstream>
#include <stdexcept>

namespace symx {

Graph::Graph() { nodes_.reserve(1 << 16); }

int Graph::make(Op op, int a, int b, int n, double c, int e) {
  char key[112];
  std::snprintf(key, sizeof key, "%d|%d|%d|%d|%a|%d", (int)op, a, b, n, c, e);
  auto it = cse_.find(key);
  if (it != cse_.end()) return it->second;
  Node nd;
  nd.op = op;
  nd.a = a;
  nd.b = b;
  nd.n = n;
  nd.c = c;
  nd.e = e;
  nd.dep = 0;
  if (a >= 0) nd.dep |= nodes_[a].dep;
  if (b >= 0) nd.dep |= nodes_[b].dep;
  if (e >= 0) nd.dep |= nodes_[e].dep;
  nodes_.push_back(nd);
  int id = (int)nodes_.size() - 1;
  cse_.emplace(key, id);
  return id;
}

int Graph::sym(int slot) {
  auto it = sym_of_slot_.find(slot);
  if (it != sym_of_slot_.end()) return it->second;
  int id = make(Op::Sym, -1, -1, slot, 0.0);
  sym_of_slot_[slot] = id;
  return id;
}

int Graph::cst(double v) {
  if (v == 0.0) v = 0.0;  // fold -0 into +0
  return make(Op::Const, -1, -1, 0, v);
}

void Graph::set_dof(int s) {
  if (nodes_[s].op != Op::Sym) throw std::runtime_error("set_dof on non-symbol");
  if (dof_bit_.count(s)) return;
  int bit = (int)dof_bit_.size();
  if (bit >= 64) throw std::runtime_error("more than 64 differentiation variables");
  dof_bit_[s] = bit;
  // only valid before the symbol is used by other nodes
  nodes_[s].dep |= (uint64_t(1) << bit);
}

static bool isc(const Node& n) { return n.op == Op::Const; }

int Graph::add(int a, int b) {
  const Node &A = nodes_[a], &B = nodes_[b];
  if (isc(A) && isc(B)) return cst(A.c + B.c);
  if (is_const(a, 0.0)) return b;
  if (is_const(b, 0.0)) return a;
  if (B.op == Op::Neg) return sub(a, B.a);
  if (A.op == Op::Neg) return sub(b, A.a);
  if (a > b) std::swap(a, b);
  return make(Op::Add, a, b, 0, 0.0);
}

int Graph::sub(int a, int b) {
  const Node &A = nodes_[a], &B = nodes_[b];
  if (isc(A) && isc(B)) return cst(A.c - B.c);
  if (is_const(b, 0.0)) return a;
  if (is_const(a, 0.0)) return neg(b);
  if (a == b) return cst(0.0);
  if (B.op == Op::Neg) return add(a, B.a);
  return make(Op::Sub, a, b, 0, 0.0);
}

int Graph::mul(int a, int b) {
  const Node &A = nodes_[a], &B = nodes_[b];
  if (isc(A) && isc(B)) return cst(A.c * B.c);
  if (is_const(a, 0.0) || is_const(b, 0.0)) return cst(0.0);
  if (is_const(a, 1.0)) return b;
  if (is_const(b, 1.0)) return a;
  if (is_const(a, -1.0)) return neg(b);
  if (is_const(b, -1.0)) return neg(a);
  if (A.op == Op::Neg && B.op == Op::Neg) return mul(A.a, B.a);
  if (A.op == Op::Neg) return neg(mul(A.a, b));
  if (B.op == Op::Neg) return neg(mul(a, B.a));
  if (a > b) std::swap(a, b);
  return make(Op::Mul, a, b, 0, 0.0);
}

int Graph::div(int a, int b) {
  const Node &A = nodes_[a], &B = nodes_[b];
  if (is_const(b, 0.0)) throw std::runtime_error("symbolic division by zero");
  if (isc(A) && isc(B)) return cst(A.c / B.c);
  if (is_const(a, 0.0)) return cst(0.0);
  if (is_const(b, 1.0)) return a;
  if (a == b) return cst(1.0);
  if (A.op == Op::Neg) return neg(div(A.a, b));
  return make(Op::Div, a, b, 0, 0.0);
}

int Graph::neg(int a) {
  const Node& A = nodes_[a];
  if (isc(A)) return cst(-A.c);
  if (A.op == Op::Neg) return A.a;
  return make(Op::Neg, a, -1, 0, 0.0);
}

int Graph::log(int a) {
  if (isc(nodes_[a])) return cst(std::log(nodes_[a].c));
  return make(Op::Log, a, -1, 0, 0.0);
}

int Graph::sqrt(int a) {
  if (isc(nodes_[a])) return cst(std::sqrt(nodes_[a].c));
  return make(Op::Sqrt, a, -1, 0, 0.0);
}

int Graph::abs(int a) {
  if (isc(nodes_[a])) return cst(std::fabs(nodes_[a].c));
  return make(Op::Abs, a, -1, 0, 0.0);
}

int Graph::pown(int a, int n) {
  if (n == 0) return cst(1.0);
  if (n == 1) return a;
  if (isc(nodes_[a])) return cst(std::pow(nodes_[a].c, n));
  return make(Op::PowN, a, -1, n, 0.0);
}

int Graph::branch(int cond, int t, int e) {
  const Node& C = nodes_[cond];
  if (isc(C)) return C.c > 0.0 ? t : e;
  if (t == e) return t;
  return make(Op::Branch, cond, t, 0, 0.0, e);
}

int Graph::diff(int f, int s) {
  auto bit_it = dof_bit_.find(s);
  if (bit_it == dof_bit_.end()) throw std::runtime_error("diff w.r.t. a non-dof symbol");
  uint64_t bit = uint64_t(1) << bit_it->second;
  if (!(nodes_[f].dep & bit)) return cst(0.0);
  uint64_t key = (uint64_t(f) << 6) | uint64_t(bit_it->second);
  auto it = dcache_.find(key);
  if (it != dcache_.end()) return it->second;
  const Node nd = nodes_[f];  // copy: nodes_ may grow
  int r;
  switch (nd.op) {
    case Op::Sym: r = cst(f == s ? 1.0 : 0.0); break;
    case Op::Const: r = cst(0.0); break;
    case Op::Add: r = add(diff(nd.a, s), diff(nd.b, s)); break;
    case Op::Sub: r = sub(diff(nd.a, s), diff(nd.b, s)); break;
    case Op::Mul: r = add(mul(diff(nd.a, s), nd.b), mul(nd.a, diff(nd.b, s))); break;
    // Quotients are differentiated through the shared reciprocal node 1/b,
    // so that all gradient and Hessian entries reuse one division.
    case Op::Div:  // (a/b)' = (a' - (a/b) b') * (1/b)
      r = mul(sub(diff(nd.a, s), mul(f, diff(nd.b, s))), div(cst(1.0), nd.b));
      break;
    case Op::Neg: r = neg(diff(nd.a, s)); break;
    case Op::Log: r = mul(diff(nd.a, s), div(cst(1.0), nd.a)); break;
    case Op::Sqrt: r = mul(diff(nd.a, s), mul(cst(0.5), div(cst(1.0), f))); break;
    case Op::Abs: r = mul(diff(nd.a, s), mul(nd.a, div(cst(1.0), f))); break;
    case Op::PowN: r = mul(mul(cst((double)nd.n), pown(nd.a, nd.n - 1)), diff(nd.a, s)); break;
    case Op::Branch: r = branch(nd.a, diff(nd.b, s), diff(nd.e, s)); break;
    default: throw std::runtime_error("diff: bad op");
  }
  dcache_[key] = r;
  return r;
}

std::vector<int> Graph::tangent(const std::vector<int>& roots,
                               const std::map<int, int>& tangent_of) {
  // bits of the moving symbols that are differentiation variables, so that
  // subtrees independent of every moving symbol get a zero tangent at once
  uint64_t moving = 0;
  bool all_dof = true;
  for (const auto& st : tangent_of) {
    auto b = dof_bit_.find(st.first);
    if (b == dof_bit_.end())
      all_dof = false;
    else
      moving |= uint64_t(1) << b->second;
  }
  std::unordered_map<int, int> memo;
  std::function<int(int)> go = [&](int id) -> int {
    auto it = memo.find(id);
    if (it != memo.end()) return it->second;
    const Node nd = nodes_[id];  // copy: nodes_ may grow
    int r;
    if (all_dof && !(nd.dep & moving)) {
      r = cst(0.0);
    } else {
      switch (nd.op) {
        case Op::Sym: {
          auto t = tangent_of.find(id);
          r = t != tangent_of.end() ? t->second : cst(0.0);
          break;
        }
        case Op::Const: r = cst(0.0); break;
        case Op::Add: r = add(go(nd.a), go(nd.b)); break;
        case Op::Sub: r = sub(go(nd.a), go(nd.b)); break;
        case Op::Mul: r = add(mul(go(nd.a), nd.b), mul(nd.a, go(nd.b))); break;
        // (a/b)' = (a' - (a/b) b') * (1/b), through the shared reciprocal
        case Op::Div: r = mul(sub(go(nd.a), mul(id, go(nd.b))), div(cst(1.0), nd.b)); break;
        case Op::Neg: r = neg(go(nd.a)); break;
        case Op::Log: r = mul(go(nd.a), div(cst(1.0), nd.a)); break;
        case Op::Sqrt: r = mul(go(nd.a), mul(cst(0.5), div(cst(1.0), id))); break;
        case Op::Abs: r = mul(go(nd.a), mul(nd.a, div(cst(1.0), id))); break;
        case Op::PowN: r = mul(mul(cst((double)nd.n), pown(nd.a, nd.n - 1)), go(nd.a)); break;
        case Op::Branch: r = branch(nd.a, go(nd.b), go(nd.e)); break;
        default: throw std::runtime_error("tangent: bad op");
      }
    }
    memo[id] = r;
    return r;
  };
  std::vector<int> out;
  out.reserve(roots.size());
  for (int r : roots) out.push_back(go(r));
  return out;
}

std::vector<int> Graph::substitute(const std::vector<int>& roots,
                                   const std::map<int, double>& slot_values) {
  std::map<int, int> slot_nodes;
  for (const auto& sv : slot_values) slot_nodes[sv.first] = cst(sv.second);
  return substitute_nodes(roots, slot_nodes);
}

std::vector<int> Graph::substitute_nodes(const std::vector<int>& roots,
                                         const std::map<int, int>& slot_nodes) {
  std::unordered_map<int, int> memo;
  std::function<int(int)> go = [&](int id) -> int {
    auto it = memo.find(id);
    if (it != memo.end()) return it->second;
    const Node nd = nodes_[id];
    int r;
    switch (nd.op) {
      case Op::Sym: {
        auto sv = slot_nodes.find(nd.n);
        r = (sv != slot_nodes.end()) ? sv->second : id;
        break;
      }
      case Op::Const: r = id; break;
      case Op::Add: r = add(go(nd.a), go(nd.b)); break;
      case Op::Sub: r = sub(go(nd.a), go(nd.b)); break;
      case Op::Mul: r = mul(go(nd.a), go(nd.b)); break;
      case Op::Div: r = div(go(nd.a), go(nd.b)); break;
      case Op::Neg: r = neg(go(nd.a)); break;
      case Op::Log: r = log(go(nd.a)); break;
      case Op::Sqrt: r = sqrt(go(nd.a)); break;
      case Op::Abs: r = abs(go(nd.a)); break;
      case Op::PowN: r = pown(go(nd.a), nd.n); break;
      case Op::Branch: r = branch(go(nd.a), go(nd.b), go(nd.e)); break;
      default: throw std::runtime_error("substitute: bad op");
    }
    memo[id] = r;
    return r;
  };
  std::vector<int> out;
  out.reserve(roots.size());
  for (int r : roots) out.push_back(go(r));
  return out;
}

// ---------------------------------------------------------------------------
// value-type operators
// ---------------------------------------------------------------------------
static Graph* G(S a, S b) { return a.g ? a.g : b.g; }
S operator+(S a, S b) { return S(G(a, b), G(a, b)->add(a.id, b.id)); }
S operator-(S a, S b) { return S(G(a, b), G(a, b)->sub(a.id, b.id)); }
S operator*(S a, S b) { return S(G(a, b), G(a, b)->mul(a.id, b.id)); }
S operator/(S a, S b) { return S(G(a, b), G(a, b)->div(a.id, b.id)); }
S operator-(S a) { return S(a.g, a.g->neg(a.id)); }
S operator+(S a, double b) { return a + S(a.g, a.g->cst(b)); }
S operator+(double a, S b) { return S(b.g, b.g->cst(a)) + b; }
S operator-(S a, double b) { return a - S(a.g, a.g->cst(b)); }
S operator-(double a, S b) { return S(b.g, b.g->cst(a)) - b; }
S operator*(S a, double b) { return a * S(a.g, a.g->cst(b)); }
S operator*(double a, S b) { return S(b.g, b.g->cst(a)) * b; }
S operator/(S a, double b) { return a / S(a.g, a.g->cst(b)); }
S log(S a) { return S(a.g, a.g->log(a.id)); }
S sqrt(S a) { return S(a.g, a.g->sqrt(a.id)); }
S abs(S a) { return S(a.g, a.g->abs(a.id)); }
S pown(S a, int n) { return S(a.g, a.g->pown(a.id, n)); }
S branch(S cond, S t, S e) {
  Graph* g = cond.g ? cond.g : (t.g ? t.g : e.g);
  return S(g, g->branch(cond.id, t.id, e.id));
}

Mat::Mat(int rr, int cc, Graph* g) : r(rr), c(cc), v(rr * cc, S(g, g->cst(0.0))) {}

Mat matmul(const Mat& A, const Mat& B) {
  Graph* g = A.v[0].g;
  Mat C(A.r, B.c, g);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < B.c; ++j) {
      S acc(g, g->cst(0.0));
      for (int k = 0; k < A.c; ++k) acc = acc + A(i, k) * B(k, j);
      C(i, j) = acc;
    }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T(A.c, A.r, A.v[0].g);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

S det2(const Mat& A) { return A(0, 0) * A(1, 1) - A(0, 1) * A(1, 0); }

S det3(const Mat& A) {
  return A(0, 0) * (A(1, 1) * A(2, 2) - A(1, 2) * A(2, 1)) -
         A(0, 1) * (A(1, 0) * A(2, 2) - A(1, 2) * A(2, 0)) +
         A(0, 2) * (A(1, 0) * A(2, 1) - A(1, 1) * A(2, 0));
}

Mat inv3(const Mat& A) {
  Graph* g = A.v[0].g;
  S d = det3(A);
  S inv_d = S(g, g->cst(1.0)) / d;
  Mat R(3, 3, g);
  // adjugate: R(j,i) = cofactor(i,j)
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      S cof = A(i1, j1) * A(i2, j2) - A(i1, j2) * A(i2, j1);
      R(j, i) = cof * inv_d;
    }
  return R;
}

Mat inv2(const Mat& A) {
  Graph* g = A.v[0].g;
  S inv_d = S(g, g->cst(1.0)) / det2(A);
  Mat R(2, 2, g);
  R(0, 0) = A(1, 1) * inv_d;
  R(0, 1) = -A(0, 1) * inv_d;
  R(1, 0) = -A(1, 0) * inv_d;
  R(1, 1) = A(0, 0) * inv_d;
  return R;
}

S trace(const Mat& A) {
  S t = A(0, 0);
  for (int i = 1; i < A.r; ++i) t = t + A(i, i);
  return t;
}

S frob2(const Mat& A) {
  S t = A.v[0] * A.v[0];
  for (size_t k = 1; k < A.v.size(); ++k) t = t + A.v[k] * A.v[k];
  return t;
}

S dot(const Vec& a, const Vec& b) {
  S t = a[0] * b[0];
  for (size_t k = 1; k < a.size(); ++k) t = t + a[k] * b[k];
  return t;
}

// ---------------------------------------------------------------------------
// emitters
// ---------------------------------------------------------------------------
static std::vector<int> topo_order(const Graph& g, const std::vector<int>& roots) {
  std::vector<int> order;
  std::vector<char> state(g.size(), 0);
  std::vector<std::pair<int, int>> stack;  // (node, next child slot 0..3)
  for (int r : roots) {
    if (state[r]) continue;
    state[r] = 1;
    stack.push_back({r, 0});
    while (!stack.empty()) {
      auto& top = stack.back();
      const Node& nd = g.node(top.first);
      const int kids[3] = {nd.a, nd.b, nd.e};
      bool pushed = false;
      while (top.second < 3) {
        const int c = kids[top.second++];
        if (c >= 0 && !state[c]) {
          state[c] = 1;
          stack.push_back({c, 0});
          pushed = true;
          break;
        }
      }
      if (pushed) continue;
      order.push_back(top.first);
      stack.pop_back();
    }
  }
  return order;
}

static std::string literal(double c, bool hip) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "%.17g", c);
  std::string s(buf);
  if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
  return hip ? "T(" + s + ")" : s;
}

// Regions of the generated code: the top level, and per region one pair of
// arms for each branch condition used there.  A node is emitted in the
// innermost region that contains all of its uses (so operations that only
// one arm needs run only when that arm is taken).  All branch nodes of one
// region with the same condition share one if/else:
//   T vB1, vB2, ...; if (cond > 0) { <then arm> vB1 = t1; ... } else { ... }
// placed, like any other item of the region, after everything it reads.
struct Regions {
  std::vector<int> parent;  // region -> enclosing region (-1 for the top level)
  std::vector<int> depth;
  std::map<std::tuple<int, int, int>, int> arm;  // (condition, arm 0/1, enclosing) -> region
  int of_arm(int cond, int which, int enclosing) {
    auto key = std::make_tuple(cond, which, enclosing);
    auto it = arm.find(key);
    if (it != arm.end()) return it->second;
    const int r = (int)parent.size();
    parent.push_back(enclosing);
    depth.push_back(depth[enclosing] + 1);
    arm[key] = r;
    return r;
  }
  int lca(int x, int y) const {
    while (depth[x] > depth[y]) x = parent[x];
    while (depth[y] > depth[x]) y = parent[y];
    while (x != y) {
      x = parent[x];
      y = parent[y];
    }
    return x;
  }
  bool inside(int x, int outer) const {  // x is outer or nested in it
    while (x >= 0 && depth[x] > depth[outer]) x = parent[x];
    return x == outer;
  }
};

static std::string emit_body(const Graph& g, const Function& f, Census* cen, bool hip) {
  Census local;
  Census& C = cen ? *cen : local;
  C = Census();
  auto name = [&](int id) -> std::string {
    const Node& nd = g.node(id);
    if (nd.op == Op::Sym) return "in[" + std::to_string(nd.n) + "]";
    if (nd.op == Op::Const) return literal(nd.c, hip);
    return "v" + std::to_string(id);
  };
  const char* ty = hip ? "const T" : "const double";
  const std::vector<int> order = topo_order(g, f.outputs);
  std::unordered_map<int, int> pos;  // node -> index in `order`
  for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;
  // regions: users come after their children in `order`, so a reverse pass
  // sees every use of a node before the node itself
  Regions R;
  R.parent.push_back(-1);
  R.depth.push_back(0);
  std::unordered_map<int, int> region;
  for (int r : f.outputs) region[r] = 0;
  for (auto it = order.rbegin(); it != order.rend(); ++it) {
    const int id = *it;
    const Node& nd = g.node(id);
    const int here = region.count(id) ? region[id] : 0;
    auto use = [&](int child, int reg) {
      if (child < 0) return;
      auto c = region.find(child);
      region[child] = c == region.end() ? reg : R.lca(c->second, reg);
    };
    if (nd.op == Op::Branch) {
      use(nd.a, here);
      use(nd.b, R.of_arm(nd.a, 0, here));
      use(nd.e, R.of_arm(nd.a, 1, here));
    } else {
      use(nd.a, here);
      use(nd.b, here);
    }
  }
  auto emitted = [&](int id) {
    const Op op = g.node(id).op;
    return op != Op::Sym && op != Op::Const;
  };
  std::ostringstream os;
  std::function<void(int, int)> emit_region = [&](int reg, int indent) {
    const std::string pad(2 * indent, ' ');
    // items of the region: its plain nodes, and one if/else per condition
    // (key: -1 - condition node) holding the branch nodes with that condition
    std::vector<int> items;
    std::map<int, std::vector<int>> groups;  // condition -> branch nodes, in order
    for (int id : order) {
      if (!emitted(id) || region[id] != reg) continue;
      const Node& nd = g.node(id);
      if (nd.op == Op::Branch) {
        if (!groups.count(nd.a)) items.push_back(-1 - nd.a);
        groups[nd.a].push_back(id);
      } else {
        items.push_back(id);
      }
    }
    // what each item reads from outside itself: a plain node its children; an
    // if/else the condition and every child, in or below its arms, that lies
    // outside them
    auto item_of = [&](int node) -> int {  // the item of this region holding node, or INT_MIN
      if (!emitted(node)) return INT_MIN;
      const int rg = region[node];
      if (rg == reg) {
        const Node& nd = g.node(node);
        return nd.op == Op::Branch ? -1 - nd.a : node;
      }
      for (const auto& gr : groups) {
        for (int w = 0; w < 2; ++w) {
          auto a = R.arm.find(std::make_tuple(gr.first, w, reg));
          if (a != R.arm.end() && R.inside(rg, a->second)) return -1 - gr.first;
        }
      }
      return INT_MIN;  // an enclosing region's node: already emitted
    };
    std::map<int, std::vector<int>> deps;  // item -> items it waits for
    for (int it : items) {
      std::vector<int> reads;
      if (it >= 0) {
        reads = {g.node(it).a, g.node(it).b};
      } else {
        const int cond = -1 - it;
        reads.push_back(cond);
        for (int id : order) {
          if (!emitted(id)) continue;
          const Node& nd = g.node(id);
          const int rg = region[id];
          bool in_group = false;
          if (rg == reg && nd.op == Op::Branch && nd.a == cond) in_group = true;
          for (int w = 0; w < 2 && !in_group; ++w) {
            auto a = R.arm.find(std::make_tuple(cond, w, reg));
            if (a != R.arm.end() && R.inside(rg, a->second)) in_group = true;
          }
          if (!in_group) continue;
          for (int c : {nd.a, nd.b, nd.e}) reads.push_back(c);
        }
      }
      for (int c : reads) {
        if (c < 0) continue;
        const int dep = item_of(c);
        if (dep != INT_MIN && dep != it) deps[it].push_back(dep);
      }
    }
    // emit in an order that respects the reads (first ready item in the
    // original order each time)
    std::vector<int> done_items;
    std::set<int> done;
    std::vector<int> pending = items;
    while (!pending.empty()) {
      size_t k = 0;
      for (; k < pending.size(); ++k) {
        bool ready = true;
        for (int d : deps[pending[k]]) ready = ready && done.count(d);
        if (ready) break;
      }
      if (k == pending.size()) throw std::runtime_error("emit: cyclic branch grouping");
      const int it = pending[k];
      pending.erase(pending.begin() + k);
      done.insert(it);
      if (it < 0) {
        const int cond = -1 - it;
        const std::vector<int>& br = groups[cond];
        C.branch++;
        for (int id : br) os << pad << (hip ? "T" : "double") << " v" << id << ";\n";
        os << pad << "if (" << name(cond) << " > " << literal(0.0, hip) << ") {\n";
        for (int w = 0; w < 2; ++w) {
          auto a = R.arm.find(std::make_tuple(cond, w, reg));
          if (a != R.arm.end()) emit_region(a->second, indent + 1);
          for (int id : br)
            os << pad << "  v" << id << " = " << name(w == 0 ? g.node(id).b : g.node(id).e)
               << ";\n";
          os << pad << (w == 0 ? "} else {\n" : "}\n");
        }
        continue;
      }
      const Node& nd = g.node(it);
      os << pad << ty << " v" << it << " = ";
      switch (nd.op) {
        case Op::Add: os << name(nd.a) << " + " << name(nd.b); C.add++; break;
        case Op::Sub: os << name(nd.a) << " - " << name(nd.b); C.sub++; break;
        case Op::Mul: os << name(nd.a) << " * " << name(nd.b); C.mul++; break;
        case Op::Div: os << name(nd.a) << " / " << name(nd.b); C.div++; break;
        case Op::Neg: os << "-" << name(nd.a); C.neg++; break;
        case Op::Log: os << (hip ? "sx_log(" : "log(") << name(nd.a) << ")"; C.log++; break;
        case Op::Sqrt: os << (hip ? "sx_sqrt(" : "sqrt(") << name(nd.a) << ")"; C.sqrt++; break;
        case Op::Abs: os << (hip ? "sx_abs(" : "fabs(") << name(nd.a) << ")"; C.abs++; break;
        case Op::PowN: {
          C.pown++;
          if (nd.n >= 2 && nd.n <= 4) {
            std::string a = name(nd.a);
            for (int k2 = 0; k2 < nd.n; ++k2) os << (k2 ? " * " : "") << a;
          } else {
            os << (hip ? "sx_pown<" : "symx_pown(") << (hip ? std::to_string(nd.n) + ">(" : "")
               << name(nd.a) << (hip ? ")" : ", " + std::to_string(nd.n) + ")");
          }
          break;
        }
        default: throw std::runtime_error("emit: bad op");
      }
      os << ";\n";
    }
  };
  emit_region(0, 1);
  for (size_t k = 0; k < f.outputs.size(); ++k)
    os << "  out[" << k << "] = " << name(f.outputs[k]) << ";\n";
  return os.str();
}

static std::string census_comment(const Census& c, const Function& f) {
  std::ostringstream os;
  os << "  // inputs " << f.n_in << ", outputs " << f.outputs.size() << "; ops: add " << c.add
     << ", sub " << c.sub << ", mul " << c.mul << ", div " << c.div << ", neg " << c.neg
     << ", log " << c.log << ", sqrt " << c.sqrt << ", abs " << c.abs << ", pown " << c.pown
     << ", total " << c.total() << "\n";
  return os.str();
}

std::string emit_hip(const Graph& g, const Function& f, Census* census) {
  Census c;
  std::string body = emit_body(g, f, &c, true);
  if (census) *census = c;
  std::ostringstream os;
  os << "template <typename T>\n__device__ __forceinline__ void " << f.name
     << "(const T* __restrict__ in, T* __restrict__ out) {\n"
     << census_comment(c, f) << body << "}\n\n";
  return os.str();
}

std::string emit_c(const Graph& g, const Function& f, Census* census) {
  Census c;
  std::string body = emit_body(g, f, &c, false);
  if (census) *census = c;
  std::ostringstream os;
  os << "void " << f.name << "(const double* in, double* out) {\n"
     << census_comment(c, f) << body << "}\n\n";
  return os.str();
}

}  // namespace symx
