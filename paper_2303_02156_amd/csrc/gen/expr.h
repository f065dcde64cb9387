// Scalar expression graph with structural hash-consing and symbolic
// differentiation -- the build-time symbolic engine of the library.
//
// Follows the paper's Sec. 5.2 (Symbolic Engine): every expression is a DAG of
// scalar nodes (symbol, constant, operation); structurally identical nodes are
// created once by looking up (op, children) in a hash map while the graph is
// built bottom-up (common subexpression elimination); derivatives are taken by
// recursive chain rule with a table of elementary derivatives and a cache of
// already differentiated sub-expressions shared by all gradient and Hessian
// entries.  Beyond the paper, trivial identities with 0 and 1 are folded while
// nodes are created, and nodes carry a mask of the differentiation symbols they
// depend on so that zero derivatives are recognised without traversal.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

namespace symx {

// Branch: the conditional expression of Sec. 5.2 (branching), a > 0 ? b : e,
// evaluated with a real if/else in the generated code (only the taken arm's
// exclusive operations run).  Its derivative is the branch of the arms'
// derivatives (the condition is not differentiated: piecewise definition).
enum class Op : uint8_t { Sym, Const, Add, Sub, Mul, Div, Neg, Log, Sqrt, Abs, PowN, Branch };

struct Node {
  Op op;
  int a = -1, b = -1;  // children (Branch: condition a, then-arm b)
  int e = -1;          // Branch: else-arm
  int n = 0;           // symbol index (Sym) or integer exponent (PowN)
  double c = 0.0;      // value (Const)
  uint64_t dep = 0;    // bit k set: depends on differentiation symbol k
};

class Graph {
 public:
  Graph();
  int sym(int input_index);          // input slot in the generated function
  int cst(double v);
  int add(int a, int b);
  int sub(int a, int b);
  int mul(int a, int b);
  int div(int a, int b);
  int neg(int a);
  int log(int a);
  int sqrt(int a);
  int abs(int a);
  int pown(int a, int n);
  int branch(int cond, int then_v, int else_v);  // cond > 0 ? then_v : else_v

  // Mark the symbol node of an input slot as a differentiation variable; its
  // bit index is the order of the calls (at most 64 variables).
  void set_dof(int sym_node);
  // d f / d (symbol node s); cached per (f, s)
  int diff(int f, int s);
  // Forward-mode (directional) derivative of `roots`: every symbol node s in
  // `tangent_of` moves along the expression tangent_of[s], all other symbols
  // stay fixed; returns d root / d eps of root(s + eps t) at eps = 0 for each
  // root, built with the same folding rules (zero tangents remove terms).
  std::vector<int> tangent(const std::vector<int>& roots, const std::map<int, int>& tangent_of);
  // Rebuild `roots` with some input slots replaced by constants (memoised);
  // folding rules apply again, so e.g. x0 = 0 removes whole subtrees.
  std::vector<int> substitute(const std::vector<int>& roots,
                              const std::map<int, double>& slot_values);
  // The same with input slots replaced by existing nodes (e.g. placeholder
  // symbols by the expressions they stand for).
  std::vector<int> substitute_nodes(const std::vector<int>& roots,
                                    const std::map<int, int>& slot_nodes);

  const Node& node(int id) const { return nodes_[id]; }
  int size() const { return (int)nodes_.size(); }
  bool is_const(int id, double v) const {
    return nodes_[id].op == Op::Const && nodes_[id].c == v;
  }

 private:
  int make(Op op, int a, int b, int n, double c, int e = -1);
  std::vector<Node> nodes_;
  std::unordered_map<std::string, int> cse_;
  std::unordered_map<uint64_t, int> dcache_;
  std::map<int, int> dof_bit_;  // sym node -> bit
  std::map<int, int> sym_of_slot_;
};

// Thin value type with operator overloading (the paper's `Scalar`).
struct S {
  Graph* g = nullptr;
  int id = -1;
  S() = default;
  S(Graph* gg, int i) : g(gg), id(i) {}
};
S operator+(S a, S b);
S operator-(S a, S b);
S operator*(S a, S b);
S operator/(S a, S b);
S operator-(S a);
S operator+(S a, double b);
S operator+(double a, S b);
S operator-(S a, double b);
S operator-(double a, S b);
S operator*(S a, double b);
S operator*(double a, S b);
S operator/(S a, double b);
S log(S a);
S sqrt(S a);
S abs(S a);
S pown(S a, int n);
S branch(S cond, S then_v, S else_v);  // cond > 0 ? then_v : else_v

// Small dense helpers (the paper's `Vector` / `Matrix` are arrays of scalars).
using Vec = std::vector<S>;
struct Mat {
  int r = 0, c = 0;
  std::vector<S> v;
  Mat() = default;
  Mat(int rr, int cc, Graph* g);
  S& operator()(int i, int j) { return v[i * c + j]; }
  const S& operator()(int i, int j) const { return v[i * c + j]; }
};
Mat matmul(const Mat& A, const Mat& B);
Mat transpose(const Mat& A);
S det3(const Mat& A);
S det2(const Mat& A);
Mat inv3(const Mat& A);  // adjugate / determinant
Mat inv2(const Mat& A);
S trace(const Mat& A);
S frob2(const Mat& A);   // squared Frobenius norm
S dot(const Vec& a, const Vec& b);

// One generated function: name, number of inputs, output expressions.
struct Function {
  std::string name;
  int n_in = 0;
  std::vector<int> outputs;
};

struct Census {
  int add = 0, sub = 0, mul = 0, div = 0, neg = 0, log = 0, sqrt = 0, abs = 0, pown = 0;
  int branch = 0;  // if/else points (not counted as operations)
  int total() const { return add + sub + mul + div + neg + log + sqrt + abs + pown; }
};

// Emitters: HIP device template (T = float | double) and test-only C (double).
std::string emit_hip(const Graph& g, const Function& f, Census* census);
std::string emit_c(const Graph& g, const Function& f, Census* census);

}  // namespace symx
