// Integrands given as text: the input format of the integration workers
// (section 4.6): the number of variables, the number of intermediate functions,
// one line per intermediate function f[1], f[2], ..., then the integrand, each
// line ended by ';', and a final line '|'.  Expressions use + - * /, brackets,
// decimal numbers, x[i] (variables), f[i] (earlier intermediate functions),
// p[base,exponent] (power), l[arg] (natural logarithm), P (pi), G (Euler's
// gamma) and PolyGamma[m,z] for the handful of arguments the paper lists.
// An integrand that uses the imaginary unit I (the complex workers of section
// 4.2) compiles to a complex tape (expr_types.h).
//
// The text is parsed into a DAG with shared subexpressions merged and
// constant subtrees folded, then linearised into an expression tape whose
// temporaries are assigned to slots by liveness.
#include <hip/hip_runtime.h>

#include <cctype>
#include <charconv>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace sdi {
namespace {

enum NodeOp : int { N_CONST, N_VAR, N_ADD, N_SUB, N_MUL, N_DIV, N_NEG, N_LOG, N_POWI, N_POW, N_IUNIT };

struct Node {
  int op;
  int a, b;      // operand nodes (-1 if unused); the variable index for N_VAR
  int k;         // integer exponent (N_POWI)
  double imm;    // value (N_CONST)
};

struct ParseError {
  int code;
  std::string msg;
  bool slots = false;   // out of slots: worth a second try without merged operations
};

// x^k by binary powering of |k|, then one division for k < 0 (the device does the same).
double powi_host(double x, int k) {
  unsigned e = k < 0 ? 0u - (unsigned)k : (unsigned)k;
  double r = 1.0, b = x;
  while (e) {
    if (e & 1u) r *= b;
    e >>= 1;
    if (e) b *= b;
  }
  return k < 0 ? 1.0 / r : r;
}

class Compiler {
 public:
  std::vector<Node> nodes;
  bool share = true;   // merge repeated operations (leaves are always merged)
  bool cplx = false;   // complex tape: logarithms and powers of negative constants are not folded

  int constant(double v) { return add(Node{N_CONST, -1, -1, 0, v}); }
  int variable(int j) { return add(Node{N_VAR, j, -1, 0, 0.0}); }
  int iunit() { return add(Node{N_IUNIT, -1, -1, 0, 0.0}); }

  // Folds constant operands (real results only); merges identical nodes.
  int op2(int op, int a, int b, int k = 0) {
    const Node& A = nodes[a];
    const bool ca = A.op == N_CONST;
    const bool cb = b >= 0 && nodes[b].op == N_CONST;
    // the complex value of a logarithm, or of a constant power, of a negative
    // constant (arg -pi): re + im I with real constants
    if (cplx && ca && A.imm < 0.0 && (op == N_LOG || (op == N_POW && cb))) {
      const double x = A.imm;
      double re, im;
      if (op == N_LOG) {
        re = std::log(-x);
        im = -3.14159265358979323846;
      } else {
        const double y = nodes[b].imm, m = std::pow(-x, y);
        re = m * std::cos(3.14159265358979323846 * y);
        im = -m * std::sin(3.14159265358979323846 * y);
      }
      return op2(N_ADD, constant(re), op2(N_MUL, constant(im), iunit()));
    }
    if (ca && (b < 0 || cb)) {
      const double x = A.imm, y = b >= 0 ? nodes[b].imm : 0.0;
      double v = 0.0;
      switch (op) {
        case N_ADD: v = x + y; break;
        case N_SUB: v = x - y; break;
        case N_MUL: v = x * y; break;
        case N_DIV: v = x / y; break;
        case N_NEG: v = -x; break;
        case N_LOG: v = std::log(x); break;
        case N_POWI: v = powi_host(x, k); break;
        case N_POW: v = std::pow(x, y); break;
        default: break;
      }
      return constant(v);
    }
    return add(Node{op, a, b, k, 0.0});
  }

 private:
  struct Key {
    int op, a, b, k;
    uint64_t bits;
    bool operator==(const Key& o) const { return op == o.op && a == o.a && b == o.b && k == o.k && bits == o.bits; }
  };
  struct KeyHash {
    size_t operator()(const Key& q) const {
      uint64_t h = 1469598103934665603ull;
      for (uint64_t v : {(uint64_t)q.op, (uint64_t)(uint32_t)q.a, (uint64_t)(uint32_t)q.b, (uint64_t)(uint32_t)q.k, q.bits})
        h = (h ^ v) * 1099511628211ull;
      return (size_t)h;
    }
  };
  std::unordered_map<Key, int, KeyHash> seen_;

  int add(const Node& n) {
    uint64_t bits = 0;
    std::memcpy(&bits, &n.imm, 8);
    const Key key{n.op, n.a, n.b, n.k, bits};
    const bool leaf = n.op == N_CONST || n.op == N_VAR;
    auto it = (share || leaf) ? seen_.find(key) : seen_.end();
    if (it != seen_.end()) return it->second;
    if (nodes.size() >= ((size_t)1 << 24)) throw ParseError{SDI_ENOTSUP, "expression has more than 2^24 operations"};
    nodes.push_back(n);
    const int id = (int)nodes.size() - 1;
    if (share || leaf) seen_.emplace(key, id);
    return id;
  }
};

// Recursive-descent parser of one expression (one line without its ';').
class Parser {
 public:
  Parser(const std::string& text, size_t begin, size_t end, int nvars, const std::vector<int>& fnodes, Compiler& c)
      : s_(text), p_(begin), end_(end), n_(nvars), f_(fnodes), c_(c) {}

  // Whether [begin, end) of the text names the imaginary unit I.
  static bool mentions_i(const std::string& t, size_t begin, size_t end) {
    for (size_t p = begin; p < end; ++p)
      if (t[p] == 'I' && (p == begin || !std::isalnum((unsigned char)t[p - 1])) &&
          (p + 1 == end || !std::isalnum((unsigned char)t[p + 1])))
        return true;
    return false;
  }

  int parse() {
    const int v = expr();
    ws();
    if (p_ != end_) fail("unexpected '" + std::string(1, s_[p_]) + "'");
    return v;
  }

 private:
  const std::string& s_;
  size_t p_, end_;
  int n_;
  const std::vector<int>& f_;
  Compiler& c_;
  int depth_ = 0;

  [[noreturn]] void fail(const std::string& m) const {
    throw ParseError{SDI_EINVAL, m + " at offset " + std::to_string(p_)};
  }
  void ws() {
    while (p_ < end_ && (s_[p_] == ' ' || s_[p_] == '\t' || s_[p_] == '\n' || s_[p_] == '\r')) ++p_;
  }
  bool eat(char ch) {
    ws();
    if (p_ < end_ && s_[p_] == ch) {
      ++p_;
      return true;
    }
    return false;
  }
  void expect(char ch) {
    if (!eat(ch)) fail(std::string("expected '") + ch + "'");
  }
  bool word(const char* w) {
    ws();
    const size_t L = std::strlen(w);
    if (p_ + L <= end_ && s_.compare(p_, L, w) == 0) {
      // a name must not continue with a letter or digit
      if (p_ + L < end_ && std::isalnum((unsigned char)s_[p_ + L])) return false;
      p_ += L;
      return true;
    }
    return false;
  }
  long integer() {
    ws();
    const size_t b = p_;
    if (p_ < end_ && (s_[p_] == '-' || s_[p_] == '+')) ++p_;
    while (p_ < end_ && std::isdigit((unsigned char)s_[p_])) ++p_;
    if (p_ == b || !std::isdigit((unsigned char)s_[p_ - 1])) fail("expected an integer");
    long v = 0;
    const auto r = std::from_chars(s_.data() + b + (s_[b] == '+'), s_.data() + p_, v);
    if (r.ec != std::errc()) fail("integer out of range");
    return v;
  }
  double number() {
    const size_t b = p_;
    while (p_ < end_ && std::isdigit((unsigned char)s_[p_])) ++p_;
    if (p_ < end_ && s_[p_] == '.') {
      ++p_;
      while (p_ < end_ && std::isdigit((unsigned char)s_[p_])) ++p_;
    }
    if (p_ < end_ && (s_[p_] == 'e' || s_[p_] == 'E')) {
      size_t q = p_ + 1;
      if (q < end_ && (s_[q] == '+' || s_[q] == '-')) ++q;
      if (q < end_ && std::isdigit((unsigned char)s_[q])) {
        p_ = q;
        while (p_ < end_ && std::isdigit((unsigned char)s_[p_])) ++p_;
      }
    }
    double v = 0.0;
    const auto r = std::from_chars(s_.data() + b, s_.data() + p_, v);
    if (r.ec != std::errc() || r.ptr != s_.data() + p_) fail("malformed number");
    return v;
  }

  int expr() {
    if (++depth_ > 10000) fail("expression nested too deeply");
    int v = term();
    for (;;) {
      if (eat('+')) v = c_.op2(N_ADD, v, term());
      else if (eat('-')) v = c_.op2(N_SUB, v, term());
      else break;
    }
    --depth_;
    return v;
  }
  int term() {
    int v = unary();
    for (;;) {
      if (eat('*')) v = c_.op2(N_MUL, v, unary());
      else if (eat('/')) v = c_.op2(N_DIV, v, unary());
      else break;
    }
    return v;
  }
  int unary() {
    if (eat('-')) {
      if (++depth_ > 10000) fail("expression nested too deeply");
      const int v = c_.op2(N_NEG, unary(), -1);
      --depth_;
      return v;
    }
    if (eat('+')) {
      if (++depth_ > 10000) fail("expression nested too deeply");
      const int v = unary();
      --depth_;
      return v;
    }
    return primary();
  }
  int primary() {
    ws();
    if (p_ >= end_) fail("unexpected end of expression");
    const char ch = s_[p_];
    if (std::isdigit((unsigned char)ch) || ch == '.') return c_.constant(number());
    if (eat('(')) {
      const int v = expr();
      expect(')');
      return v;
    }
    if (word("PolyGamma")) {
      expect('[');
      const long m = integer();
      expect(',');
      const long z = integer();
      expect(']');
      return c_.constant(polygamma(m, z));
    }
    if (word("x")) {
      expect('[');
      const long i = integer();
      expect(']');
      if (i < 1 || i > n_) fail("x[" + std::to_string(i) + "] outside x[1] .. x[" + std::to_string(n_) + "]");
      return c_.variable((int)i - 1);
    }
    if (word("f")) {
      expect('[');
      const long i = integer();
      expect(']');
      if (i < 1 || i > (long)f_.size()) fail("f[" + std::to_string(i) + "] is not an earlier intermediate function");
      return f_[i - 1];
    }
    if (word("p")) {
      expect('[');
      const int base = expr();
      expect(',');
      const int ex = expr();
      expect(']');
      const Node& E = c_.nodes[ex];
      if (E.op == N_CONST && std::nearbyint(E.imm) == E.imm && std::fabs(E.imm) <= 64.0)
        return c_.op2(N_POWI, base, -1, (int)E.imm);
      return c_.op2(N_POW, base, ex);
    }
    if (word("l")) {
      expect('[');
      const int v = expr();
      expect(']');
      return c_.op2(N_LOG, v, -1);
    }
    if (word("I")) return c_.iunit();
    if (word("Pi") || word("P")) return c_.constant(3.14159265358979323846);
    if (word("EulerGamma") || word("G")) return c_.constant(0.57721566490153286061);
    fail("unknown symbol");
  }

  // The polygamma values the paper's workers know without Mathematica, from
  // psi_1(1) = pi^2/6, psi_2(1) = -2 zeta(3), psi_3(1) = pi^4/15 and the
  // recurrence psi_m(z+1) = psi_m(z) + (-1)^m m! / z^(m+1), to 22 digits.
  double polygamma(long m, long z) {
    if (m == 1 && z == 1) return 1.644934066848226436472;
    if (m == 2 && z == 1) return -2.404113806319188570799;
    if (m == 2 && z == 2) return -0.4041138063191885707995;
    if (m == 2 && z == 3) return -0.1541138063191885707995;
    if (m == 2 && z == 4) return -0.0800397322451144967254;
    if (m == 3 && z == 1) return 6.493939402266829149096;
    if (m == 3 && z == 2) return 0.493939402266829149096;
    throw ParseError{SDI_ENOTSUP, "PolyGamma[" + std::to_string(m) + "," + std::to_string(z) + "] is not built in"};
  }
};

// Splits the text into ';'-terminated statements up to the '|' line.
std::vector<std::pair<size_t, size_t>> statements(const std::string& t, size_t from) {
  std::vector<std::pair<size_t, size_t>> out;
  size_t p = from;
  for (;;) {
    while (p < t.size() && std::isspace((unsigned char)t[p])) ++p;
    if (p >= t.size()) throw ParseError{SDI_EINVAL, "missing the final '|' line"};
    if (t[p] == '|') {
      ++p;
      while (p < t.size() && std::isspace((unsigned char)t[p])) ++p;
      if (p != t.size()) throw ParseError{SDI_EINVAL, "text after the final '|'"};
      return out;
    }
    const size_t q = t.find(';', p);
    const size_t bar = t.find('|', p);
    if (q == std::string::npos || (bar != std::string::npos && bar < q))
      throw ParseError{SDI_EINVAL, "line without ';' at offset " + std::to_string(p)};
    out.push_back({p, q});
    p = q + 1;
  }
}

// Parses the intermediate functions and the integrand, then lowers the DAG
// to a tape in depth-first order: dead nodes dropped, constants carried in
// their users' immediate, slots assigned by liveness.
int lower(const std::string& text, const std::vector<std::pair<size_t, size_t>>& st, int n, long m, bool share,
          bool cplx, std::vector<ExprIns>& tape, int& nslots, int& out) {
  Compiler e;
  e.share = share;
  e.cplx = cplx;
  const int max_slots = cplx ? EXPR_MAX_SLOTS_CPLX : EXPR_MAX_SLOTS;
  for (int j = 0; j < n; ++j) e.variable(j);
  std::vector<int> fn;
  for (long i = 0; i < m; ++i) {
    Parser q(text, st[2 + i].first, st[2 + i].second, n, fn, e);
    fn.push_back(q.parse());
  }
  Parser q(text, st[2 + m].first, st[2 + m].second, n, fn, e);
  const int root = q.parse();

  const int N = (int)e.nodes.size();
  auto leaf = [&](int i) { return e.nodes[i].op == N_VAR || e.nodes[i].op == N_CONST; };
  std::vector<char> live(N, 0);
  live[root] = 1;
  for (int i = N - 1; i >= 0; --i) {
    if (!live[i] || leaf(i)) continue;
    if (e.nodes[i].a >= 0) live[e.nodes[i].a] = 1;   // X_IUNIT has no operand
    if (e.nodes[i].b >= 0) live[e.nodes[i].b] = 1;
  }
  // operations in dependency (creation) order
  std::vector<int> order;
  for (int i = 0; i < N; ++i)
    if (live[i] && !leaf(i)) order.push_back(i);
  // last operation reading each value (positions in `order`)
  std::vector<int> pos(N, -1);
  for (size_t k = 0; k < order.size(); ++k) pos[order[k]] = (int)k;
  std::vector<int> lastb(N, -1);
  for (int i : order) {
    const Node& d = e.nodes[i];
    for (int o : {d.a, d.b})
      if (o >= 0 && !leaf(o)) lastb[o] = std::max(lastb[o], pos[i]);
  }
  std::vector<int> slot(N, -1);
  for (int j = 0; j < n; ++j) slot[j] = j;   // variables: nodes 0..n-1, pinned
  std::vector<int> free_slots;
  int top = n;
  auto alloc = [&]() {
    int sl;
    if (!free_slots.empty()) {
      sl = free_slots.back();
      free_slots.pop_back();
    } else {
      sl = top++;
    }
    if (sl >= max_slots)
      throw ParseError{SDI_ENOTSUP, "the integrand needs more than " + std::to_string(max_slots) +
                                        (cplx ? " live complex temporaries" : " live temporaries"), true};
    return sl;
  };
  tape.clear();
  for (size_t bi = 0; bi < order.size(); ++bi) {
    const std::vector<int> b{order[bi]};
    std::vector<ExprIns> ins(b.size());
    for (size_t u = 0; u < b.size(); ++u) {
      const Node& d = e.nodes[b[u]];
      ExprIns& I = ins[u];
      I = ExprIns{};
      I.k = d.k;
      switch (d.op) {
        case N_ADD: I.op = X_ADD; break;
        case N_SUB: I.op = X_SUB; break;
        case N_MUL: I.op = X_MUL; break;
        case N_DIV: I.op = X_DIV; break;
        case N_NEG: I.op = X_NEG; break;
        case N_LOG: I.op = X_LOG; break;
        case N_POWI: I.op = X_POWI; break;
        case N_IUNIT: I.op = X_IUNIT; break;
        default: I.op = X_POW; break;
      }
      // constant operands ride in imm (folding leaves at most one per operation)
      if (d.a < 0) {
        // no operand
      } else if (e.nodes[d.a].op == N_CONST) {
        I.op |= X_IMMA;
        I.imm = e.nodes[d.a].imm;
      } else {
        I.a = (uint8_t)slot[d.a];
      }
      if (d.b >= 0) {
        if (e.nodes[d.b].op == N_CONST) {
          I.op |= X_IMMB;
          I.imm = e.nodes[d.b].imm;
        } else {
          I.b = (uint8_t)slot[d.b];
        }
      }
    }
    // values read for the last time free their slots before the result is
    // placed (an instruction reads its operands before it writes)
    for (int i : b) {
      const Node& d = e.nodes[i];
      for (int o : {d.a, d.b})
        if (o >= 0 && !leaf(o) && lastb[o] == (int)bi && slot[o] >= n) {
          free_slots.push_back(slot[o]);
          slot[o] = -2;
        }
    }
    for (size_t u = 0; u < b.size(); ++u) {
      slot[b[u]] = alloc();
      ins[u].dst = (uint8_t)slot[b[u]];
      tape.push_back(ins[u]);
    }
  }
  if (e.nodes[root].op == N_CONST) {
    ExprIns c{};
    c.op = X_CONST;
    c.imm = e.nodes[root].imm;
    c.dst = (uint8_t)alloc();
    slot[root] = c.dst;
    tape.push_back(c);
  }
  while (tape.size() % EXPR_FETCH) {
    ExprIns nop{};
    nop.op = X_NOP;
    tape.push_back(nop);
  }
  out = slot[root];
  nslots = std::max(top, n);
  return SDI_OK;
}

}  // namespace

// Compiles the text into a tape; n receives the number of variables.
int compile_expression(const std::string& text, int& n, std::vector<ExprIns>& tape, int& nslots, int& out,
                       bool& cplx, std::string& err) {
  cplx = false;
  try {
    size_t start = 0;
    {
      size_t p = 0;
      while (p < text.size() && std::isspace((unsigned char)text[p])) ++p;
      if (text.compare(p, 9, "Integrate") == 0) start = p + 9;
    }
    const auto st = statements(text, start);
    if (st.size() < 3) throw ParseError{SDI_EINVAL, "need the variable count, the function count and the integrand"};
    Compiler c;
    std::vector<int> none;
    auto as_int = [&](size_t i, long lo, long hi, const char* what) {
      Parser q(text, st[i].first, st[i].second, 0, none, c);
      const int v = q.parse();
      const Node& N = c.nodes[v];
      if (N.op != N_CONST || std::nearbyint(N.imm) != N.imm || N.imm < lo || N.imm > hi)
        throw ParseError{SDI_EINVAL, std::string(what) + " must be an integer in " + std::to_string(lo) + ".." +
                                         std::to_string(hi)};
      return (long)N.imm;
    };
    n = (int)as_int(0, 1, MAXV, "the number of variables");
    const long m = as_int(1, 0, 1 << 20, "the number of intermediate functions");
    if (st.size() != (size_t)(3 + m))
      throw ParseError{SDI_EINVAL, "expected " + std::to_string(m) + " intermediate functions and one integrand, found " +
                                       std::to_string(st.size() - 2) + " lines"};
    for (size_t i = 2; i < st.size(); ++i) cplx = cplx || Parser::mentions_i(text, st[i].first, st[i].second);
    // Merged repeated operations keep their values alive until the last use; if
    // that needs too many slots, compile again sharing only leaves and f[i].
    try {
      return lower(text, st, n, m, true, cplx, tape, nslots, out);
    } catch (const ParseError& pe) {
      if (!pe.slots) throw;
    }
    return lower(text, st, n, m, false, cplx, tape, nslots, out);
  } catch (const ParseError& pe) {
    err = pe.msg;
    return pe.code;
  }
}

}  // namespace sdi

using namespace sdi;

extern "C" int sdi_text_info(const char* text, int32_t* nvars, int64_t* ninstructions, int32_t* nslots, char* err,
                             size_t errlen) {
  if (err && errlen) err[0] = '\0';
  if (!text) return SDI_EINVAL;
  int n = 0, ns = 0, oslot = 0;
  bool cplx = false;
  std::vector<ExprIns> tape;
  std::string msg;
  const int rc = compile_expression(std::string(text), n, tape, ns, oslot, cplx, msg);
  if (rc != SDI_OK) {
    if (err && errlen) snprintf(err, errlen, "%s", msg.c_str());
    return rc;
  }
  if (nvars) *nvars = n;
  if (ninstructions) *ninstructions = (int64_t)tape.size();
  if (nslots) *nslots = ns;
  return SDI_OK;
}

extern "C" int sdi_problem_from_text(sdi_ctx* ctx, const char* text, sdi_problem** out) {
  if (!ctx || !text || !out) return fail(ctx, SDI_EINVAL, "problem_from_text: null argument");
  *out = nullptr;
  int n = 0, nslots = 0, oslot = 0;
  bool cplx = false;
  std::vector<ExprIns> tape;
  std::string err;
  const int rc = compile_expression(std::string(text), n, tape, nslots, oslot, cplx, err);
  if (rc != SDI_OK) return fail(ctx, rc, "problem_from_text: " + err);
  sdi_problem* pb = new sdi_problem();
  pb->ctx = ctx;
  pb->nsec = 1;
  pb->K = 1;
  pb->order_min = 0;
  pb->kfmax = 1;
  pb->nvmax = 16;
  pb->expr = tape;
  pb->expr_slots = nslots;
  pb->expr_out = oslot;
  pb->expr_cplx = cplx;
  SecDev R{};
  R.n = n;
  R.ns = 0;
  R.nfac = 0;
  R.kf = 1;
  R.K = 1;
  R.nvc = n <= 4 ? 0 : (n <= 8 ? 1 : 2);
  R.cls = R.nvc;
  for (int j = 0; j < n; ++j) R.perm[j] = j;
  R.fold_re[0][0] = 1.0;
  pb->secs.push_back(R);
  pb->cost.push_back(1.0 + (double)tape.size());
  pb->terms.push_back(Term{0.0, 0});
  if (pb->expr.empty()) pb->expr.push_back(ExprIns{});   // a variable integrand: nothing to execute
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_secs, sizeof(SecDev));
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_terms, sizeof(Term));
  if (e == hipSuccess) e = hipMalloc((void**)&pb->d_expr, pb->expr.size() * sizeof(ExprIns));
  if (e == hipSuccess) e = hipMemcpy(pb->d_secs, pb->secs.data(), sizeof(SecDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pb->d_terms, pb->terms.data(), sizeof(Term), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pb->d_expr, pb->expr.data(), pb->expr.size() * sizeof(ExprIns), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sdi_problem_destroy(pb);
    return fail(ctx, SDI_EDEVICE, std::string("problem upload: ") + hipGetErrorString(e));
  }
  pb->expr_nins = tape.size();
  *out = pb;
  return SDI_OK;
}
