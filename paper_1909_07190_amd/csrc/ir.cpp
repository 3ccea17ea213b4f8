// Pipeline IR: stage DAG, dependence offsets and the pointwise expression
// language (the paper, Section 2.2 "PolyMage DSL" and Section 2.3
// "Dependence Vectors").
#include <algorithm>
#include <cctype>
#include <cmath>
#include <sstream>

#include "wt_internal.h"

namespace wt {

void fail(wt_status s, const std::string& msg) { throw Error(s, msg); }

std::vector<std::vector<int>> Pipeline::consumers() const {
    std::vector<std::vector<int>> c(nodes.size());
    for (const Node& n : nodes)
        for (int s : n.srcs)
            if (c[s].empty() || c[s].back() != n.id) c[s].push_back(n.id);
    return c;
}

// Largest finite FP16 value.
constexpr double kHalfMax = 65504.0;

bool Pipeline::half_storable(int n) const {
    const Node& nd = nodes[n];
    return nd.kind != Kind::Input && !nd.is_int() && nd.bound <= kHalfMax;
}

bool Pipeline::is_output(int n) const {
    for (int o : outputs)
        if (o == n) return true;
    return false;
}

// Dependence vectors of consumer c on producer p as (dx, dy) offsets: the
// consumer at (x, y) reads the producer at (x + dx, y + dy).
int Pipeline::fold_source(int u) const {
    if (u < 0 || u >= (int)nodes.size() || nodes[u].kind != Kind::Up2) return -1;
    const Node& d = nodes[nodes[u].srcs[0]];
    if (d.kind != Kind::Down2) return -1;
    const Node& s = nodes[d.srcs[0]];
    if ((s.kind != Kind::Stencil && s.kind != Kind::Pointwise) || s.is_int() || nodes[u].is_int()) return -1;
    if (s.channels != nodes[u].channels || s.level != nodes[u].level) return -1;
    return s.id;
}

std::vector<Tap> Pipeline::taps(int c, int p) const {
    const Node& n = nodes[c];
    std::vector<Tap> t;
    if (n.kind == Kind::Up2) {
        if (fold_source(c) != p) return t;
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) t.push_back({dx, dy, 0.0});
        return t;
    }
    if (n.kind == Kind::Stencil) {
        if (n.srcs[0] != p) return t;
        for (int j = 0; j < n.kh; ++j)
            for (int i = 0; i < n.kw; ++i) {
                double w = n.weights[j * n.kw + i];
                if (w != 0.0) t.push_back({i - n.ax, j - n.ay, w * n.scale});
            }
        if (t.empty()) t.push_back({0, 0, 0.0});  // keeps the dependence
    } else if (n.kind == Kind::Pointwise) {
        for (int s : n.srcs)
            if (s == p) { t.push_back({0, 0, 1.0}); break; }
    } else if (n.kind == Kind::Equalize) {
        if (n.srcs[0] == p) t.push_back({0, 0, 1.0});  // the histogram is read whole, not by offsets
    }
    return t;
}

// ------------------------------------------------------------------------
// Expression parser: recursive descent over
//   expr := cmp ; cmp := sum [(<|<=|>|>=) sum] ; sum := prod {(+|-) prod}
//   prod := unary {(*|/) unary} ; unary := - unary | atom
//   atom := number | s<i> | s<i>[k] | f(args) | ( expr )
// ------------------------------------------------------------------------
namespace {
struct Parser {
    const std::string& s;
    size_t i = 0;
    int nsrc;
    Parser(const std::string& t, int n) : s(t), nsrc(n) {}
    void ws() { while (i < s.size() && std::isspace((unsigned char)s[i])) ++i; }
    bool eat(const char* tok) {
        ws();
        size_t n = std::char_traits<char>::length(tok);
        if (s.compare(i, n, tok) == 0) { i += n; return true; }
        return false;
    }
    [[noreturn]] void err(const std::string& m) {
        fail(WT_E_INVALID, "expression '" + s + "': " + m + " at offset " + std::to_string(i));
    }
    Expr bin(Expr::Op op, Expr a, Expr b) {
        Expr e; e.op = op; e.kids = {std::move(a), std::move(b)}; return e;
    }
    Expr expr() {
        Expr a = sum();
        ws();
        if (eat("<=")) return bin(Expr::Le, std::move(a), sum());
        if (eat(">=")) return bin(Expr::Ge, std::move(a), sum());
        if (eat("<")) return bin(Expr::Lt, std::move(a), sum());
        if (eat(">")) return bin(Expr::Gt, std::move(a), sum());
        return a;
    }
    Expr sum() {
        Expr a = prod();
        for (;;) {
            if (eat("+")) a = bin(Expr::Add, std::move(a), prod());
            else if (eat("-")) a = bin(Expr::Sub, std::move(a), prod());
            else return a;
        }
    }
    Expr prod() {
        Expr a = unary();
        for (;;) {
            if (eat("*")) a = bin(Expr::Mul, std::move(a), unary());
            else if (eat("/")) a = bin(Expr::Div, std::move(a), unary());
            else return a;
        }
    }
    Expr unary() {
        if (eat("-")) { Expr e; e.op = Expr::Neg; e.kids = {unary()}; return e; }
        if (eat("+")) return unary();
        return atom();
    }
    Expr atom() {
        ws();
        if (i >= s.size()) err("unexpected end");
        char c = s[i];
        if (c == '(') {
            ++i;
            Expr e = expr();
            if (!eat(")")) err("expected ')'");
            return e;
        }
        if (std::isdigit((unsigned char)c) || c == '.') {
            const char* b = s.c_str() + i;
            char* end = nullptr;
            double v = std::strtod(b, &end);
            if (end == b) err("bad number");
            i += end - b;
            Expr e; e.op = Expr::Const; e.value = v; return e;
        }
        if (std::isalpha((unsigned char)c)) {
            size_t b = i;
            while (i < s.size() && (std::isalnum((unsigned char)s[i]) || s[i] == '_')) ++i;
            std::string id = s.substr(b, i - b);
            if (id.size() > 1 && id[0] == 's' &&
                id.find_first_not_of("0123456789", 1) == std::string::npos) {
                Expr e; e.op = Expr::Src; e.src = std::stoi(id.substr(1));
                if (e.src >= nsrc) err("source index out of range");
                if (eat("[")) {
                    ws();
                    size_t d = i;
                    while (i < s.size() && std::isdigit((unsigned char)s[i])) ++i;
                    if (d == i) err("expected channel index");
                    e.chan = std::stoi(s.substr(d, i - d));
                    if (!eat("]")) err("expected ']'");
                }
                return e;
            }
            struct F { const char* n; Expr::Op op; int ar; };
            static const F fs[] = {{"abs", Expr::Abs, 1}, {"min", Expr::Min, 2},
                                   {"max", Expr::Max, 2}, {"select", Expr::Select, 3},
                                   {"sqrt", Expr::Sqrt, 1}, {"floor", Expr::Floor, 1}};
            for (const F& f : fs) {
                if (id != f.n) continue;
                if (!eat("(")) err("expected '('");
                Expr e; e.op = f.op;
                for (int k = 0; k < f.ar; ++k) {
                    if (k && !eat(",")) err("expected ','");
                    e.kids.push_back(expr());
                }
                if (!eat(")")) err("expected ')'");
                return e;
            }
            err("unknown identifier '" + id + "'");
        }
        err(std::string("unexpected character '") + c + "'");
    }
};
bool is_cmp(Expr::Op op) {
    return op == Expr::Lt || op == Expr::Le || op == Expr::Gt || op == Expr::Ge;
}
void check_types(const Expr& e, bool want_bool, const std::string& text) {
    if (is_cmp(e.op) != want_bool)
        fail(WT_E_INVALID, "expression '" + text + "': comparisons may appear only as "
                                                   "the first argument of select");
    for (size_t k = 0; k < e.kids.size(); ++k)
        check_types(e.kids[k], e.op == Expr::Select && k == 0, text);
}
}  // namespace

Expr parse_expr(const std::string& text, int nsrc) {
    Parser ps(text, nsrc);
    Expr e = ps.expr();
    ps.ws();
    if (ps.i != text.size()) ps.err("trailing characters");
    check_types(e, false, text);
    return e;
}

double expr_bound(const Expr& e, const std::vector<double>& sb) {
    auto k = [&](int i) { return expr_bound(e.kids[i], sb); };
    switch (e.op) {
        case Expr::Const: return std::fabs(e.value);
        case Expr::Src: return sb[e.src];
        case Expr::Neg: case Expr::Abs: case Expr::Floor: return k(0) + (e.op == Expr::Floor);
        case Expr::Add: case Expr::Sub: return k(0) + k(1);
        case Expr::Mul: return k(0) * k(1);
        case Expr::Div: return INFINITY;
        case Expr::Min: case Expr::Max: return std::max(k(0), k(1));
        case Expr::Select: return std::max(k(1), k(2));
        case Expr::Sqrt: return std::sqrt(k(0));
        default: return 1.0;  // comparisons
    }
}

bool is_int_dtype(int dt) { return dt == WT_U8 || dt == WT_U16 || dt == WT_I16 || dt == WT_I32; }

int dtype_size(int dt) {
    switch (dt) {
        case WT_U8: return 1;
        case WT_U16: case WT_I16: case WT_F16: return 2;
        default: return 4;
    }
}

std::pair<long long, long long> dtype_range(int dt) {
    switch (dt) {
        case WT_U8: return {0, 255};
        case WT_U16: return {0, 65535};
        case WT_I16: return {-32768, 32767};
        case WT_I32: return {-2147483648LL, 2147483647LL};
        default: fail(WT_E_INTERNAL, "dtype_range of a float type");
    }
}

const char* dtype_ctype(int dt) {
    switch (dt) {
        case WT_U8: return "unsigned char";
        case WT_U16: return "unsigned short";
        case WT_I16: return "short";
        case WT_I32: return "int";
        case WT_F16: return "_Float16";
        default: return "float";
    }
}

// Interval arithmetic over the expression tree; comparisons yield [0, 1].
Interval expr_range(const Expr& e, const std::vector<Interval>& sr, double* max_abs) {
    auto k = [&](int i) { return expr_range(e.kids[i], sr, max_abs); };
    Interval r{0, 0};
    switch (e.op) {
        case Expr::Const: r = {e.value, e.value}; break;
        case Expr::Src: r = sr[e.src]; break;
        case Expr::Neg: { Interval a = k(0); r = {-a.hi, -a.lo}; break; }
        case Expr::Abs: {
            Interval a = k(0);
            double m = std::max(std::fabs(a.lo), std::fabs(a.hi));
            r = {(a.lo <= 0 && a.hi >= 0) ? 0.0 : std::min(std::fabs(a.lo), std::fabs(a.hi)), m};
            break;
        }
        case Expr::Add: { Interval a = k(0), b = k(1); r = {a.lo + b.lo, a.hi + b.hi}; break; }
        case Expr::Sub: { Interval a = k(0), b = k(1); r = {a.lo - b.hi, a.hi - b.lo}; break; }
        case Expr::Mul: {
            Interval a = k(0), b = k(1);
            double c[4] = {a.lo * b.lo, a.lo * b.hi, a.hi * b.lo, a.hi * b.hi};
            r = {*std::min_element(c, c + 4), *std::max_element(c, c + 4)};
            break;
        }
        case Expr::Min: { Interval a = k(0), b = k(1); r = {std::min(a.lo, b.lo), std::min(a.hi, b.hi)}; break; }
        case Expr::Max: { Interval a = k(0), b = k(1); r = {std::max(a.lo, b.lo), std::max(a.hi, b.hi)}; break; }
        case Expr::Select: { k(0); Interval a = k(1), b = k(2); r = {std::min(a.lo, b.lo), std::max(a.hi, b.hi)}; break; }
        case Expr::Lt: case Expr::Le: case Expr::Gt: case Expr::Ge: k(0); k(1); r = {0, 1}; break;
        default: r = {-INFINITY, INFINITY}; break;  // division, sqrt, floor: not integer operations
    }
    if (max_abs) *max_abs = std::max(*max_abs, std::max(std::fabs(r.lo), std::fabs(r.hi)));
    return r;
}

bool expr_has_explicit_channel(const Expr& e) {
    if (e.op == Expr::Src && e.chan >= 0) return true;
    for (const Expr& k : e.kids)
        if (expr_has_explicit_channel(k)) return true;
    return false;
}

int expr_max_channel(const Expr& e, int src) {
    int m = -1;
    if (e.op == Expr::Src && e.src == src) m = e.chan;
    for (const Expr& k : e.kids) m = std::max(m, expr_max_channel(k, src));
    return m;
}

}  // namespace wt
