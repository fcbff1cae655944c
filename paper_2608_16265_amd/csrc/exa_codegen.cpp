// Lowering of pattern trees to straight-line gfx950 code (Sec. 6.2, Sec. 7.2.1).
//
// For every callback ("mode") one kernel is generated.  A workgroup takes one
// tile (unit, first data point, count) from a tile list; each lane runs the
// whole evaluation of one data point at a time: coalesced struct-of-arrays
// loads, gathers of x, the forward sweep, and depending on the mode a reverse
// sweep (gradient, Jacobian rows), a forward tangent (J v), or
// forward-over-reverse (Hessian columns, H v, parameter adjoint).
//
// A unit is one pattern, or several patterns declared over the same data
// arrays evaluated in the same lane (their loads, gathers and common
// subexpressions are then shared: the cross-pattern fusion the paper points
// to in Sec. 8.3).  All sweeps are emitted as scalar SSA statements with the
// structural zeros and ones folded away (Sec. 7.2.2 affine nodes); a liveness
// pass keeps only the statements that reach an output, and records which
// inputs a unit really reads.  Results of a lane go to its own disjoint slice
// (Sec. 5.3.2); multi-entry slices are staged through LDS so that the
// workgroup writes contiguous memory.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <sstream>
#include <unordered_map>

#include "exa_internal.h"

namespace exa {

namespace {

const std::string Z = "0.0";
const std::string ONE = "1.0";
const std::string MONE = "(-1.0)";

std::string lit(double v) {
    if (v == 0.0 && !std::signbit(v)) return Z;
    if (v == 1.0) return ONE;
    if (v == -1.0) return MONE;
    if (std::isnan(v)) return "__builtin_nan(\"\")";
    if (std::isinf(v)) return v > 0 ? "__builtin_inf()" : "(-__builtin_inf())";
    char buf[64];
    snprintf(buf, sizeof buf, "%.17g", v);
    std::string s(buf);
    if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
    return "(" + s + ")";
}

bool is_unary(int op) { return op >= EXA_OP_NEG && op <= EXA_OP_EXPM1; }

// ---------------------------------------------------------------------------
// Statement recorder: SSA definitions, folding of the literals 0, 1, -1, and
// liveness from the outputs back to the loads.
struct Stmt {
    std::string type, name, expr;
    std::vector<int> deps;
    bool out = false;
    bool raw = false;  // a line emitted verbatim, in recorded order
};

struct Em {
    std::vector<Stmt> st;
    std::unordered_map<std::string, int> byname;
    int& ntmp;
    explicit Em(int& n) : ntmp(n) {}

    std::vector<int> deps_of(const std::string& e) const {
        std::vector<int> d;
        for (size_t i = 0; i < e.size();) {
            if (std::isalpha((unsigned char)e[i]) || e[i] == '_') {
                size_t j = i;
                while (j < e.size() && (std::isalnum((unsigned char)e[j]) || e[j] == '_')) ++j;
                auto it = byname.find(e.substr(i, j - i));
                if (it != byname.end()) d.push_back(it->second);
                i = j;
            } else {
                ++i;
            }
        }
        return d;
    }
    // a named value several jobs use (a row weight) is defined once
    std::string named_once(const std::string& type, const std::string& name, const std::string& e) {
        return byname.count(name) ? name : named(type, name, e);
    }
    std::string named(const std::string& type, const std::string& name, const std::string& e) {
        Stmt s{type, name, e, deps_of(e), false};
        st.push_back(s);
        byname[name] = (int)st.size() - 1;
        return name;
    }
    // identical pure expressions get one name (common subexpressions within
    // and across the patterns of a unit, and across Jacobian/Hessian sweeps)
    std::unordered_map<std::string, std::string> memo;
    std::string def(const std::string& e) {
        auto it = memo.find(e);
        if (it != memo.end()) return it->second;
        const std::string n = named("double", "t" + std::to_string(ntmp++), e);
        memo[e] = n;
        return n;
    }
    // an output statement; names in its destination (e.g. the index of an
    // in-place gradient entry) are as live as those in its value
    void out(const std::string& lhs, const std::string& e) {
        Stmt s{"", lhs, e, deps_of(lhs + " " + e), true};
        st.push_back(s);
    }
    void raw(const std::string& line) {
        Stmt s{"", "", line, deps_of(line), true, true};
        st.push_back(s);
    }
    std::string mul(const std::string& a, const std::string& b) {
        if (a == Z || b == Z) return Z;
        if (a == ONE) return b;
        if (b == ONE) return a;
        if (a == MONE) return neg(b);
        if (b == MONE) return neg(a);
        return def(a + " * " + b);
    }
    std::string add(const std::string& a, const std::string& b) {
        if (a == Z) return b;
        if (b == Z) return a;
        return def(a + " + " + b);
    }
    std::string sub(const std::string& a, const std::string& b) {
        if (b == Z) return a;
        if (a == Z) return neg(b);
        return def(a + " - " + b);
    }
    std::string neg(const std::string& a) {
        if (a == Z) return Z;
        if (a == ONE) return MONE;
        if (a == MONE) return ONE;
        return def("-" + a);
    }
    // Emit live statements; returns the set of live names.
    std::set<std::string> emit(std::ostream& os, const std::string& ind) const {
        std::vector<char> live(st.size(), 0);
        for (size_t i = st.size(); i-- > 0;) {
            if (st[i].out) live[i] = 1;
            if (live[i])
                for (int d : st[i].deps) live[d] = 1;
        }
        // sin and cos of one argument, both live: one sincos call (a
        // shared argument reduction), emitted at the first of the two
        std::map<std::string, std::pair<int, int>> trig;  // argument -> (sin stmt, cos stmt)
        auto trig_arg = [&](const Stmt& s, bool& is_sin) -> std::string {
            if (s.raw || s.out || s.expr.size() < 6 || s.expr.back() != ')') return "";
            const std::string f = s.expr.substr(0, 4);
            if (f != "sin(" && f != "cos(") return "";
            const std::string a = s.expr.substr(4, s.expr.size() - 5);
            for (char c : a)
                if (!(std::isalnum((unsigned char)c) || c == '_')) return "";
            is_sin = f == "sin(";
            return a;
        };
        for (size_t i = 0; i < st.size(); ++i) {
            if (!live[i]) continue;
            bool is_sin = false;
            const std::string a = trig_arg(st[i], is_sin);
            if (a.empty()) continue;
            auto it = trig.emplace(a, std::make_pair(-1, -1)).first;
            (is_sin ? it->second.first : it->second.second) = (int)i;
        }
        std::set<std::string> names;
        for (size_t i = 0; i < st.size(); ++i) {
            if (!live[i]) continue;
            const Stmt& s = st[i];
            bool is_sin = false;
            const std::string a = trig_arg(s, is_sin);
            auto tp = a.empty() ? trig.end() : trig.find(a);
            if (tp != trig.end() && tp->second.first >= 0 && tp->second.second >= 0) {
                const int si = tp->second.first, ci = tp->second.second;
                const std::string sn = st[si].name + "_s", cn = st[si].name + "_c";
                if ((int)i == std::min(si, ci))
                    os << ind << "double " << sn << ", " << cn << ";\n" << ind << "sincos(" << a << ", &" << sn
                       << ", &" << cn << ");\n";
                os << ind << "const double " << s.name << " = " << (is_sin ? sn : cn) << ";\n";
                names.insert(s.name);
                continue;
            }
            if (s.raw) {
                os << ind << s.expr << "\n";
            } else if (s.out) {
                os << ind << s.name << " = " << s.expr << ";\n";
            } else {
                os << ind << "const " << s.type << " " << s.name << " = " << s.expr << ";\n";
                names.insert(s.name);
            }
        }
        return names;
    }
};

enum SeedKind { SEED_DIR, SEED_VEC };

// Names of a pattern's inputs inside a unit (group-level loads).
struct Names {
    std::vector<std::string> x, v, ix, p;  // per var slot / param slot
    std::string wgt;
};

// ---------------------------------------------------------------------------
// Sweeps over one pattern tree.
class PatternCg {
  public:
    PatternCg(const Pattern& P, int mode, Em& e, const Names& nm) : P_(P), mode_(mode), t_(P.nodes), e_(e), nm_(nm) {
        const size_t n = t_.size();
        hasvar_.assign(n, 0);
        haspar_.assign(n, 0);
        for (size_t i = 0; i < n; ++i) {
            const TNode& q = t_[i];
            if (q.op == EXA_OP_VAR) hasvar_[i] = 1;
            if (q.op == EXA_OP_PARAM) haspar_[i] = 1;
            if (q.a >= 0) { hasvar_[i] |= hasvar_[q.a]; haspar_[i] |= haspar_[q.a]; }
            if (q.b >= 0) { hasvar_[i] |= hasvar_[q.b]; haspar_[i] |= haspar_[q.b]; }
        }
    }

    // Records the statements of this pattern; outputs go to `out`[s] (array
    // modes) or to `out` itself (scalar modes).
    void body(const std::string& out) {
        const bool second = mode_ == M_HESS || mode_ == M_HPROD || mode_ == M_ADJ;
        const bool first = mode_ != M_OBJ && mode_ != M_CONS;
        forward(first, second);
        const int root = (int)t_.size() - 1;
        auto slot = [&](int s) { return out + "[" + std::to_string(s) + "]"; };
        switch (mode_) {
            case M_OBJ:
            case M_CONS:
                e_.out(out, val_[root]);
                break;
            case M_GRAD:
            case M_JAC:
            case M_JTPROD: {
                // J^T w contributions are the Jacobian entries (seed 1, the
                // jac job's very statements) times the row's weight, one
                // rounding each: so the reduction of the Jacobian's COO
                // values times w gives the same bits
                std::vector<std::string> J(P_.o1step(), Z), Pacc, adj;
                reverse(ONE, adj, J, Pacc, false);
                for (int s = 0; s < P_.o1step(); ++s)
                    e_.out(slot(s), mode_ == M_JTPROD ? e_.mul(J[s], nm_.wgt) : J[s]);
                break;
            }
            case M_JPROD: {
                std::vector<std::string> tg;
                tangent(SEED_VEC, -1, tg);
                e_.out(out, tg[root]);
                break;
            }
            case M_HESS:
                hessian(slot);
                break;
            case M_HPROD: {
                std::vector<std::string> J(P_.o1step(), Z), Pacc, adj;
                reverse(nm_.wgt, adj, J, Pacc, false);
                std::vector<std::string> tg;
                tangent(SEED_VEC, -1, tg);
                std::vector<std::string> Hc(P_.o1step(), Z), Pt;
                reverse_tangent(adj, tg, Hc, Pt, false);
                for (size_t i = 0; i < P_.hvs.size(); ++i) e_.out(slot((int)i), Hc[P_.hvs[i]]);
                break;
            }
            case M_ADJ: {
                std::vector<std::string> J(P_.o1step(), Z), Pacc(P_.pstep(), Z), adj;
                reverse(nm_.wgt, adj, J, Pacc, true);
                std::vector<std::string> tg;
                tangent(SEED_VEC, -1, tg);
                std::vector<std::string> Hc(P_.o1step(), Z), Pt(P_.pstep(), Z);
                reverse_tangent(adj, tg, Hc, Pt, true);
                for (int s = 0; s < P_.pstep(); ++s) e_.out(slot(s), Pt[s]);
                break;
            }
            default:
                break;
        }
    }

  private:
    const Pattern& P_;
    int mode_;
    const std::vector<TNode>& t_;
    Em& e_;
    const Names& nm_;
    std::vector<char> hasvar_, haspar_;
    std::vector<std::string> val_, d1_, d2_, daa_, dab_, dbb_;  // unary: F', F''; binary: dA, dB

    bool rev_active(int i) const { return hasvar_[i] || (mode_ == M_ADJ && haspar_[i]); }

    void forward(bool first, bool second) {
        const size_t n = t_.size();
        val_.assign(n, Z);
        d1_.assign(n, Z);
        d2_.assign(n, Z);
        daa_.assign(n, Z);
        dab_.assign(n, Z);
        dbb_.assign(n, Z);
        for (size_t i = 0; i < n; ++i) {
            const TNode& q = t_[i];
            switch (q.op) {
                case EXA_OP_CONST: val_[i] = lit(q.val); continue;
                case EXA_OP_DATA: val_[i] = "fc" + std::to_string(q.col); continue;
                case EXA_OP_VAR: val_[i] = nm_.x[q.slot]; continue;
                case EXA_OP_PARAM: val_[i] = nm_.p[q.slot]; continue;
                default: break;
            }
            if (is_unary(q.op))
                unary((int)i, first && rev_active(q.a), second && rev_active(q.a));
            else
                binary((int)i, first, second);
        }
    }

    void unary(int i, bool f1, bool f2) {
        Em& e = e_;
        const TNode& q = t_[i];
        const std::string u = val_[q.a];
        std::string& v = val_[i];
        std::string& d = d1_[i];
        std::string& dd = d2_[i];
        switch (q.op) {
            case EXA_OP_NEG:
                v = e.neg(u);
                if (f1) d = MONE;
                break;
            case EXA_OP_ABS2:
                v = e.mul(u, u);
                if (f1) d = e.def("2.0 * " + u);
                if (f2) dd = "2.0";
                break;
            case EXA_OP_INV:
                v = e.def("1.0 / " + u);
                if (f1) d = e.def("-(" + v + " * " + v + ")");
                if (f2) dd = e.def("2.0 * " + v + " * " + v + " * " + v);
                break;
            case EXA_OP_SQRT:
                v = e.def("sqrt(" + u + ")");
                if (f1 || f2) d = e.def("0.5 / " + v);
                if (f2) dd = e.def("-0.5 * " + d + " / " + u);
                break;
            case EXA_OP_EXP:
                v = e.def("exp(" + u + ")");
                if (f1) d = v;
                if (f2) dd = v;
                break;
            case EXA_OP_LOG:
                v = e.def("log(" + u + ")");
                if (f1 || f2) d = e.def("1.0 / " + u);
                if (f2) dd = e.def("-(" + d + " * " + d + ")");
                break;
            case EXA_OP_SIN:
                v = e.def("sin(" + u + ")");
                if (f1) d = e.def("cos(" + u + ")");
                if (f2) dd = e.neg(v);
                break;
            case EXA_OP_COS:
                v = e.def("cos(" + u + ")");
                if (f1) d = e.neg(e.def("sin(" + u + ")"));
                if (f2) dd = e.neg(v);
                break;
            case EXA_OP_TAN:
                v = e.def("tan(" + u + ")");
                if (f1 || f2) d = e.def("1.0 + " + v + " * " + v);
                if (f2) dd = e.def("2.0 * " + v + " * " + d);
                break;
            case EXA_OP_ATAN:
                v = e.def("atan(" + u + ")");
                if (f1 || f2) d = e.def("1.0 / (1.0 + " + u + " * " + u + ")");
                if (f2) dd = e.def("-2.0 * " + u + " * " + d + " * " + d);
                break;
            case EXA_OP_SINH:
                v = e.def("sinh(" + u + ")");
                if (f1) d = e.def("cosh(" + u + ")");
                if (f2) dd = v;
                break;
            case EXA_OP_COSH:
                v = e.def("cosh(" + u + ")");
                if (f1) d = e.def("sinh(" + u + ")");
                if (f2) dd = v;
                break;
            case EXA_OP_TANH:
                v = e.def("tanh(" + u + ")");
                if (f1 || f2) d = e.def("1.0 - " + v + " * " + v);
                if (f2) dd = e.def("-2.0 * " + v + " * " + d);
                break;
            case EXA_OP_LOG1P:
                v = e.def("log1p(" + u + ")");
                if (f1 || f2) d = e.def("1.0 / (1.0 + " + u + ")");
                if (f2) dd = e.def("-(" + d + " * " + d + ")");
                break;
            case EXA_OP_EXPM1:
                v = e.def("expm1(" + u + ")");
                if (f1 || f2) d = e.def("exp(" + u + ")");
                if (f2) dd = d;
                break;
            default:
                fail(EXA_EINVAL, "codegen: unknown unary operator");
        }
    }

    static bool small_int(const TNode& q, int& n) {
        if (q.op != EXA_OP_CONST) return false;
        const double r = std::nearbyint(q.val);
        if (r != q.val || std::fabs(r) > 8) return false;
        n = (int)r;
        return true;
    }

    void binary(int i, bool first, bool second) {
        Em& e = e_;
        const TNode& q = t_[i];
        const std::string u = val_[q.a], w = val_[q.b];
        const bool ua = rev_active(q.a), wa = rev_active(q.b);
        const bool f1 = first && (ua || wa), f2 = second && (ua || wa);
        std::string& v = val_[i];
        std::string& dA = d1_[i];
        std::string& dB = d2_[i];
        switch (q.op) {
            case EXA_OP_ADD:
                v = e.add(u, w);
                if (f1) { dA = ONE; dB = ONE; }
                break;
            case EXA_OP_SUB:
                v = e.sub(u, w);
                if (f1) { dA = ONE; dB = MONE; }
                break;
            case EXA_OP_MUL:
                v = e.mul(u, w);
                if (f1) { dA = w; dB = u; }
                if (f2 && ua && wa) dab_[i] = ONE;
                break;
            case EXA_OP_DIV: {
                v = e.def(u + " / " + w);
                if (f1 || f2) {
                    const std::string iw = e.def("1.0 / " + w);
                    dA = iw;
                    if (wa) dB = e.def("-(" + v + " * " + iw + ")");
                    if (f2 && ua && wa) dab_[i] = e.def("-(" + iw + " * " + iw + ")");
                    if (f2 && wa) dbb_[i] = e.def("2.0 * " + v + " * " + iw + " * " + iw);
                }
                break;
            }
            case EXA_OP_POW: {
                int n = 0;
                if (!wa && small_int(t_[q.b], n)) {
                    v = e.def("exa_powi(" + u + ", " + std::to_string(n) + ")");
                    if (f1 || f2)
                        dA = e.def(std::to_string(n) + ".0 * exa_powi(" + u + ", " + std::to_string(n - 1) + ")");
                    if (f2)
                        daa_[i] = (n - 1 == 0) ? Z
                                  : e.def(std::to_string(n * (n - 1)) + ".0 * exa_powi(" + u + ", " +
                                          std::to_string(n - 2) + ")");
                } else if (!wa) {
                    v = e.def("pow(" + u + ", " + w + ")");
                    if (f1 || f2) dA = e.def(w + " * pow(" + u + ", " + w + " - 1.0)");
                    if (f2) daa_[i] = e.def(w + " * (" + w + " - 1.0) * pow(" + u + ", " + w + " - 2.0)");
                } else if (!ua) {
                    v = e.def("pow(" + u + ", " + w + ")");
                    if (f1 || f2) {
                        const std::string lu = e.def("log(" + u + ")");
                        dB = e.def(v + " * " + lu);
                        if (f2) dbb_[i] = e.def(dB + " * " + lu);
                    }
                } else {
                    v = e.def("pow(" + u + ", " + w + ")");
                    if (f1 || f2) {
                        const std::string lu = e.def("log(" + u + ")");
                        const std::string pm1 = e.def("pow(" + u + ", " + w + " - 1.0)");
                        dA = e.def(w + " * " + pm1);
                        dB = e.def(v + " * " + lu);
                        if (f2) {
                            daa_[i] = e.def(w + " * (" + w + " - 1.0) * pow(" + u + ", " + w + " - 2.0)");
                            dab_[i] = e.def(pm1 + " * (1.0 + " + w + " * " + lu + ")");
                            dbb_[i] = e.def(dB + " * " + lu);
                        }
                    }
                }
                break;
            }
            default:
                fail(EXA_EINVAL, "codegen: unknown binary operator");
        }
        if (!ua) { dA = Z; daa_[i] = Z; dab_[i] = Z; }
        if (!wa) { dB = Z; dbb_[i] = Z; dab_[i] = Z; }
    }

    // Reverse sweep: adjoint of every node from the root seed; var leaves
    // accumulate into J, param leaves (when with_par) into Pacc.
    void reverse(const std::string& seed, std::vector<std::string>& adj, std::vector<std::string>& J,
                 std::vector<std::string>& Pacc, bool with_par) {
        Em& e = e_;
        const int n = (int)t_.size();
        adj.assign(n, Z);
        adj[n - 1] = seed;
        for (int i = n - 1; i >= 0; --i) {
            const TNode& q = t_[i];
            const std::string& a = adj[i];
            if (q.op == EXA_OP_VAR) { J[q.slot] = e.add(J[q.slot], a); continue; }
            if (q.op == EXA_OP_PARAM) { if (with_par) Pacc[q.slot] = e.add(Pacc[q.slot], a); continue; }
            if (q.a < 0 || a == Z) continue;
            if (rev_active(q.a)) adj[q.a] = e.mul(a, d1_[i]);
            if (!is_unary(q.op) && rev_active(q.b)) adj[q.b] = e.mul(a, d2_[i]);
        }
    }

    // Forward tangent: SEED_DIR seeds 1 on var slot `dir`; SEED_VEC seeds v_s.
    void tangent(SeedKind kind, int dir, std::vector<std::string>& tg) {
        Em& e = e_;
        const int n = (int)t_.size();
        tg.assign(n, Z);
        for (int i = 0; i < n; ++i) {
            const TNode& q = t_[i];
            if (q.op == EXA_OP_VAR) {
                tg[i] = kind == SEED_DIR ? (q.slot == dir ? ONE : Z) : nm_.v[q.slot];
                continue;
            }
            if (q.a < 0) continue;
            if (is_unary(q.op))
                tg[i] = e.mul(d1_[i], tg[q.a]);
            else
                tg[i] = e.add(e.mul(d1_[i], tg[q.a]), e.mul(d2_[i], tg[q.b]));
        }
    }

    // Reverse sweep of the tangent (forward-over-reverse): the tangent of every
    // adjoint; var leaves accumulate into Hc, param leaves into Pt.
    void reverse_tangent(const std::vector<std::string>& adj, const std::vector<std::string>& tg,
                         std::vector<std::string>& Hc, std::vector<std::string>& Pt, bool with_par) {
        Em& e = e_;
        const int n = (int)t_.size();
        std::vector<std::string> ta(n, Z);
        for (int i = n - 1; i >= 0; --i) {
            const TNode& q = t_[i];
            if (q.op == EXA_OP_VAR) { Hc[q.slot] = e.add(Hc[q.slot], ta[i]); continue; }
            if (q.op == EXA_OP_PARAM) { if (with_par) Pt[q.slot] = e.add(Pt[q.slot], ta[i]); continue; }
            if (q.a < 0) continue;
            if (is_unary(q.op)) {
                if (!rev_active(q.a)) continue;
                const std::string td = e.mul(d2_[i], tg[q.a]);
                ta[q.a] = e.add(e.mul(ta[i], d1_[i]), e.mul(adj[i], td));
            } else {
                const std::string tdA = e.add(e.mul(daa_[i], tg[q.a]), e.mul(dab_[i], tg[q.b]));
                const std::string tdB = e.add(e.mul(dab_[i], tg[q.a]), e.mul(dbb_[i], tg[q.b]));
                if (rev_active(q.a)) ta[q.a] = e.add(e.mul(ta[i], d1_[i]), e.mul(adj[i], tdA));
                if (rev_active(q.b)) ta[q.b] = e.add(e.mul(ta[i], d2_[i]), e.mul(adj[i], tdB));
            }
        }
    }

    // Smallest set of tangent directions that covers every Hessian slot: each
    // diagonal slot needs its own variable, each off-diagonal one either end.
    std::vector<int> directions() const {
        const int k = P_.o1step();
        std::vector<int> best;
        int best_n = k + 1;
        if (k > 20) {
            for (int s = 0; s < k; ++s) best.push_back(s);
            return best;
        }
        for (unsigned mask = 0; mask < (1u << k); ++mask) {
            const int cnt = __builtin_popcount(mask);
            if (cnt >= best_n) continue;
            bool ok = true;
            for (auto& h : P_.hslots)
                if (!((mask >> h.first) & 1u) && !((mask >> h.second) & 1u)) { ok = false; break; }
            if (!ok) continue;
            best_n = cnt;
            best.clear();
            for (int s = 0; s < k; ++s)
                if ((mask >> s) & 1u) best.push_back(s);
        }
        return best;
    }

    template <class SlotName>
    void hessian(SlotName slot) {
        std::vector<std::string> J(P_.o1step(), Z), Pacc, adj;
        reverse(nm_.wgt, adj, J, Pacc, false);
        std::map<int, std::vector<std::string>> col;  // direction -> column
        for (int d : directions()) {
            std::vector<std::string> tg, Hc(P_.o1step(), Z), Pt;
            tangent(SEED_DIR, d, tg);
            reverse_tangent(adj, tg, Hc, Pt, false);
            col[d] = Hc;
        }
        for (int s = 0; s < P_.o2step(); ++s) {
            const int a = P_.hslots[s].first, b = P_.hslots[s].second;
            const std::string h = col.count(b) ? col[b][a] : col[a][b];
            const RefKey& ra = P_.vslots[a];
            const RefKey& rb = P_.vslots[b];
            // different slots over the same index column (or both literal)
            // have different offsets, so only different columns can alias
            const bool may_alias = a != b && ra.col != rb.col;
            if (may_alias && h != Z)
                e_.out(slot(s), "(" + nm_.ix[a] + " == " + nm_.ix[b] + ") ? 2.0 * " + h + " : " + h);
            else
                e_.out(slot(s), h);
        }
    }
};

int out_step(const Pattern& P, int mode) {
    switch (mode) {
        case M_HPROD: return (int)P.hvs.size();
        case M_GRAD: case M_JAC: case M_JTPROD: return P.o1step();
        case M_HESS: return P.o2step();
        case M_ADJ: return P.pstep();
        default: return 1;
    }
}

bool scalar_mode(int mode) { return mode == M_OBJ || mode == M_CONS || mode == M_JPROD; }

const char* mode_name(int m) {
    static const char* n[] = {"obj", "cons", "grad", "jac", "hess", "jprod", "jtprod", "hprod", "adj", "jh",
                              "sfull", "sipm"};
    return n[m];
}

bool multi_unit(int mode) { return multi_unit_mode(mode); }

// Staging through LDS is used while a workgroup's slice fits in this many
// doubles (64 KiB at the largest workgroup); wider patterns store directly.
constexpr int kLdsCapDoubles = 8192;

bool staged(const Pattern& P, int mode) { return out_step(P, mode) * EXA_BLOCK_MAX <= kLdsCapDoubles; }

// Output destination of member P's slice for data point kb (first of the
// workgroup's current points).
// (at_kb false: the start of the member's block, for slot-major buffers).
std::string dest(const Pattern& P, int mode, const std::string& pd, const std::string& out = "C.out0",
                 bool at_kb = true) {
    const std::string st = at_kb ? " + kb * " + std::to_string(out_step(P, mode)) : "";
    switch (mode) {
        case M_GRAD: return out + " + I.off[" + std::to_string(EXA_OFF_FO_OBJ) + "] + " + pd + ".ob" + st;
        case M_JAC: return out + " + I.off[" + std::to_string(EXA_OFF_JAC) + "] + " + pd + ".o1" + st;
        case M_JTPROD: return out + " + I.off[" + std::to_string(EXA_OFF_FO_CON) + "] + " + pd + ".ob" + st;
        case M_HPROD: return out + " + I.off[" + std::to_string(EXA_OFF_HV) + "] + " + pd + ".oh" + st;
        case M_HESS: return out + " + I.off[" + std::to_string(EXA_OFF_HESS) + "] + " + pd + ".o2" + st;
        case M_ADJ: return out + " + I.off[" + std::to_string(EXA_OFF_PAR) + "] + " + pd + ".op" + st;
        default: return "";
    }
}

// Modes whose per-point outputs go to a work buffer read back by a
// reduction (stored slot-major); the others write final outputs.
bool buffer_mode(int mode) { return mode == M_GRAD || mode == M_JTPROD || mode == M_HPROD || mode == M_ADJ; }

// The evaluations a unit performs for one data point: (pattern, sub-mode).
// A combined Jacobian + Hessian unit runs both sweeps of each member over
// one set of loads (Jacobian values to out0, Hessian values to out1).
struct Job {
    int p, mode;
    std::string out;
};

// Call record a job of `mode` reads and writes inside a unit of `umode`.
std::string call_of(int umode, int mode) { return multi_unit(umode) ? "C.c[" + std::to_string(mode) + "]" : "C"; }

std::vector<Job> jobs_of(const Model& M, int mode, const Unit& U) {
    std::vector<Job> j;
    for (int p : U.members) {
        if (mode != M_JH && !multi_unit(mode)) {
            j.push_back({p, mode, "C.out0"});
            continue;
        }
        for (int m : job_modes(mode))
            if (pattern_in_mode(M.pats[p], m))
                j.push_back({p, m, mode == M_JH ? (m == M_JAC ? "C.out0" : "C.out1") : call_of(mode, m) + ".out0"});
    }
    return j;
}

bool needs_weight(int mode) { return mode == M_HESS || mode == M_HPROD || mode == M_ADJ || mode == M_JTPROD; }

// Index columns the code replaces by the data point itself: the patterns'
// own flags, or (for code shared by a batch) the flags every instance has.
thread_local const std::vector<std::vector<char>>* g_ident = nullptr;
bool ident(const Model& M, int p, int c) {
    const std::vector<char>& f = g_ident ? (*g_ident)[p] : M.pats[p].ident;
    return c < (int)f.size() && f[c] != 0;
}

// H v references whose code may store into the output: the groups' own
// flags, or (for code shared by a batch) those of any instance.
thread_local const std::vector<std::vector<char>>* g_hvd = nullptr;
bool may_store_hv(const Model& M, int g, int at) {
    const std::vector<char>& f = g_hvd ? (*g_hvd)[g] : M.groups[g].hv_direct;
    return at < (int)f.size() && f[at] != 0;
}

// Value (cons) or tangent (jprod) of augmentation pattern a at one of its
// data points, for the base row that pulls it; fills `live`.
std::string aug_fn(const Model& M, int mode, int a, int& ntmp, UnitLive& live) {
    const Pattern& P = M.pats[a];
    std::ostringstream os;
    os << "__device__ __forceinline__ double aug_" << mode_name(mode) << "_" << a
       << "(const ExaCall& C, const ExaInstDev& I, long long k) {\n";
    os << "    const ExaPatDev& Pa = I.pat[" << a << "];\n";
    os << "    const double* __restrict__ X = C.x + I.off[" << EXA_OFF_X << "];\n";
    os << "    const double* __restrict__ V = C.v + I.off[" << EXA_OFF_X << "];\n";
    os << "    const double* __restrict__ TH = I.theta;\n";
    os << "    (void)X; (void)V; (void)TH;\n";
    os << "    double r = 0.0;\n";
    Em e(ntmp);
    std::set<int> icols, fcols;
    for (auto& r : P.vslots) if (r.col >= 0) icols.insert(r.col);
    for (auto& r : P.pslots) if (r.col >= 0) icols.insert(r.col);
    for (auto& q : P.nodes) if (q.op == EXA_OP_DATA) fcols.insert(q.col);
    for (int c : icols)
        e.named("long long", "ic" + std::to_string(c), ident(M, a, c) ? "k" : "Pa.ic[" + std::to_string(c) + "][k]");
    for (int c : fcols) e.named("double", "fc" + std::to_string(c), "Pa.fc[" + std::to_string(c) + "][k]");
    Names nm;
    for (int s = 0; s < P.o1step(); ++s) {
        const RefKey& k = P.vslots[s];
        const std::string off = "Pa.roff[" + std::to_string(s) + "]";
        const std::string idx = k.col < 0 ? off : "ic" + std::to_string(k.col) + " + " + off;
        e.named("long long", "ix" + std::to_string(s), idx);
        e.named("double", "x" + std::to_string(s), "X[ix" + std::to_string(s) + "]");
        if (mode == M_JPROD) e.named("double", "v" + std::to_string(s), "V[ix" + std::to_string(s) + "]");
        nm.x.push_back("x" + std::to_string(s));
        nm.v.push_back("v" + std::to_string(s));
        nm.ix.push_back("ix" + std::to_string(s));
    }
    for (int s = 0; s < P.pstep(); ++s) {
        const RefKey& k = P.pslots[s];
        const std::string off = "Pa.roff[" + std::to_string(P.o1step() + s) + "]";
        const std::string idx = k.col < 0 ? off : "ic" + std::to_string(k.col) + " + " + off;
        e.named("double", "p" + std::to_string(s), "TH[" + idx + "]");
        nm.p.push_back("p" + std::to_string(s));
    }
    PatternCg cg(P, mode, e, nm);
    cg.body("r");
    const std::set<std::string> names = e.emit(os, "    ");
    os << "    return r;\n}\n";
    for (int c : icols) if (names.count("ic" + std::to_string(c)) && !ident(M, a, c)) live.icols.push_back(c);
    for (int c : fcols) if (names.count("fc" + std::to_string(c))) live.fcols.push_back(c);
    for (int s = 0; s < P.o1step(); ++s) {
        if (names.count("x" + std::to_string(s))) live.vrefs.push_back(s);
        if (names.count("v" + std::to_string(s))) live.vseeds.push_back(s);
    }
    for (int s = 0; s < P.pstep(); ++s) if (names.count("p" + std::to_string(s))) live.prefs.push_back(s);
    return os.str();
}

// Generates the tile function of one unit; fills `live`.  A plain unit runs
// one callback's job per member (two for JH); a multi unit (M_SFULL,
// M_SIPM) runs every job of its modes per member from one set of loads and
// sweeps, each job with its own mode's call record of the ExaMulti.
std::string unit_tile(const Model& M, int mode, const Unit& U, int& ntmp, UnitLive& live) {
    const Group& G = M.groups[U.group];
    const int m0 = G.members[0];  // owner of the shared column pointers
    const bool multi = multi_unit(mode);
    const std::vector<int>& jm = job_modes(mode);
    auto has = [&](int m) { return std::find(jm.begin(), jm.end(), m) != jm.end(); };
    auto call = [&](int m) { return call_of(mode, m); };
    std::ostringstream os;
    const std::string fn = std::string("unit_") + mode_name(mode) + "_" + std::to_string(U.code);
    os << "__device__ __forceinline__ void " << fn << "(const " << (multi ? "ExaMulti" : "ExaCall")
       << "& C, const ExaInstDev& I, const ExaTile& T, double* lds) {\n";
    os << "    const ExaPatDev& P0 = I.pat[" << m0 << "];\n";
    for (int p : U.members) os << "    const ExaPatDev& P" << p << "_ = I.pat[" << p << "];\n";
    // inputs: x for every job; v seeds jprod/hprod; y weighs hess/hprod
    // (sigma for objectives); w weighs jtprod (in a plain jtprod call it is C.y)
    const std::string cx = multi ? call(M_JAC) : "C", cv = multi ? call(M_JPROD) : "C",
                      cy = multi ? call(M_HESS) : "C", cw = multi ? call(M_JTPROD) : "C";
    os << "    const double* __restrict__ X = " << cx << ".x + I.off[" << EXA_OFF_X << "];\n";
    os << "    const double* __restrict__ V = " << cv << ".v + I.off[" << EXA_OFF_X << "];\n";
    os << "    const double* __restrict__ Y = " << cy << ".y + I.off[" << EXA_OFF_Y << "];\n";
    os << "    const double* __restrict__ W = " << cw << ".y + I.off[" << EXA_OFF_Y << "];\n";
    os << "    const double* __restrict__ TH = I.theta;\n";
    os << "    (void)X; (void)V; (void)Y; (void)W; (void)TH; (void)P0;\n";
    os << "    const int nthr = (int)blockDim.x;\n";
    os << "    const long long kend = T.start + T.count;\n";
    if (mode == M_OBJ) {
        // virtual lanes (see exa_vlane_sum): one pass per lane this thread holds
        // every round is unrolled and branch-free (lanes past the end
        // recompute the last point and add 0.0, as an empty lane always
        // did), so the loads of all the tile's points can be in flight at once
        os << "    double acc[EXA_VLANES / 64] = {};\n";
        os << "#pragma unroll\n";
        os << "    for (int rd = 0; rd < EXA_OBJ_ROUNDS; ++rd) {\n";
        os << "        const long long kb = T.start + (long long)rd * EXA_VLANES;\n";
        os << "#pragma unroll\n";
        os << "    for (int q = 0; q < EXA_VLANES / 64; ++q) {\n";
        os << "        if (q * nthr >= EXA_VLANES) break;\n";
        os << "        const long long kr = kb + threadIdx.x + q * nthr;\n";
        os << "        const long long k = kr < kend ? kr : kend - 1;\n";
    } else {
        os << "    for (long long kb = T.start; kb < kend; kb += nthr) {\n";
        os << "        const long long kr = kb + threadIdx.x;\n";
        os << "        const int npts = (int)((kend - kb) < nthr ? (kend - kb) : nthr);\n";
        // every lane runs the statements (no divergent region around them),
        // so that each job's staged store (workgroup barriers) can follow its
        // sweep: lanes past the end recompute the last point and store nothing
        os << "        const long long k = kr < kend ? kr : kend - 1;\n";
    }
    const std::vector<Job> jobs = jobs_of(M, mode, U);
    const bool several = jm.size() > 1;
    auto oname = [&](const Job& j) {
        return (scalar_mode(j.mode) ? "r" : "o") + std::to_string(j.p) + (several ? std::string("_") + mode_name(j.mode) : "");
    };
    for (const Job& j : jobs) {
        if (scalar_mode(j.mode))
            os << "        double " << oname(j) << " = 0.0;\n";
        else
            os << "        double " << oname(j) << "[" << out_step(M.pats[j.p], j.mode) << "] = {};\n";
    }
    // J^T w / H v: the members' contributions summed per group reference
    const Group& UG = M.groups[U.group];
    std::map<int, std::string> gout;  // mode -> output array of its first job
    for (const Job& j : jobs)
        if ((j.mode == M_JTPROD || j.mode == M_HPROD) && !gout.count(j.mode)) gout[j.mode] = j.out;
    auto gname = [](int m) { return std::string(m == M_JTPROD ? "gjt" : "ghv"); };
    auto grefs = [&](int m) -> const std::vector<int>& { return m == M_JTPROD ? UG.jt_refs : UG.hv_refs; };
    // (mode, group slot) -> the last member whose job adds to it
    std::map<std::pair<int, int>, int> last_adder;
    for (const Job& j : jobs) {
        if (j.mode != M_JTPROD && j.mode != M_HPROD) continue;
        const Pattern& P = M.pats[j.p];
        const std::vector<int>& refs = grefs(j.mode);
        for (int i = 0; i < out_step(P, j.mode); ++i) {
            const int r = P.vg[j.mode == M_HPROD ? P.hvs[i] : i];
            last_adder[{j.mode, (int)(std::find(refs.begin(), refs.end(), r) - refs.begin())}] = j.p;
        }
    }
    for (auto& kv : gout)
        os << "        double " << gname(kv.first) << "[" << std::max<size_t>(1, grefs(kv.first).size()) << "] = {};\n";
    os << "        {\n";

    // ---- statements: loads (all candidates), then every job's sweeps
    bool weighs = false, seeds = false;
    for (int m : jm) {
        weighs |= needs_weight(m);
        seeds |= m == M_JPROD || m == M_HPROD || m == M_ADJ;
    }
    Em e(ntmp);
    std::set<int> icols, fcols;
    for (int p : U.members) {
        const Pattern& P = M.pats[p];
        for (auto& r : P.vslots) if (r.col >= 0) icols.insert(r.col);
        for (auto& r : P.pslots) if (r.col >= 0) icols.insert(r.col);
        for (auto& q : P.nodes) if (q.op == EXA_OP_DATA) fcols.insert(q.col);
        if (weighs && P.kind == EXA_AUG) icols.insert(P.row_icol);
    }
    const int p0 = U.members[0];  // the unit's data arrays
    for (int c : icols)
        e.named("long long", "ic" + std::to_string(c), ident(M, p0, c) ? "k" : "P0.ic[" + std::to_string(c) + "][k]");
    for (int c : fcols) e.named("double", "fc" + std::to_string(c), "P0.fc[" + std::to_string(c) + "][k]");
    std::set<int> vrefs, prefs;
    for (int p : U.members) {
        for (int r : M.pats[p].vg) vrefs.insert(r);
        for (int r : M.pats[p].pg) prefs.insert(r);
    }
    for (int r : vrefs) {
        const RefKey& k = G.vrefs[r];
        const std::pair<int, int> src = G.vsrc[r];
        const std::string off = "I.pat[" + std::to_string(G.members[src.first]) + "].roff[" +
                                std::to_string(src.second) + "]";
        const std::string idx = k.col < 0 ? off : "ic" + std::to_string(k.col) + " + " + off;
        e.named("long long", "ix" + std::to_string(r), idx);
        e.named("double", "x" + std::to_string(r), "X[ix" + std::to_string(r) + "]");
        if (seeds) e.named("double", "v" + std::to_string(r), "V[ix" + std::to_string(r) + "]");
    }
    for (int r : prefs) {
        const RefKey& k = G.prefs[r];
        const std::pair<int, int> src = G.psrc[r];
        const int member = G.members[src.first];
        // a parameter slot's offset sits after the member's variable slots
        const std::string off = "I.pat[" + std::to_string(member) + "].roff[" +
                                std::to_string(M.pats[member].o1step() + src.second) + "]";
        const std::string idx = k.col < 0 ? off : "ic" + std::to_string(k.col) + " + " + off;
        e.named("double", "p" + std::to_string(r), "TH[" + idx + "]");
    }
    for (const Job& j : jobs) {
        const int p = j.p;
        const Pattern& P = M.pats[p];
        const std::string pd = "P" + std::to_string(p) + "_";
        Names nm;
        for (int s = 0; s < P.o1step(); ++s) {
            nm.x.push_back("x" + std::to_string(P.vg[s]));
            nm.v.push_back("v" + std::to_string(P.vg[s]));
            nm.ix.push_back("ix" + std::to_string(P.vg[s]));
        }
        for (int s = 0; s < P.pstep(); ++s) nm.p.push_back("p" + std::to_string(P.pg[s]));
        if (needs_weight(j.mode)) {
            // row weight: w for J^T w, y (sigma for objectives) otherwise
            const bool byw = j.mode == M_JTPROD;
            const std::string src = byw ? "W" : "Y";
            std::string w;
            if (P.kind == EXA_OBJ)
                w = cy + ".sigma";
            else if (P.kind == EXA_CON)
                w = src + "[" + pd + ".o0 + k]";
            else
                w = src + "[" + pd + ".tgt0 + ic" + std::to_string(P.row_icol) + " + " + pd + ".row_off]";
            nm.wgt = e.named_once("double", (byw ? "ww" : "wy") + std::to_string(p), w);
        }
        PatternCg cg(P, j.mode, e, nm);
        cg.body(oname(j));
        if (j.mode == M_GRAD)
            // every variable has at most one contribution: write g directly
            for (int s = 0; s < P.o1step(); ++s)
                e.out("if (" + call(M_GRAD) + ".direct && kr < kend) " + call(M_GRAD) + ".out0[I.off[" +
                          std::to_string(EXA_OFF_X) + "] + " + nm.ix[s] + "]",
                      oname(j) + "[" + std::to_string(s) + "]");
        if (j.mode == M_JTPROD || j.mode == M_HPROD) {
            // this member's contributions added to the group's, members in
            // declaration order; a reference's sum is stored (slot-major, as
            // exa_store_soa does) right after the last member that adds to
            // it, so that it leaves registers early
            const std::vector<int>& refs = grefs(j.mode);
            const int n = out_step(P, j.mode);
            const std::string stride = "((" + pd + ".ndata + 15) & ~15LL)";
            for (int i = 0; i < n; ++i) {
                const int r = P.vg[j.mode == M_HPROD ? P.hvs[i] : i];
                const int at = (int)(std::find(refs.begin(), refs.end(), r) - refs.begin());
                const std::string g = gname(j.mode) + "[" + std::to_string(at) + "]";
                e.out(g, g + " + " + oname(j) + "[" + std::to_string(i) + "]");
                if (last_adder[{j.mode, at}] != p) continue;
                const std::string buf = "(" + dest(P, j.mode, pd, j.out, false) + ")[" + std::to_string(at) + " * " +
                                        stride + " + kr] = " + g + ";";
                if (j.mode == M_HPROD && at < 32 && may_store_hv(M, U.group, at))
                    // a reference whose entries are their variables' only H v
                    // contributions (this instance's bit) goes to the output
                    e.raw("if (kr < kend) { if ((" + pd + ".hvd >> " + std::to_string(at) + ") & 1) " +
                          call(M_HPROD) + ".out1[I.off[" + std::to_string(EXA_OFF_X) + "] + ix" + std::to_string(r) +
                          "] = " + g + "; else " + buf + " }");
                else
                    e.raw("if (kr < kend) " + buf);
            }
        } else if (buffer_mode(j.mode)) {
            // contributions to a work buffer that a reduction reads back: slot
            // s of data point k at block + s * stride + k (stride: ndata
            // rounded up to 16, so every slot array starts on a 128-byte
            // line), one coalesced store per slot and no staging (the
            // reduction's gathers of one slot over neighbouring points are
            // then neighbouring too)
            std::string line = j.mode == M_GRAD ? "if (!" + call(M_GRAD) + ".direct) " : "";
            line += "exa_store_soa<" + std::to_string(out_step(P, j.mode)) + ">(" + dest(P, j.mode, pd, j.out, false) +
                    ", (" + pd + ".ndata + 15) & ~15LL, kr, kend, " + oname(j) + ");";
            e.raw(line);
        } else if (!scalar_mode(j.mode)) {
            // this job's outputs leave registers as soon as they are complete
            const bool final_out = j.mode == M_JAC || j.mode == M_HESS;
            const std::string st = std::to_string(out_step(P, j.mode)), nt = final_out ? "true" : "false";
            const std::string args = "(" + dest(P, j.mode, pd, j.out) + ", " + oname(j) + ", npts, lds);";
            std::string line;
            if (staged(P, j.mode) && out_step(P, j.mode) > 1)
                // staged through LDS into contiguous 16-byte stores, unless the
                // call asks for each lane's own stores (a schedule choice; the
                // flag is the same for the whole workgroup)
                line = "if (" + call(j.mode) + ".unstaged) exa_store_direct<" + st + ", " + nt + ">" + args +
                       " else exa_store<" + st + ", " + nt + ">" + args;
            else if (staged(P, j.mode))
                line = "exa_store<" + st + ", " + nt + ">" + args;
            else
                line = "exa_store_direct<" + st + ", " + nt + ">" + args;
            e.raw(line);
        }
    }
    const std::set<std::string> names = e.emit(os, "            ");

    // ---- augmentation pulls of the scalar jobs (cons values, jprod tangents)
    // Base rows pull the augmentation terms that add to them, in declaration
    // order of the augmentations, points ascending.  Terms are evaluated in
    // rounds of R before any of the round is added, so that their chains of
    // dependent loads (row bounds, term index, data, x) overlap; the first
    // round of every pull is issued before any addition.  Augmentations over
    // the same data arrays whose rows come from the same index column and
    // offset have the same row lists (their targets are members of this unit,
    // hence of one size): they share one walk (row bounds and term indices).
    // The additions keep the order.
    struct Pull {
        std::string out;
        int a, R, mode, walk;
    };
    std::vector<Pull> pulls;
    for (const Job& j : jobs) {
        const Pattern& P = M.pats[j.p];
        if ((j.mode != M_CONS && j.mode != M_JPROD) || P.kind != EXA_CON) continue;
        for (int a : P.augs) {
            if (M.pats[a].ndata == 0) continue;
            const size_t nn = M.pats[a].nodes.size();
            pulls.push_back({oname(j), a, nn <= 16 ? 4 : nn <= 64 ? 2 : 1, j.mode, a});
        }
    }
    for (Pull& q : pulls)
        for (const Pull& r : pulls)
            if (same_walk(M, r.a, q.a)) {
                q.walk = r.a;
                break;
            }
    // at most kPullTerms terms in flight per lane, shared by the pulls, so
    // that a round does not cost occupancy
    constexpr int kPullTerms = 12;
    const int share = pulls.empty() ? 1 : std::max(1, kPullTerms / (int)pulls.size());
    for (Pull& q : pulls) q.R = std::min(q.R, share);
    // one round size per walk: the smallest of its pulls'
    std::map<int, int> walk_R;
    for (const Pull& q : pulls) walk_R[q.walk] = walk_R.count(q.walk) ? std::min(walk_R[q.walk], q.R) : q.R;
    for (Pull& q : pulls) q.R = walk_R[q.walk];
    auto wname = [](int w) { return std::to_string(w); };
    for (auto& wr : walk_R) {
        const std::string pa = "I.pat[" + wname(wr.first) + "]", w = wname(wr.first);
        os << "            const int ab" << w << " = " << pa << ".rptr[k], ae" << w << " = " << pa << ".rptr[k + 1];\n";
        for (int i = 0; i < wr.second; ++i)
            os << "            const long long at" << w << "_" << i << " = " << pa << ".ridx[exa_term(ab" << w << " + "
               << i << ", ae" << w << ")];\n";
    }
    auto aq = [&](const Pull& q, int i) {
        return "aq" + std::to_string(q.a) + "_" + mode_name(q.mode) + "_" + std::to_string(i);
    };
    auto fn_of = [&](const Pull& q) {
        return std::string("aug_") + mode_name(q.mode) + "_" + std::to_string(q.a) + "(" + call(q.mode) + ", I, ";
    };
    for (const Pull& q : pulls)
        for (int i = 0; i < q.R; ++i)
            os << "            const double " << aq(q, i) << " = " << fn_of(q) << "at" << wname(q.walk) << "_" << i
               << ");\n";
    live.pulls = !pulls.empty();
    for (const Pull& q : pulls) {
        const std::string w = wname(q.walk), pa = "I.pat[" + w + "]";
        for (int i = 0; i < q.R; ++i)
            os << "            if (ab" << w << " + " << i << " < ae" << w << ") " << q.out << " += " << aq(q, i) << ";\n";
        // later rounds: the round's term indices and values first, then
        // its additions in order
        os << "            for (int j0 = ab" << w << " + " << q.R << "; j0 < ae" << w << "; j0 += " << q.R << ") {\n";
        for (int i = 0; i < q.R; ++i)
            os << "                const double u" << i << " = " << fn_of(q) << "(long long)" << pa << ".ridx["
               << (i == 0 ? std::string("j0") : "exa_term(j0 + " + std::to_string(i) + ", ae" + w + ")") << "]);\n";
        for (int i = 0; i < q.R; ++i)
            os << "                " << (i ? "if (j0 + " + std::to_string(i) + " < ae" + w + ") " : std::string())
               << q.out << " += u" << i << ";\n";
        os << "            }\n";
    }
    os << "        }\n";

    // ---- liveness record
    for (int c : icols) if (names.count("ic" + std::to_string(c)) && !ident(M, p0, c)) live.icols.push_back(c);
    for (int c : fcols) if (names.count("fc" + std::to_string(c))) live.fcols.push_back(c);
    for (int r : vrefs) {
        if (names.count("x" + std::to_string(r))) live.vrefs.push_back(r);
        if (names.count("v" + std::to_string(r))) live.vseeds.push_back(r);
    }
    for (int r : prefs) if (names.count("p" + std::to_string(r))) live.prefs.push_back(r);
    for (int p : U.members)
        // an objective's weight is the scalar sigma, not a per-point load
        if (M.pats[p].kind != EXA_OBJ)
            for (const char* w : {"wy", "ww"})
                if (names.count(w + std::to_string(p))) live.weights++;
    for (const Job& j : jobs)
        if (j.mode != M_JTPROD && j.mode != M_HPROD) live.outputs += out_step(M.pats[j.p], j.mode);
    for (auto& kv : gout) live.outputs += (int64_t)grefs(kv.first).size();

    // ---- outputs that are not staged: objective sums, constraint rows
    if (mode == M_OBJ) {
        std::string sum;
        for (const Job& j : jobs) sum += (sum.empty() ? "" : " + ") + oname(j);
        os << "        acc[q] += kr < kend ? " << (jobs.size() > 1 ? "(" + sum + ")" : sum) << " : 0.0;\n";
        os << "    }\n";  // virtual lanes
    }
    for (const Job& j : jobs)
        if (j.mode == M_CONS || j.mode == M_JPROD)
            os << "        if (kr < kend) __builtin_nontemporal_store(" << oname(j) << ", &" << call(j.mode) << ".out0[I.off["
               << EXA_OFF_ROWS << "] + P" << j.p << "_.o0 + k]);\n";
    os << "    }\n";
    if (mode == M_OBJ) {
        os << "    const double tot = exa_vlane_sum(acc, lds);\n";
        os << "    if (threadIdx.x == 0) C.out0[I.off[" << EXA_OFF_TILE << "] + T.slot] = tot;\n";
    }
    os << "}\n";
    return os.str();
}

}  // namespace

const std::vector<int>& job_modes(int mode) {
    static const std::vector<int> one[M_COUNT] = {{0}, {1}, {2}, {3}, {4}, {5}, {6}, {7}, {8}, {M_JAC, M_HESS}};
    // J^T w runs as tiles of its own beside the one-pass units (with it, the
    // units hold too many registers)
    static const std::vector<int> full = {M_GRAD, M_CONS, M_JAC, M_HESS, M_JPROD, M_HPROD};
    static const std::vector<int> ipm = {M_GRAD, M_CONS, M_JAC, M_HESS};
    return mode == M_SFULL ? full : mode == M_SIPM ? ipm : one[mode];
}

bool pattern_in_mode(const Pattern& P, int mode) {
    if (P.ndata == 0) return false;
    if (multi_unit(mode)) {
        for (int m : job_modes(mode))
            if (pattern_in_mode(P, m)) return true;
        return false;
    }
    switch (mode) {
        case M_OBJ: return P.kind == EXA_OBJ;
        case M_CONS: return P.kind == EXA_CON;
        case M_GRAD: return P.kind == EXA_OBJ && P.o1step() > 0;
        case M_JAC: return P.kind != EXA_OBJ && P.o1step() > 0;
        case M_HESS: return P.o2step() > 0;
        case M_JPROD: return P.kind == EXA_CON;
        case M_JTPROD: return P.kind != EXA_OBJ && P.o1step() > 0 && !P.wread;
        case M_HPROD: return P.o2step() > 0;
        case M_ADJ: return P.pstep() > 0 && P.o1step() > 0;
        case M_JH: return pattern_in_mode(P, M_JAC) || pattern_in_mode(P, M_HESS);
        default: return false;
    }
}

std::vector<Unit> units_for(const Model& M, int mode, bool fused) {
    // J^T w and H v contributions are summed over a group's members in the
    // lane: their units always hold the whole group
    if (mode == M_JTPROD || mode == M_HPROD) fused = true;
    if (multi_unit(mode))
        for (int m : job_modes(mode)) fused = fused || m == M_JTPROD || m == M_HPROD;
    std::vector<Unit> out;
    for (size_t g = 0; g < M.groups.size(); ++g) {
        const Group& G = M.groups[g];
        std::vector<int> in;
        for (int p : G.members)
            if (pattern_in_mode(M.pats[p], mode)) in.push_back(p);
        if (in.empty()) continue;
        if (fused && in.size() > 1) {
            Unit u;
            u.code = EXA_MAX_PATTERNS + (int)g;
            u.group = (int)g;
            u.members = in;
            u.ndata = G.ndata;
            out.push_back(u);
        } else {
            for (int p : in) {
                Unit u;
                u.code = p;
                u.group = (int)g;
                u.members = {p};
                u.ndata = M.pats[p].ndata;
                out.push_back(u);
            }
        }
    }
    // declaration order of the first member keeps tile lists stable
    std::stable_sort(out.begin(), out.end(),
                     [](const Unit& a, const Unit& b) { return a.members[0] < b.members[0]; });
    return out;
}

int mode_lds_doubles(const Model& M, int mode) {
    if (mode == M_JH || multi_unit(mode)) {
        int d = EXA_BLOCK_MAX;
        for (int m : job_modes(mode)) d = std::max(d, mode_lds_doubles(M, m));
        return d;
    }
    int st = 1;
    if (!buffer_mode(mode))
        for (auto& P : M.pats)
            if (pattern_in_mode(P, mode) && staged(P, mode)) st = std::max(st, out_step(P, mode));
    return st * EXA_BLOCK_MAX;
}

std::string kernel_name(int mode) { return std::string("exa_k_") + mode_name(mode); }

const std::vector<int>& multi_modes(bool jh) {
    static const std::vector<int> m = {M_OBJ, M_GRAD, M_CONS, M_JAC, M_HESS, M_JPROD, M_JTPROD, M_HPROD};
    static const std::vector<int> mjh = {M_OBJ, M_GRAD, M_CONS, M_JH, M_JPROD, M_JTPROD, M_HPROD};
    return jh ? mjh : m;
}

std::string generate_source(const Model& M, std::map<std::pair<int, int>, UnitLive>* live,
                            const std::vector<std::vector<char>>* ident_flags,
                            const std::vector<std::vector<char>>* hvd_flags) {
    struct Restore {
        const std::vector<std::vector<char>>* prev;
        const std::vector<std::vector<char>>** where;
        ~Restore() { *where = prev; }
    } restore_ident{g_ident, &g_ident}, restore_hvd{g_hvd, &g_hvd};
    g_ident = ident_flags;
    g_hvd = hvd_flags;
    std::ostringstream os;
    os << "// generated: straight-line evaluation kernels for one pattern set\n";
    os << EXA_STR(EXA_DEVICE_STRUCTS) << "\n";
    os << "static_assert(sizeof(ExaPatDev) == " << sizeof(ExaPatDev) << ", \"layout\");\n";
    os << "static_assert(sizeof(ExaInstDev) == " << sizeof(ExaInstDev) << ", \"layout\");\n";
    os << "static_assert(sizeof(ExaTile) == " << sizeof(ExaTile) << ", \"layout\");\n";
    os << "static_assert(sizeof(ExaCall) == " << sizeof(ExaCall) << ", \"layout\");\n";
    std::string pre = R"(
__device__ __forceinline__ double exa_powi(double u, int n) {
    double r = 1.0, b = u;
    unsigned m = n < 0 ? (unsigned)(-n) : (unsigned)n;
    while (m) { if (m & 1u) r *= b; b *= b; m >>= 1; }
    return n < 0 ? 1.0 / r : r;
}
// Writes the per-lane slices of `npts` consecutive data points (ST doubles
// each) to dst through LDS, so that the workgroup stores contiguous memory.
// NT marks final outputs, written with non-temporal stores: they are never
// read back by the kernel, and streaming them past the caches keeps x and the
// data columns resident (intermediate buffers read back by a reduction use
// ordinary stores).
typedef double exa_d2 __attribute__((ext_vector_type(2)));
template <int ST, bool NT>
__device__ __forceinline__ void exa_store(double* __restrict__ dst, const double* o, int npts, double* lds) {
    if (ST == 1) {
        if ((int)threadIdx.x < npts) {
            if (NT) __builtin_nontemporal_store(o[0], &dst[threadIdx.x]);
            else dst[threadIdx.x] = o[0];
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < ST; ++s) lds[threadIdx.x * ST + s] = o[s];
    __syncthreads();
    // 16-byte stores from dst's first 16-byte boundary on; the element
    // before it (dst is only 8-byte aligned) and an odd last element are
    // stored on their own
    const int n = npts * ST;
    const int a = (int)(((unsigned long long)dst >> 3) & 1ull);
    const int h = a < n ? a : n;
    const int n2 = (n - h) >> 1;
    for (int i = threadIdx.x; i < n2; i += (int)blockDim.x) {
        exa_d2 v;
        v.x = lds[h + 2 * i];
        v.y = lds[h + 2 * i + 1];
        exa_d2* p = (exa_d2*)(dst + h + 2 * i);
        if (NT) __builtin_nontemporal_store(v, p);
        else *p = v;
    }
    if (threadIdx.x == 0) {
        if (h) {
            if (NT) __builtin_nontemporal_store(lds[0], &dst[0]);
            else dst[0] = lds[0];
        }
        const int last = h + 2 * n2;
        if (last < n) {
            if (NT) __builtin_nontemporal_store(lds[last], &dst[last]);
            else dst[last] = lds[last];
        }
    }
    __syncthreads();
}
// Zeros to dst[0 .. n) by the whole workgroup: 16-byte stores from dst's
// first 16-byte boundary on, the element before it and an odd last element
// on their own (ordinary stores: a reduction may read the entries back).
__device__ __forceinline__ void exa_zero_fill(double* __restrict__ dst, long long n) {
    const long long h = ((((unsigned long long)dst >> 3) & 1ull) && n > 0) ? 1 : 0;
    const long long n2 = (n - h) >> 1;
    exa_d2 z;
    z.x = 0.0;
    z.y = 0.0;
    for (long long i = threadIdx.x; i < n2; i += blockDim.x) *(exa_d2*)(dst + h + 2 * i) = z;
    if (threadIdx.x == 0) {
        if (h) dst[0] = 0.0;
        if (h + 2 * n2 < n) dst[n - 1] = 0.0;
    }
}
// Slot-major store to a work buffer: slot s of data point k at
// base[s * n + k], n the padded slot stride (lanes past the end of the tile
// store nothing).
template <int ST>
__device__ __forceinline__ void exa_store_soa(double* __restrict__ base, long long n, long long k, long long kend,
                                              const double* o) {
    if (k < kend) {
#pragma unroll
        for (int s = 0; s < ST; ++s) base[s * n + k] = o[s];
    }
}
// Direct (unstaged) variant: each lane stores its own slice (slices too wide
// for LDS, or when the call asks for unstaged stores); NT as in exa_store.
template <int ST, bool NT>
__device__ __forceinline__ void exa_store_direct(double* __restrict__ dst, const double* o, int npts, double*) {
    if ((int)threadIdx.x < npts) {
#pragma unroll
        for (int s = 0; s < ST; ++s) {
            if (NT) __builtin_nontemporal_store(o[s], &dst[threadIdx.x * ST + s]);
            else dst[threadIdx.x * ST + s] = o[s];
        }
    }
}
// Objective tiles are summed over 256 virtual lanes whatever the workgroup
// width: virtual lane l takes points l, l + 256, ... of the tile in order,
// thread t holds lanes t, t + blockDim.x, ...; the 256 lane sums then go
// through a fixed tree in LDS.  The order never depends on the launch.
#define EXA_VLANES 256
__device__ __forceinline__ double exa_vlane_sum(const double* acc, double* lds) {
    const int nthr = (int)blockDim.x;
#pragma unroll
    for (int q = 0; q < EXA_VLANES / 64; ++q)
        if (q * nthr < EXA_VLANES) lds[threadIdx.x + q * nthr] = acc[q];
    __syncthreads();
    for (int s = EXA_VLANES / 2; s > 0; s >>= 1) {
        for (int t = threadIdx.x; t < s; t += nthr) lds[t] += lds[t + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();  // lds is free again for the next tile
    return r;
}
// Index of the i-th augmentation term of a row whose terms are
// ridx[jb, je), clamped into [0, je) so that every lane loads a valid term
// even when its row has fewer (the surplus values are not added).  Valid
// when the pattern has at least one data point.
__device__ __forceinline__ int exa_term(int j, int je) { return j < je ? j : (je > 0 ? je - 1 : 0); }
)";
    os << pre;
    static_assert(kObjBlock * kObjEpl % 256 == 0, "objective tiles hold whole rounds of 256 virtual lanes");
    os << "// rounds of EXA_VLANES points in one objective tile\n#define EXA_OBJ_ROUNDS " << kObjBlock * kObjEpl / 256
       << "\n";
    int ntmp = 0;
    // Tile loop shared by every kernel: one tile per workgroup; workgroup w
    // runs on XCD w % 8, so tile indices are remapped to give each XCD a
    // contiguous range.
    auto kernel = [&](const std::string& name, int lds, const std::vector<std::string>& cases) {
        os << "extern \"C\" __global__ void __launch_bounds__(" << EXA_BLOCK_MAX << ") " << name << "(ExaCall C) {\n";
        os << "    __shared__ double lds[" << lds << "];\n";
        os << "    (void)lds;\n";
        os << "    {\n";
        os << "        const long long w = (blockIdx.x % 8) * C.per_xcd + blockIdx.x / 8;\n";
        os << "        if (w >= C.ntiles) return;\n";
        os << "        const ExaTile T = C.tiles[w];\n";
        os << "        const ExaInstDev& I = C.inst[T.inst];\n";
        os << "        switch (T.pat) {\n";
        for (auto& c : cases) os << "            " << c << "\n";
        os << "            default: break;\n";
        os << "        }\n";
        os << "    }\n";
        os << "}\n";
    };
    for (int mode = 0; mode < M_COUNT; ++mode) {
        // units of both schedules (separate patterns, fused groups)
        std::map<int, Unit> all;
        for (int fused = 0; fused < 2; ++fused)
            for (auto& u : units_for(M, mode, fused != 0)) all[u.code] = u;
        if (mode == M_CONS || mode == M_JPROD)
            for (size_t a = 0; a < M.pats.size(); ++a)
                if (M.pats[a].kind == EXA_AUG && M.pats[a].ndata > 0) {
                    UnitLive L;
                    os << aug_fn(M, mode, (int)a, ntmp, L);
                    if (live) (*live)[{mode, 1000 + (int)a}] = L;
                }
        std::vector<std::string> cases;
        for (auto& kv : all) {
            UnitLive L;
            os << unit_tile(M, mode, kv.second, ntmp, L);
            if (live) (*live)[{mode, kv.first}] = L;
            cases.push_back("case " + std::to_string(kv.first) + ": unit_" + mode_name(mode) + "_" +
                            std::to_string(kv.first) + "(C, I, T, lds); break;");
        }
        if (mode == M_GRAD)  // entries of g no objective term touches
            cases.push_back("case " + std::to_string(EXA_ZERO_TILE) + ": exa_zero_fill(C.out0 + I.off[" +
                            std::to_string(EXA_OFF_X) + "] + T.start, T.count); break;");
        kernel(kernel_name(mode), mode_lds_doubles(M, mode), cases);
    }
    // Several callbacks in one launch: a tile's mode sits above
    // EXA_MODE_SHIFT in its code, and its case passes that mode's call (a
    // constant index, so the calls stay in kernel arguments).  One tile per
    // workgroup, remapped per XCD as in the single-callback kernels.
    // exa_k_multi runs per-callback tiles; exa_k_onepass runs multi units
    // (every selected job of a point from one set of loads) with the
    // objective's and the gradient's zero tiles.  Two kernels, so that each
    // gets the register budget of its own cases.
    auto multi_kernel = [&](const std::string& name, int lds, const std::vector<std::string>& cases, int min_waves) {
        os << "extern \"C\" __global__ void __launch_bounds__(" << EXA_BLOCK_MAX;
        if (min_waves) os << ", " << min_waves;
        os << ") " << name << "(ExaMulti C) {\n";
        os << "    __shared__ double lds[" << lds << "];\n";
        os << "    (void)lds;\n";
        os << "    const long long w = (blockIdx.x % 8) * C.per_xcd + blockIdx.x / 8;\n";
        os << "    if (w >= C.ntiles) return;\n";
        os << "    const ExaTile T = C.tiles[w];\n";
        os << "    switch (T.pat) {\n";
        for (auto& c : cases) os << "        " << c << "\n";
        os << "        default: break;\n";
        os << "    }\n";
        os << "}\n";
    };
    auto mode_cases = [&](int mode, std::vector<std::string>& cases) {
        std::set<int> codes;
        for (int fused = 0; fused < 2; ++fused)
            for (auto& u : units_for(M, mode, fused != 0)) codes.insert(u.code);
        const std::string K = "C.c[" + std::to_string(mode) + "]";
        for (int c : codes)
            cases.push_back("case " + std::to_string((mode << EXA_MODE_SHIFT) | c) + ": unit_" + mode_name(mode) + "_" +
                            std::to_string(c) + "(" + K + ", " + K + ".inst[T.inst], T, lds); break;");
    };
    const std::string G = "C.c[" + std::to_string(M_GRAD) + "]";
    const std::string zero_case = "case " + std::to_string((M_GRAD << EXA_MODE_SHIFT) | EXA_ZERO_TILE) +
                                  ": exa_zero_fill(" + G + ".out0 + " + G + ".inst[T.inst].off[" +
                                  std::to_string(EXA_OFF_X) + "] + T.start, T.count); break;";
    // every unit's tiles share a kernel's register budget: ask for at least
    // four waves per SIMD, so that one wave of the launch fits on the chip at
    // once.  The Jacobian + Hessian units need the most registers, so they
    // get a kernel of their own: exa_k_multi runs the Jacobian and the
    // Hessian as separate tiles and asks for five waves (its latency-bound
    // pulls and gathers gain more from the fifth wave than the few values
    // it then keeps in scratch cost), exa_k_multijh runs them as JH units.
    for (bool jh : {false, true}) {
        int lds = 0;
        std::vector<std::string> cases;
        for (int mode : multi_modes(jh)) {
            lds = std::max(lds, mode_lds_doubles(M, mode));
            mode_cases(mode, cases);
        }
        cases.push_back(zero_case);
        multi_kernel(jh ? "exa_k_multijh" : "exa_k_multi", lds, cases, jh ? 4 : 5);
    }
    {
        int lds = mode_lds_doubles(M, M_OBJ);
        std::vector<std::string> cases;
        for (int mode : {M_SFULL, M_SIPM}) {
            lds = std::max(lds, mode_lds_doubles(M, mode));
            std::map<int, Unit> all;
            for (int fused = 0; fused < 2; ++fused)
                for (auto& u : units_for(M, mode, fused != 0)) all[u.code] = u;
            for (auto& kv : all) {
                UnitLive L;
                os << unit_tile(M, mode, kv.second, ntmp, L);
                if (live) (*live)[{mode, kv.first}] = L;
                cases.push_back("case " + std::to_string((mode << EXA_MODE_SHIFT) | kv.first) + ": unit_" +
                                mode_name(mode) + "_" + std::to_string(kv.first) + "(C, C.c[" + std::to_string(M_JAC) +
                                "].inst[T.inst], T, lds); break;");
            }
        }
        // the objective's and J^T w's tiles
        mode_cases(M_OBJ, cases);
        mode_cases(M_JTPROD, cases);
        lds = std::max(lds, mode_lds_doubles(M, M_JTPROD));
        cases.push_back(zero_case);
        multi_kernel("exa_k_onepass", lds, cases, 0);
    }
    return os.str();
}

}  // namespace exa
