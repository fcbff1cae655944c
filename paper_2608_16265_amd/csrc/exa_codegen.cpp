// Lowering of pattern trees to straight-line gfx950 code (Sec. 6.2, Sec. 7.2.1).
//
// For every callback ("mode") one kernel is generated.  A workgroup takes one
// tile (pattern, first data point, count) from a tile list; each lane runs the
// whole evaluation of one data point at a time: coalesced struct-of-arrays
// loads, gathers of x, the forward sweep, and depending on the mode a reverse
// sweep (gradient, Jacobian rows), a forward tangent (J v), or
// forward-over-reverse (Hessian columns, H v, parameter adjoint).  All sweeps
// are emitted as scalar code with structural zeros and ones removed, so only
// the work a pattern really needs survives (Sec. 7.2.2 affine nodes).  Results
// of a lane go to its own disjoint slice (Sec. 5.3.2); multi-entry slices are
// staged through LDS so that the workgroup writes them with contiguous stores.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <sstream>

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

// Emits SSA statements and folds the literals 0, 1, -1.
struct Em {
    std::ostringstream& os;
    int& ntmp;
    std::string ind;
    Em(std::ostringstream& o, int& n, std::string i) : os(o), ntmp(n), ind(std::move(i)) {}

    std::string def(const std::string& e) {
        std::string n = "t" + std::to_string(ntmp++);
        os << ind << "const double " << n << " = " << e << ";\n";
        return n;
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
};

struct Sweep {
    // per-node symbolic quantities
    std::vector<std::string> val, d1, d2;       // unary: F', F''; binary: dA, dB
    std::vector<std::string> daa, dab, dbb;     // binary second partials
};

enum SeedKind { SEED_NONE, SEED_DIR, SEED_VEC };

class PatternCg {
  public:
    PatternCg(const Pattern& P, int mode) : P_(P), mode_(mode), t_(P.nodes) {
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

    // Body evaluated for one data point; defines the outputs named o0..o{n-1}
    // (or "res" for value modes).  Variables in scope: k, P, I, C, X, V, Y, TH.
    std::string body(int& ntmp) {
        std::ostringstream os;
        Em e(os, ntmp, "            ");
        loads(e);
        const bool second = mode_ == M_HESS || mode_ == M_HPROD || mode_ == M_ADJ;
        const bool first = mode_ != M_OBJ && mode_ != M_CONS;
        forward(e, first, second);
        const int root = (int)t_.size() - 1;
        switch (mode_) {
            case M_OBJ:
            case M_CONS:
                os << e.ind << "res = " << S_.val[root] << ";\n";
                break;
            case M_GRAD:
            case M_JAC:
            case M_JTPROD: {
                std::string seed = mode_ == M_JTPROD ? "wgt" : ONE;
                std::vector<std::string> J(P_.o1step(), Z), Pacc;
                std::vector<std::string> adj;
                reverse(e, seed, adj, J, Pacc, false);
                for (int s = 0; s < P_.o1step(); ++s) os << e.ind << "o[" << s << "] = " << J[s] << ";\n";
                break;
            }
            case M_JPROD: {
                std::vector<std::string> tg;
                tangent(e, SEED_VEC, -1, tg);
                os << e.ind << "res = " << tg[root] << ";\n";
                break;
            }
            case M_HESS:
                hessian(e);
                break;
            case M_HPROD: {
                std::vector<std::string> J(P_.o1step(), Z), Pacc, adj;
                reverse(e, "wgt", adj, J, Pacc, false);
                std::vector<std::string> tg;
                tangent(e, SEED_VEC, -1, tg);
                std::vector<std::string> Hc(P_.o1step(), Z), Pt;
                reverse_tangent(e, adj, tg, Hc, Pt, false);
                for (int s = 0; s < P_.o1step(); ++s) os << e.ind << "o[" << s << "] = " << Hc[s] << ";\n";
                break;
            }
            case M_ADJ: {
                std::vector<std::string> J(P_.o1step(), Z), Pacc(P_.pstep(), Z), adj;
                reverse(e, "wgt", adj, J, Pacc, true);
                std::vector<std::string> tg;
                tangent(e, SEED_VEC, -1, tg);
                std::vector<std::string> Hc(P_.o1step(), Z), Pt(P_.pstep(), Z);
                reverse_tangent(e, adj, tg, Hc, Pt, true);
                for (int s = 0; s < P_.pstep(); ++s) os << e.ind << "o[" << s << "] = " << Pt[s] << ";\n";
                break;
            }
            default:
                break;
        }
        return os.str();
    }

    bool needs_weight() const { return mode_ == M_HESS || mode_ == M_HPROD || mode_ == M_ADJ || mode_ == M_JTPROD; }

  private:
    const Pattern& P_;
    int mode_;
    const std::vector<TNode>& t_;
    std::vector<char> hasvar_, haspar_;
    Sweep S_;

    bool rev_active(int i) const { return hasvar_[i] || (mode_ == M_ADJ && haspar_[i]); }

    // Index of reference slot s (variables 0.., parameters after them); the
    // offset comes from the instance's descriptor, not from the code.
    std::string idx_expr(const RefKey& r, int s) const {
        if (r.col < 0) return "P.roff[" + std::to_string(s) + "]";
        return "(ic" + std::to_string(r.col) + " + P.roff[" + std::to_string(s) + "])";
    }

    void loads(Em& e) {
        std::set<int> ic, fc;
        for (auto& r : P_.vslots) if (r.col >= 0) ic.insert(r.col);
        for (auto& r : P_.pslots) if (r.col >= 0) ic.insert(r.col);
        for (auto& q : t_) if (q.op == EXA_OP_DATA) fc.insert(q.col);
        const bool need_row = P_.kind != EXA_OBJ && needs_weight();
        if (need_row && P_.kind == EXA_AUG) ic.insert(P_.row_icol);
        for (int c : ic) e.os << e.ind << "const long long ic" << c << " = P.ic[" << c << "][k];\n";
        for (int c : fc) e.os << e.ind << "const double fc" << c << " = P.fc[" << c << "][k];\n";
        for (int s = 0; s < P_.o1step(); ++s) {
            e.os << e.ind << "const long long ix" << s << " = " << idx_expr(P_.vslots[s], s) << ";\n";
            e.os << e.ind << "const double x" << s << " = X[ix" << s << "];\n";
        }
        if (mode_ == M_JPROD || mode_ == M_HPROD || mode_ == M_ADJ)
            for (int s = 0; s < P_.o1step(); ++s)
                e.os << e.ind << "const double v" << s << " = V[ix" << s << "];\n";
        for (int s = 0; s < P_.pstep(); ++s)
            e.os << e.ind << "const double p" << s << " = TH[" << idx_expr(P_.pslots[s], P_.o1step() + s) << "];\n";
        if (needs_weight()) {
            if (P_.kind == EXA_OBJ) {
                e.os << e.ind << "const double wgt = C.sigma;\n";
            } else if (P_.kind == EXA_CON) {
                e.os << e.ind << "const double wgt = Y[P.o0 + k];\n";
            } else {
                e.os << e.ind << "const double wgt = Y[P.tgt0 + ic" << P_.row_icol << " + P.row_off];\n";
            }
        }
    }

    // Forward sweep: values, and local partials of active children.
    void forward(Em& e, bool first, bool second) {
        const size_t n = t_.size();
        S_.val.assign(n, Z);
        S_.d1.assign(n, Z);
        S_.d2.assign(n, Z);
        S_.daa.assign(n, Z);
        S_.dab.assign(n, Z);
        S_.dbb.assign(n, Z);
        for (size_t i = 0; i < n; ++i) {
            const TNode& q = t_[i];
            auto& v = S_.val[i];
            switch (q.op) {
                case EXA_OP_CONST: v = lit(q.val); continue;
                case EXA_OP_DATA: v = "fc" + std::to_string(q.col); continue;
                case EXA_OP_VAR: v = "x" + std::to_string(q.slot); continue;
                case EXA_OP_PARAM: v = "p" + std::to_string(q.slot); continue;
                default: break;
            }
            if (is_unary(q.op)) {
                unary(e, (int)i, first && rev_active(q.a), second && rev_active(q.a));
            } else {
                binary(e, (int)i, first, second);
            }
        }
    }

    void unary(Em& e, int i, bool f1, bool f2) {
        const TNode& q = t_[i];
        const std::string u = S_.val[q.a];
        std::string& v = S_.val[i];
        std::string& d = S_.d1[i];
        std::string& dd = S_.d2[i];
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
                if (f1) d = e.def("-sin(" + u + ")");
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

    void binary(Em& e, int i, bool first, bool second) {
        const TNode& q = t_[i];
        const std::string u = S_.val[q.a], w = S_.val[q.b];
        const bool ua = rev_active(q.a), wa = rev_active(q.b);
        const bool f1 = first && (ua || wa), f2 = second && (ua || wa);
        std::string& v = S_.val[i];
        std::string& dA = S_.d1[i];
        std::string& dB = S_.d2[i];
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
                if (f2 && ua && wa) S_.dab[i] = ONE;
                break;
            case EXA_OP_DIV: {
                v = e.def(u + " / " + w);
                if (f1 || f2) {
                    const std::string iw = e.def("1.0 / " + w);
                    dA = iw;
                    if (wa) dB = e.def("-(" + v + " * " + iw + ")");
                    if (f2 && ua && wa) S_.dab[i] = e.def("-(" + iw + " * " + iw + ")");
                    if (f2 && wa) S_.dbb[i] = e.def("2.0 * " + v + " * " + iw + " * " + iw);
                }
                break;
            }
            case EXA_OP_POW: {
                int n = 0;
                if (!wa && small_int(t_[q.b], n)) {
                    v = e.def("exa_powi(" + u + ", " + std::to_string(n) + ")");
                    if (f1 || f2) dA = e.def(std::to_string(n) + ".0 * exa_powi(" + u + ", " + std::to_string(n - 1) + ")");
                    if (f2) S_.daa[i] = (n - 1 == 0) ? Z
                        : e.def(std::to_string(n * (n - 1)) + ".0 * exa_powi(" + u + ", " + std::to_string(n - 2) + ")");
                } else if (!wa) {
                    v = e.def("pow(" + u + ", " + w + ")");
                    if (f1 || f2) dA = e.def(w + " * pow(" + u + ", " + w + " - 1.0)");
                    if (f2) S_.daa[i] = e.def(w + " * (" + w + " - 1.0) * pow(" + u + ", " + w + " - 2.0)");
                } else if (!ua) {
                    v = e.def("pow(" + u + ", " + w + ")");
                    if (f1 || f2) {
                        const std::string lu = e.def("log(" + u + ")");
                        dB = e.def(v + " * " + lu);
                        if (f2) S_.dbb[i] = e.def(dB + " * " + lu);
                    }
                } else {
                    v = e.def("pow(" + u + ", " + w + ")");
                    if (f1 || f2) {
                        const std::string lu = e.def("log(" + u + ")");
                        const std::string pm1 = e.def("pow(" + u + ", " + w + " - 1.0)");
                        dA = e.def(w + " * " + pm1);
                        dB = e.def(v + " * " + lu);
                        if (f2) {
                            S_.daa[i] = e.def(w + " * (" + w + " - 1.0) * pow(" + u + ", " + w + " - 2.0)");
                            S_.dab[i] = e.def(pm1 + " * (1.0 + " + w + " * " + lu + ")");
                            S_.dbb[i] = e.def(dB + " * " + lu);
                        }
                    }
                }
                break;
            }
            default:
                fail(EXA_EINVAL, "codegen: unknown binary operator");
        }
        if (!ua) { dA = Z; S_.daa[i] = Z; S_.dab[i] = Z; }
        if (!wa) { dB = Z; S_.dbb[i] = Z; S_.dab[i] = Z; }
    }

    // Reverse sweep: adjoint of every node from the root seed; var leaves
    // accumulate into J, param leaves (when with_par) into Pacc.
    void reverse(Em& e, const std::string& seed, std::vector<std::string>& adj,
                 std::vector<std::string>& J, std::vector<std::string>& Pacc, bool with_par) {
        const int n = (int)t_.size();
        adj.assign(n, Z);
        adj[n - 1] = seed;
        for (int i = n - 1; i >= 0; --i) {
            const TNode& q = t_[i];
            const std::string& a = adj[i];
            if (q.op == EXA_OP_VAR) { J[q.slot] = e.add(J[q.slot], a); continue; }
            if (q.op == EXA_OP_PARAM) { if (with_par) Pacc[q.slot] = e.add(Pacc[q.slot], a); continue; }
            if (q.a < 0 || a == Z) continue;
            if (is_unary(q.op)) {
                if (rev_active(q.a)) adj[q.a] = e.mul(a, S_.d1[i]);
            } else {
                if (rev_active(q.a)) adj[q.a] = e.mul(a, S_.d1[i]);
                if (rev_active(q.b)) adj[q.b] = e.mul(a, S_.d2[i]);
            }
        }
    }

    // Forward tangent: SEED_DIR seeds 1 on var slot `dir`; SEED_VEC seeds v_s.
    void tangent(Em& e, SeedKind kind, int dir, std::vector<std::string>& tg) {
        const int n = (int)t_.size();
        tg.assign(n, Z);
        for (int i = 0; i < n; ++i) {
            const TNode& q = t_[i];
            if (q.op == EXA_OP_VAR) {
                tg[i] = kind == SEED_DIR ? (q.slot == dir ? ONE : Z) : "v" + std::to_string(q.slot);
                continue;
            }
            if (q.a < 0) continue;
            if (is_unary(q.op)) {
                tg[i] = e.mul(S_.d1[i], tg[q.a]);
            } else {
                tg[i] = e.add(e.mul(S_.d1[i], tg[q.a]), e.mul(S_.d2[i], tg[q.b]));
            }
        }
    }

    // Reverse sweep of the tangent (forward-over-reverse): the tangent of every
    // adjoint; var leaves accumulate into Hc, param leaves into Pt.
    void reverse_tangent(Em& e, const std::vector<std::string>& adj, const std::vector<std::string>& tg,
                         std::vector<std::string>& Hc, std::vector<std::string>& Pt, bool with_par) {
        const int n = (int)t_.size();
        std::vector<std::string> ta(n, Z);
        for (int i = n - 1; i >= 0; --i) {
            const TNode& q = t_[i];
            if (q.op == EXA_OP_VAR) { Hc[q.slot] = e.add(Hc[q.slot], ta[i]); continue; }
            if (q.op == EXA_OP_PARAM) { if (with_par) Pt[q.slot] = e.add(Pt[q.slot], ta[i]); continue; }
            if (q.a < 0) continue;
            if (is_unary(q.op)) {
                if (!rev_active(q.a)) continue;
                const std::string td = e.mul(S_.d2[i], tg[q.a]);
                ta[q.a] = e.add(e.mul(ta[i], S_.d1[i]), e.mul(adj[i], td));
            } else {
                const std::string tdA = e.add(e.mul(S_.daa[i], tg[q.a]), e.mul(S_.dab[i], tg[q.b]));
                const std::string tdB = e.add(e.mul(S_.dab[i], tg[q.a]), e.mul(S_.dbb[i], tg[q.b]));
                if (rev_active(q.a)) ta[q.a] = e.add(e.mul(ta[i], S_.d1[i]), e.mul(adj[i], tdA));
                if (rev_active(q.b)) ta[q.b] = e.add(e.mul(ta[i], S_.d2[i]), e.mul(adj[i], tdB));
            }
        }
    }

    // Smallest set of tangent directions that covers every Hessian slot: each
    // diagonal slot needs its own variable, each off-diagonal one either end.
    std::vector<int> directions() const {
        const int k = P_.o1step();
        std::vector<int> best;
        int best_n = k + 1;
        if (k > 20) {  // fall back to every variable
            for (int s = 0; s < k; ++s) best.push_back(s);
            return best;
        }
        for (unsigned mask = 0; mask < (1u << k); ++mask) {
            int cnt = __builtin_popcount(mask);
            if (cnt >= best_n) continue;
            bool ok = true;
            for (auto& h : P_.hslots)
                if (!((mask >> h.first) & 1u) && !((mask >> h.second) & 1u)) { ok = false; break; }
            if (!ok) continue;
            best_n = cnt;
            best.clear();
            for (int s = 0; s < k; ++s) if ((mask >> s) & 1u) best.push_back(s);
        }
        return best;
    }

    void hessian(Em& e) {
        std::vector<std::string> J(P_.o1step(), Z), Pacc, adj;
        reverse(e, "wgt", adj, J, Pacc, false);
        const std::vector<int> D = directions();
        std::map<int, std::vector<std::string>> col;  // direction -> column
        for (int d : D) {
            std::vector<std::string> tg, Hc(P_.o1step(), Z), Pt;
            tangent(e, SEED_DIR, d, tg);
            reverse_tangent(e, adj, tg, Hc, Pt, false);
            col[d] = Hc;
        }
        for (int s = 0; s < P_.o2step(); ++s) {
            const int a = P_.hslots[s].first, b = P_.hslots[s].second;
            std::string h = col.count(b) ? col[b][a] : col[a][b];
            const RefKey& ra = P_.vslots[a];
            const RefKey& rb = P_.vslots[b];
            // different slots over the same index column (or both literal)
            // have different offsets, so only different columns can alias
            const bool may_alias = a != b && ra.col != rb.col;
            if (may_alias && h != Z)
                e.os << e.ind << "o[" << s << "] = (ix" << a << " == ix" << b << ") ? 2.0 * " << h << " : " << h << ";\n";
            else
                e.os << e.ind << "o[" << s << "] = " << h << ";\n";
        }
    }
};

int out_step(const Pattern& P, int mode) {
    switch (mode) {
        case M_GRAD: case M_JAC: case M_JTPROD: case M_HPROD: return P.o1step();
        case M_HESS: return P.o2step();
        case M_ADJ: return P.pstep();
        default: return 1;
    }
}

const char* mode_name(int m) {
    static const char* n[] = {"obj", "cons", "grad", "jac", "hess", "jprod", "jtprod", "hprod", "adj"};
    return n[m];
}

}  // namespace

bool pattern_in_mode(const Pattern& P, int mode) {
    if (P.ndata == 0) return false;
    switch (mode) {
        case M_OBJ: return P.kind == EXA_OBJ;
        case M_CONS: return P.kind != EXA_OBJ;
        case M_GRAD: return P.kind == EXA_OBJ && P.o1step() > 0;
        case M_JAC: return P.kind != EXA_OBJ && P.o1step() > 0;
        case M_HESS: return P.o2step() > 0;
        case M_JPROD: return P.kind != EXA_OBJ;
        case M_JTPROD: return P.kind != EXA_OBJ && P.o1step() > 0;
        case M_HPROD: return P.o2step() > 0;
        case M_ADJ: return P.pstep() > 0 && P.o1step() > 0;
        default: return false;
    }
}

// Staging through LDS is used while a workgroup's slice fits in this many
// doubles (64 KiB); wider patterns store their slices directly.
constexpr int kLdsCapDoubles = 8192;

bool staged(const Pattern& P, int mode, int block) {
    return out_step(P, mode) * block <= kLdsCapDoubles;
}

int mode_lds_doubles(const Model& M, int mode, int block) {
    int st = 1;
    for (auto& P : M.pats)
        if (pattern_in_mode(P, mode) && staged(P, mode, block)) st = std::max(st, out_step(P, mode));
    return st * block;
}

std::string kernel_name(int mode) { return std::string("exa_k_") + mode_name(mode); }

std::string generate_source(const Model& M, int block) {
    std::ostringstream os;
    os << "// generated: straight-line evaluation kernels for one pattern set\n";
    os << "#define EXA_BLOCK " << block << "\n";
    os << EXA_STR(EXA_DEVICE_STRUCTS) << "\n";
    os << "static_assert(sizeof(ExaPatDev) == " << sizeof(ExaPatDev) << ", \"layout\");\n";
    os << "static_assert(sizeof(ExaInstDev) == " << sizeof(ExaInstDev) << ", \"layout\");\n";
    os << "static_assert(sizeof(ExaTile) == " << sizeof(ExaTile) << ", \"layout\");\n";
    os << "static_assert(sizeof(ExaCall) == " << sizeof(ExaCall) << ", \"layout\");\n";
    os << R"(
__device__ __forceinline__ double exa_powi(double u, int n) {
    double r = 1.0, b = u;
    unsigned m = n < 0 ? (unsigned)(-n) : (unsigned)n;
    while (m) { if (m & 1u) r *= b; b *= b; m >>= 1; }
    return n < 0 ? 1.0 / r : r;
}
// Writes the per-lane slices of `npts` consecutive data points (ST doubles
// each) to dst through LDS, so that the workgroup stores contiguous memory.
template <int ST>
__device__ __forceinline__ void exa_store(double* __restrict__ dst, const double* o, int npts, double* lds) {
    if (ST == 1) {
        if ((int)threadIdx.x < npts) dst[threadIdx.x] = o[0];
        return;
    }
#pragma unroll
    for (int s = 0; s < ST; ++s) lds[threadIdx.x * ST + s] = o[s];
    __syncthreads();
    const int n = npts * ST;
    for (int i = threadIdx.x; i < n; i += EXA_BLOCK) dst[i] = lds[i];
    __syncthreads();
}
// Direct (unstaged) variant for slices too wide for LDS.
template <int ST>
__device__ __forceinline__ void exa_store_direct(double* __restrict__ dst, const double* o, int npts, double*) {
    if ((int)threadIdx.x < npts) {
#pragma unroll
        for (int s = 0; s < ST; ++s) dst[threadIdx.x * ST + s] = o[s];
    }
}
// Sum over the workgroup in a fixed order (tree in LDS); result in lane 0.
__device__ __forceinline__ double exa_block_sum(double v, double* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = EXA_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}
)";
    int ntmp = 0;
    for (int mode = 0; mode < M_COUNT; ++mode) {
        std::vector<int> members;
        for (size_t p = 0; p < M.pats.size(); ++p)
            if (pattern_in_mode(M.pats[p], mode)) members.push_back((int)p);
        // tile functions
        for (int p : members) {
            const Pattern& P = M.pats[p];
            PatternCg cg(P, mode);
            const int st = out_step(P, mode);
            os << "__device__ __forceinline__ void tile_" << mode_name(mode) << "_" << p
               << "(const ExaCall& C, const ExaInstDev& I, const ExaTile& T, double* lds) {\n";
            os << "    const ExaPatDev& P = I.pat[" << p << "];\n";
            os << "    const double* __restrict__ X = C.x + I.off[" << EXA_OFF_X << "];\n";
            os << "    const double* __restrict__ V = C.v + I.off[" << EXA_OFF_X << "];\n";
            os << "    const double* __restrict__ Y = C.y + I.off[" << EXA_OFF_Y << "];\n";
            os << "    const double* __restrict__ TH = I.theta;\n";
            os << "    (void)X; (void)V; (void)Y; (void)TH;\n";
            os << "    const long long kend = T.start + T.count;\n";
            if (mode == M_OBJ) os << "    double acc = 0.0;\n";
            os << "    for (long long kb = T.start; kb < kend; kb += EXA_BLOCK) {\n";
            os << "        const long long k = kb + threadIdx.x;\n";
            os << "        const int npts = (int)((kend - kb) < EXA_BLOCK ? (kend - kb) : EXA_BLOCK);\n";
            const bool scalar_out = mode == M_OBJ || mode == M_CONS || mode == M_JPROD;
            const std::string store = staged(P, mode, block) ? "exa_store<" : "exa_store_direct<";
            if (scalar_out) os << "        double res = 0.0;\n";
            else os << "        double o[" << st << "];\n";
            os << "        if (k < kend) {\n";
            os << cg.body(ntmp);
            os << "        } else {\n";
            if (!scalar_out) os << "            for (int s = 0; s < " << st << "; ++s) o[s] = 0.0;\n";
            os << "        }\n";
            switch (mode) {
                case M_OBJ:
                    os << "        acc += exa_block_sum(res, lds);\n";
                    break;
                case M_CONS:
                case M_JPROD:
                    if (P.kind == EXA_CON)
                        os << "        if (k < kend) C.out0[I.off[" << EXA_OFF_ROWS << "] + P.o0 + k] = res;\n";
                    else
                        os << "        if (k < kend) C.out1[I.off[" << EXA_OFF_AUG << "] + P.o0 + k] = res;\n";
                    break;
                case M_GRAD:
                    os << "        " << store << st << ">(C.out0 + I.off[" << EXA_OFF_FO_OBJ << "] + P.o1 + kb * " << st << ", o, npts, lds);\n";
                    break;
                case M_JAC:
                    os << "        " << store << st << ">(C.out0 + I.off[" << EXA_OFF_JAC << "] + P.o1 + kb * " << st << ", o, npts, lds);\n";
                    break;
                case M_JTPROD:
                    os << "        " << store << st << ">(C.out0 + I.off[" << EXA_OFF_FO_CON << "] + P.o1 + kb * " << st << ", o, npts, lds);\n";
                    break;
                case M_HPROD:
                    os << "        " << store << st << ">(C.out0 + I.off[" << (P.kind == EXA_OBJ ? EXA_OFF_FO_OBJ : EXA_OFF_FO_CON)
                       << "] + P.o1 + kb * " << st << ", o, npts, lds);\n";
                    break;
                case M_HESS:
                    os << "        " << store << st << ">(C.out0 + I.off[" << EXA_OFF_HESS << "] + P.o2 + kb * " << st << ", o, npts, lds);\n";
                    break;
                case M_ADJ:
                    os << "        " << store << st << ">(C.out0 + I.off[" << EXA_OFF_PAR << "] + P.op + kb * " << st << ", o, npts, lds);\n";
                    break;
            }
            os << "    }\n";
            if (mode == M_OBJ)
                os << "    if (threadIdx.x == 0) C.out0[I.off[" << EXA_OFF_TILE << "] + T.slot] = acc;\n";
            os << "}\n";
        }
        // kernel
        const int lds = mode_lds_doubles(M, mode, block);
        os << "extern \"C\" __global__ void __launch_bounds__(EXA_BLOCK) " << kernel_name(mode)
           << "(ExaCall C) {\n";
        os << "    __shared__ double lds[" << lds << "];\n";
        os << "    (void)lds;\n";
        os << "    long long w = blockIdx.x;\n";
        os << "    for (;;) {\n";
        os << "        long long t;\n";
        os << "        if (C.persistent) {\n";
        os << "            if (w >= C.ntiles) return;\n";
        os << "            t = w;\n";
        os << "        } else {\n";
        os << "            // workgroup w runs on XCD w % 8: give each XCD a contiguous tile range\n";
        os << "            t = (w % 8) * C.per_xcd + w / 8;\n";
        os << "            if (t >= C.ntiles) return;\n";
        os << "        }\n";
        os << "        const ExaTile T = C.tiles[t];\n";
        os << "        const ExaInstDev& I = C.inst[T.inst];\n";
        os << "        switch (T.pat) {\n";
        for (int p : members)
            os << "            case " << p << ": tile_" << mode_name(mode) << "_" << p << "(C, I, T, lds); break;\n";
        os << "            default: break;\n";
        os << "        }\n";
        os << "        if (!C.persistent) return;\n";
        os << "        w += gridDim.x;\n";
        os << "    }\n";
        os << "}\n";
    }
    // Jacobian and Hessian values in one launch (batched evaluation): tile
    // pat < 32 is a Jacobian tile of pattern pat, pat >= 32 a Hessian tile of
    // pattern pat - 32; Jacobian values go to out0, Hessian values to out1.
    {
        const int lds = std::max(mode_lds_doubles(M, M_JAC, block), mode_lds_doubles(M, M_HESS, block));
        os << "extern \"C\" __global__ void __launch_bounds__(EXA_BLOCK) exa_k_jh(ExaCall C) {\n";
        os << "    __shared__ double lds[" << lds << "];\n";
        os << "    (void)lds;\n";
        os << "    ExaCall H = C;\n";
        os << "    H.out0 = C.out1;\n";
        os << "    for (long long w = blockIdx.x; w < C.ntiles; w += gridDim.x) {\n";
        os << "        const ExaTile T = C.tiles[w];\n";
        os << "        const ExaInstDev& I = C.inst[T.inst];\n";
        os << "        switch (T.pat) {\n";
        for (size_t p = 0; p < M.pats.size(); ++p) {
            if (pattern_in_mode(M.pats[p], M_JAC))
                os << "            case " << p << ": tile_jac_" << p << "(C, I, T, lds); break;\n";
            if (pattern_in_mode(M.pats[p], M_HESS))
                os << "            case " << (p + EXA_MAX_PATTERNS) << ": tile_hess_" << p << "(H, I, T, lds); break;\n";
        }
        os << "            default: break;\n";
        os << "        }\n";
        os << "    }\n";
        os << "}\n";
    }
    return os.str();
}

}  // namespace exa
