// Model build on the host: validation, build-time simplification (Sec. 7.1.2),
// sparsity structure by the probe rule of Sec. 5.2, output offsets and strides
// (Sec. 3.4, Sec. 5.3.2) and the sorted reduction maps (Sec. 7.2.3).
#include <set>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <sstream>

#include "exa_internal.h"

namespace exa {

namespace {

bool is_unary(int op) { return op >= EXA_OP_NEG && op <= EXA_OP_EXPM1; }
bool is_binary(int op) { return op >= EXA_OP_ADD && op <= EXA_OP_POW; }
bool is_leaf(int op) { return op >= EXA_OP_CONST && op <= EXA_OP_PARAM; }

struct Builder {
    std::vector<TNode> out;
    const exa_pattern_desc& d;
    explicit Builder(const exa_pattern_desc& dd) : d(dd) {}

    int push(TNode n) {
        out.push_back(n);
        return (int)out.size() - 1;
    }
    int cnst(double v) {
        TNode n;
        n.op = EXA_OP_CONST;
        n.val = v;
        return push(n);
    }
    bool is_c(int i, double v) const { return out[i].op == EXA_OP_CONST && out[i].val == v; }

    // Rebuild the subtree rooted at description node i, simplified bottom-up.
    // Identities (Sec. 7.1.2): x+0, 0+x -> x; x*1, 1*x -> x; x/1 -> x;
    // x^0 -> 1; x^1 -> x; x^2 -> abs2(x); x^-1 -> inv(x); 0*x, x*0 -> 0;
    // 0/x -> 0.  Only literal constants trigger a rule; nothing is folded.
    int rebuild(int i) {
        const int op = d.op[i];
        if (is_leaf(op)) {
            TNode n;
            n.op = op;
            if (op == EXA_OP_CONST) n.val = d.val[i];
            if (op == EXA_OP_DATA) n.col = d.a[i];
            if (op == EXA_OP_VAR || op == EXA_OP_PARAM) {
                n.col = d.a[i];
                n.off = d.off[i];
            }
            return push(n);
        }
        if (is_unary(op)) {
            int a = rebuild(d.a[i]);
            TNode n;
            n.op = op;
            n.a = a;
            return push(n);
        }
        int a = rebuild(d.a[i]);
        int b = rebuild(d.b[i]);
        switch (op) {
            case EXA_OP_ADD:
                if (is_c(b, 0.0)) return a;
                if (is_c(a, 0.0)) return b;
                break;
            case EXA_OP_MUL:
                if (is_c(a, 0.0) || is_c(b, 0.0)) return cnst(0.0);
                if (is_c(b, 1.0)) return a;
                if (is_c(a, 1.0)) return b;
                break;
            case EXA_OP_DIV:
                if (is_c(a, 0.0)) return cnst(0.0);
                if (is_c(b, 1.0)) return a;
                break;
            case EXA_OP_POW:
                if (out[b].op == EXA_OP_CONST) {
                    const double e = out[b].val;
                    if (e == 0.0) return cnst(1.0);
                    if (e == 1.0) return a;
                    if (e == 2.0 || e == -1.0) {
                        TNode n;
                        n.op = e == 2.0 ? EXA_OP_ABS2 : EXA_OP_INV;
                        n.a = a;
                        return push(n);
                    }
                }
                break;
            default:
                break;
        }
        TNode n;
        n.op = op;
        n.a = a;
        n.b = b;
        return push(n);
    }
};

// Compact a node list so that only nodes reachable from `root` remain, in
// post-order (orphans appear when a rule returns a child).
std::vector<TNode> compact(const std::vector<TNode>& in, int root) {
    std::vector<TNode> out;
    std::function<int(int)> rec = [&](int i) -> int {
        TNode n = in[i];
        if (n.a >= 0) n.a = rec(in[i].a);
        if (n.b >= 0) n.b = rec(in[i].b);
        out.push_back(n);
        return (int)out.size() - 1;
    };
    rec(root);
    return out;
}

// ---- structure (Sec. 5.2) -------------------------------------------------
struct Analysis {
    const std::vector<TNode>& t;
    std::vector<char> hv;                 // subtree contains a VAR
    std::vector<std::vector<int>> leaves; // VAR leaves (node ids), DFS order
    explicit Analysis(const std::vector<TNode>& tt) : t(tt), hv(tt.size(), 0), leaves(tt.size()) {
        for (size_t i = 0; i < t.size(); ++i) {  // post-order: children first
            const TNode& n = t[i];
            if (n.op == EXA_OP_VAR) {
                hv[i] = 1;
                leaves[i].push_back((int)i);
            }
            if (n.a >= 0) {
                hv[i] |= hv[n.a];
                leaves[i].insert(leaves[i].end(), leaves[n.a].begin(), leaves[n.a].end());
            }
            if (n.b >= 0) {
                hv[i] |= hv[n.b];
                leaves[i].insert(leaves[i].end(), leaves[n.b].begin(), leaves[n.b].end());
            }
        }
    }
};

// d2F/du2 of a unary operator identically zero?
bool unary_affine(int op) { return op == EXA_OP_NEG; }

// Binary with both sides carrying variables: nonzero F11, F12, F22.
void binary_curv(int op, bool& f11, bool& f12, bool& f22) {
    f11 = f12 = f22 = false;
    switch (op) {
        case EXA_OP_MUL: f12 = true; break;
        case EXA_OP_DIV: f12 = f22 = true; break;
        case EXA_OP_POW: f11 = f12 = f22 = true; break;
        default: break;  // ADD, SUB: affine
    }
}

// Binary with one variable-free side, as a map of the other side: affine?
// (Sec. 7.2.2, FirstFixed / SecondFixed.)
bool one_sided_affine(int op, bool var_left) {
    if (op == EXA_OP_ADD || op == EXA_OP_SUB || op == EXA_OP_MUL) return true;
    if (op == EXA_OP_DIV) return var_left;  // u/c yes, c/u no
    return false;                           // u^c, c^u
}

int find_or_add(std::vector<RefKey>& v, RefKey k) {
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i] == k) return (int)i;
    v.push_back(k);
    return (int)v.size() - 1;
}

void analyse_structure(Pattern& P) {
    const auto& t = P.nodes;
    const int root = (int)t.size() - 1;
    // first-order visits: left-to-right depth-first walk (Sec. 5.2.1)
    std::function<void(int)> fo = [&](int i) {
        const TNode& n = t[i];
        if (n.op == EXA_OP_VAR) {
            P.nodes[i].slot = find_or_add(P.vslots, RefKey{n.col, n.off});
            return;
        }
        if (n.op == EXA_OP_PARAM) {
            P.nodes[i].slot = find_or_add(P.pslots, RefKey{n.col, n.off});
            return;
        }
        if (n.a >= 0) fo(n.a);
        if (n.b >= 0) fo(n.b);
    };
    fo(root);

    // second-order emission: a second adjoint is structurally zero until an
    // ancestor with curvature is met (Sec. 5.1.3, Sec. 7.2.2).
    Analysis A(t);
    std::vector<std::pair<int, int>>& H = P.hslots;
    auto emit = [&](int sa, int sb) {
        const int lo = std::min(sa, sb), hi = std::max(sa, sb);
        for (auto& p : H)
            if (std::min(p.first, p.second) == lo && std::max(p.first, p.second) == hi) return;
        H.emplace_back(sa, sb);
    };
    std::function<void(int, bool)> rec = [&](int i, bool nl) {
        const TNode& n = t[i];
        if (n.op == EXA_OP_VAR) {
            if (nl) emit(n.slot, n.slot);
            return;
        }
        if (is_leaf(n.op)) return;
        if (is_unary(n.op)) {
            rec(n.a, nl || !unary_affine(n.op));
            return;
        }
        const bool hu = A.hv[n.a], hw = A.hv[n.b];
        if (hu && hw) {
            bool f11, f12, f22;
            binary_curv(n.op, f11, f12, f22);
            rec(n.a, nl || f11);
            rec(n.b, nl || f22);
            if (nl || f12)
                for (int lu : A.leaves[n.a])
                    for (int lw : A.leaves[n.b]) emit(t[lu].slot, t[lw].slot);
        } else if (hu) {
            rec(n.a, nl || !one_sided_affine(n.op, true));
        } else if (hw) {
            rec(n.b, nl || !one_sided_affine(n.op, false));
        }
    };
    rec(root, false);
}

void validate_desc(const exa_pattern_desc& d, int p, int npats, const exa_pattern_desc* all) {
    auto bad = [&](const std::string& m) {
        fail(EXA_EINVAL, "pattern " + std::to_string(p) + ": " + m);
    };
    if (d.kind != EXA_OBJ && d.kind != EXA_CON && d.kind != EXA_AUG) bad("unknown kind");
    if (d.nnodes < 1 || d.nnodes > EXA_MAX_NODES) bad("node count out of range");
    if (!d.op || !d.a || !d.b) bad("missing node arrays");
    if (d.ndata < 0) bad("negative ndata");
    if (d.n_icols < 0 || d.n_icols > EXA_MAX_COLS || d.n_fcols < 0 || d.n_fcols > EXA_MAX_COLS)
        bad("too many data columns");
    if (d.ndata > 0) {
        for (int c = 0; c < d.n_icols; ++c)
            if (!d.icols || !d.icols[c]) bad("missing integer column");
        for (int c = 0; c < d.n_fcols; ++c)
            if (!d.fcols || !d.fcols[c]) bad("missing float column");
    }
    for (int i = 0; i < d.nnodes; ++i) {
        const int op = d.op[i];
        if (is_leaf(op)) {
            if (op == EXA_OP_DATA && (d.a[i] < 0 || d.a[i] >= d.n_fcols))
                bad("data node " + std::to_string(i) + " names a missing float column");
            if ((op == EXA_OP_VAR || op == EXA_OP_PARAM) && (d.a[i] < -1 || d.a[i] >= d.n_icols))
                bad("index node " + std::to_string(i) + " names a missing integer column");
            if ((op == EXA_OP_VAR || op == EXA_OP_PARAM) && !d.off) bad("missing offsets");
            if (op == EXA_OP_CONST && !d.val) bad("missing literals");
        } else if (is_unary(op)) {
            if (d.a[i] < 0 || d.a[i] >= i) bad("child of node " + std::to_string(i) + " is not below it");
        } else if (is_binary(op)) {
            if (d.a[i] < 0 || d.a[i] >= i || d.b[i] < 0 || d.b[i] >= i)
                bad("child of node " + std::to_string(i) + " is not below it");
        } else {
            bad("unknown operator " + std::to_string(op) + " at node " + std::to_string(i));
        }
    }
    if (d.kind == EXA_AUG) {
        if (d.target < 0 || d.target >= p || all[d.target].kind != EXA_CON)
            bad("augmentation target must be an earlier constraint pattern");
        if (d.row_icol < 0 || d.row_icol >= d.n_icols) bad("augmentation row column missing");
    }
    (void)npats;
}

void build_map(SegMap& M, int64_t nseg, const std::vector<std::pair<int64_t, int64_t>>& tp) {
    // tp: (target segment, buffer position) in summation order; a segment
    // keeps its entries in that order
    M.ptr.assign(nseg + 1, 0);
    for (auto& e : tp) M.ptr[e.first + 1]++;
    for (int64_t s = 0; s < nseg; ++s) M.ptr[s + 1] += M.ptr[s];
    M.idx.assign(tp.size(), 0);
    std::vector<int64_t> fill(M.ptr.begin(), M.ptr.end() - 1);
    for (auto& e : tp) M.idx[fill[e.first]++] = e.second;
}

}  // namespace

void build_host(Model& M, const exa_pattern_desc* pats, int32_t npats) {
    if (npats < 0 || npats > EXA_MAX_PATTERNS)
        fail(EXA_EINVAL, "pattern count must be in 0.." + std::to_string(EXA_MAX_PATTERNS));
    if (npats > 0 && !pats) fail(EXA_EINVAL, "null pattern array");
    for (int p = 0; p < npats; ++p) validate_desc(pats[p], p, npats, pats);

    M.pats.resize(npats);
    for (int p = 0; p < npats; ++p) {
        const exa_pattern_desc& d = pats[p];
        Pattern& P = M.pats[p];
        P.kind = d.kind;
        P.index = p;
        P.ndata = d.ndata;
        P.n_icols = d.n_icols;
        P.n_fcols = d.n_fcols;
        Builder B(d);
        int root = B.rebuild(d.nnodes - 1);
        P.nodes = compact(B.out, root);
        P.icols.resize(d.n_icols);
        for (int c = 0; c < d.n_icols; ++c)
            P.icols[c].assign(d.icols ? d.icols[c] : nullptr,
                              d.icols ? d.icols[c] + d.ndata : nullptr);
        P.fcols_src.resize(d.n_fcols);
        for (int c = 0; c < d.n_fcols; ++c) P.fcols_src[c] = d.fcols ? d.fcols[c] : nullptr;
        P.target = d.target;
        P.row_icol = d.row_icol;
        P.row_off = d.row_off;
        if (d.kind == EXA_CON) {
            P.lcon.assign(d.ndata, 0.0);
            P.ucon.assign(d.ndata, 0.0);
            if (d.lcon) std::copy(d.lcon, d.lcon + d.ndata, P.lcon.begin());
            if (d.ucon) std::copy(d.ucon, d.ucon + d.ndata, P.ucon.begin());
        }
        analyse_structure(P);
        if (P.o1step() + P.pstep() > EXA_MAX_REFS)
            fail(EXA_EINVAL, "pattern " + std::to_string(p) + " has more than " +
                                 std::to_string(EXA_MAX_REFS) + " distinct variable/parameter references");
    }

    // ---- data-set groups ---------------------------------------------------
    for (int p = 0; p < npats; ++p) {
        const exa_pattern_desc& d = pats[p];
        int g = -1;
        for (size_t q = 0; q < M.groups.size() && g < 0; ++q) {
            const exa_pattern_desc& e = pats[M.groups[q].members[0]];
            bool same = d.ndata > 0 && e.ndata == d.ndata && e.n_icols == d.n_icols &&
                        e.n_fcols == d.n_fcols;
            for (int c = 0; same && c < d.n_icols; ++c) same = d.icols[c] == e.icols[c];
            for (int c = 0; same && c < d.n_fcols; ++c) same = d.fcols[c] == e.fcols[c];
            if (same) g = (int)q;
        }
        if (g < 0) {
            M.groups.emplace_back();
            g = (int)M.groups.size() - 1;
            M.groups[g].ndata = d.ndata;
        }
        Group& G = M.groups[g];
        Pattern& P = M.pats[p];
        P.group = g;
        const int mi = (int)G.members.size();
        G.members.push_back(p);
        for (int s = 0; s < P.o1step(); ++s) {
            int r = find_or_add(G.vrefs, P.vslots[s]);
            if (r == (int)G.vsrc.size()) G.vsrc.emplace_back(mi, s);
            P.vg.push_back(r);
        }
        for (int s = 0; s < P.pstep(); ++s) {
            int r = find_or_add(G.prefs, P.pslots[s]);
            if (r == (int)G.psrc.size()) G.psrc.emplace_back(mi, s);
            P.pg.push_back(r);
        }
    }

    // ---- offsets in declaration order (Sec. 3.1 running counts) ----------
    int64_t ncon = 0, nnzj = 0, nnzh = 0, nnzg = 0, naug = 0, nnzp = 0, nobj = 0;
    for (auto& P : M.pats) {
        P.o2 = nnzh;
        nnzh += P.ndata * P.o2step();
        if (P.kind == EXA_OBJ) {
            P.o0 = nobj;
            nobj += P.ndata;
            P.o1 = nnzg;
            nnzg += P.ndata * P.o1step();
        } else {
            if (P.kind == EXA_CON) {
                P.o0 = ncon;
                ncon += P.ndata;
            } else {
                P.o0 = naug;
                naug += P.ndata;
                P.tgt0 = M.pats[P.target].o0;
            }
            P.o1 = nnzj;
            nnzj += P.ndata * P.o1step();
        }
        const int64_t bs = P.bstride();
        if (P.kind == EXA_OBJ) {
            P.ob = M.fo_obj_len;
            M.fo_obj_len += bs * P.o1step();
        }
        if (P.pstep() > 0 && P.o1step() > 0) {
            P.op = M.par_len;
            M.par_len += bs * P.pstep();
            nnzp += P.ndata * P.pstep();
        }
        for (int s = 0; s < P.o1step(); ++s) {
            bool curved = false;
            for (auto& h : P.hslots) curved |= h.first == s || h.second == s;
            if (curved) P.hvs.push_back(s);
        }
    }
    // J^T w and H v blocks per data-set group: the members' contributions to
    // one variable reference are summed in the lane (members in declaration
    // order), so a group writes one slot per reference instead of one per
    // member and slot
    for (Group& G : M.groups) {
        // an augmentation term that is +-(one variable) and the only J^T w
        // contribution of the group to that reference adds +-w[row] to it:
        // the reduction reads that weight itself
        std::map<int, int> users;  // reference -> members that contribute J^T w to it
        for (int p : G.members) {
            const Pattern& P = M.pats[p];
            if (P.ndata > 0 && P.kind != EXA_OBJ)
                for (int s = 0; s < P.o1step(); ++s) users[P.vg[s]]++;
        }
        for (int p : G.members) {
            Pattern& P = M.pats[p];
            P.wread = 0;
            if (P.kind != EXA_AUG || P.ndata == 0 || P.o1step() != 1 || P.pstep() != 0 || users[P.vg[0]] != 1) continue;
            const std::vector<TNode>& n = P.nodes;
            if (n.size() == 1 && n[0].op == EXA_OP_VAR)
                P.wread = 1;
            else if (n.size() == 2 && n[0].op == EXA_OP_VAR && n[1].op == EXA_OP_NEG && n[1].a == 0)
                P.wread = -1;
        }
        std::set<int> jr, hr;
        for (int p : G.members) {
            const Pattern& P = M.pats[p];
            if (P.ndata == 0) continue;
            if (P.kind != EXA_OBJ && !P.wread)
                for (int s = 0; s < P.o1step(); ++s) jr.insert(P.vg[s]);
            for (int s : P.hvs) hr.insert(P.vg[s]);
        }
        G.jt_refs.assign(jr.begin(), jr.end());
        G.hv_refs.assign(hr.begin(), hr.end());
        const int64_t bs = (G.ndata + 15) & ~(int64_t)15;
        G.ob = M.fo_con_len;
        M.fo_con_len += bs * (int64_t)G.jt_refs.size();
        G.oh = M.hv_len;
        M.hv_len += bs * (int64_t)G.hv_refs.size();
        M.nhv += G.ndata * (int64_t)G.hv_refs.size();
        for (int p : G.members) {
            Pattern& P = M.pats[p];
            if (P.kind != EXA_OBJ) P.ob = G.ob;
            P.oh = G.oh;
        }
    }
    // chunked sums' padding lanes read position 0 of the first-order buffer
    if (M.fo_obj_len + M.fo_con_len == 0) M.fo_con_len = 16;
    M.ncon = ncon;
    M.nnzj = nnzj;
    M.nnzh = nnzh;
    M.nnzg = nnzg;
    M.naug = naug;
    M.nnzp = nnzp;
    M.nobj = nobj;
    if (ncon >= INT32_MAX || M.nvar >= INT32_MAX)
        fail(EXA_EINVAL, "row or variable count exceeds the int32 COO index range");

    // ---- index validation at every data point -----------------------------
    for (auto& P : M.pats) {
        for (int s = 0; s < P.o1step(); ++s)
            for (int64_t k = 0; k < P.ndata; ++k) {
                int64_t g = P.var_index(s, k);
                if (g < 0 || g >= M.nvar)
                    fail(EXA_EINVAL, "pattern " + std::to_string(P.index) + ": variable index " +
                                         std::to_string(g) + " out of range at data point " +
                                         std::to_string(k));
            }
        for (int s = 0; s < P.pstep(); ++s)
            for (int64_t k = 0; k < P.ndata; ++k) {
                int64_t g = P.par_index(s, k);
                if (g < 0 || g >= M.ntheta)
                    fail(EXA_EINVAL, "pattern " + std::to_string(P.index) + ": parameter index " +
                                         std::to_string(g) + " out of range at data point " +
                                         std::to_string(k));
            }
        if (P.kind == EXA_AUG) {
            const int64_t nrows = M.pats[P.target].ndata;
            for (int64_t k = 0; k < P.ndata; ++k) {
                int64_t r = (int64_t)P.icols[P.row_icol][k] + P.row_off;
                if (r < 0 || r >= nrows)
                    fail(EXA_EINVAL, "pattern " + std::to_string(P.index) +
                                         ": augmentation row out of range at data point " +
                                         std::to_string(k));
            }
        }
    }

    // ---- augmentation rows: each base row pulls the terms that add to it
    for (auto& P : M.pats) {
        if (P.kind != EXA_AUG) continue;
        Pattern& T = M.pats[P.target];
        T.augs.push_back(P.index);
        P.rptr.assign(T.ndata + 1, 0);
        for (int64_t k = 0; k < P.ndata; ++k) P.rptr[(int64_t)P.icols[P.row_icol][k] + P.row_off + 1]++;
        for (int64_t r = 0; r < T.ndata; ++r) P.rptr[r + 1] += P.rptr[r];
        P.ridx.assign(P.ndata, 0);
        std::vector<int32_t> fill(P.rptr.begin(), P.rptr.end() - 1);
        for (int64_t k = 0; k < P.ndata; ++k) P.ridx[fill[(int64_t)P.icols[P.row_icol][k] + P.row_off]++] = (int32_t)k;
    }

    // ---- reduction maps (Sec. 7.2.3): sorted by target; within a target
    // the contributions are summed in (pattern, data point, slot) order, and
    // the J^T w and H v group entries in (group, data point, reference) order.
    // The work buffers hold each pattern's block slot-major: slot s of data
    // point k at block + s * bstride() + k (the constraint part of the
    // first-order buffer after the objective part).
    std::vector<std::pair<int64_t, int64_t>> g, jt, h, pr;
    auto gvar = [&](const Group& G, int r, int64_t k) {
        const RefKey& rk = G.vrefs[r];
        return rk.col < 0 ? rk.off : (int64_t)M.pats[G.members[0]].icols[rk.col][k] + rk.off;
    };
    // H v references whose every entry is the only H v contribution to its
    // variable (at most 32 per group): the kernel stores those entries into
    // the output directly, so they take no buffer round trip and no map
    // entry, and the reduction skips their variables
    std::vector<int32_t> hcount(M.nvar, 0);
    for (const Group& G : M.groups)
        for (int64_t k = 0; k < G.ndata; ++k)
            for (int r : G.hv_refs) hcount[gvar(G, r, k)]++;
    for (Group& G : M.groups) {
        G.hv_direct.assign(G.hv_refs.size(), 0);
        for (size_t j = 0; j < G.hv_refs.size() && j < 32; ++j) {
            bool alone = G.ndata > 0;
            for (int64_t k = 0; k < G.ndata && alone; ++k) alone = hcount[gvar(G, G.hv_refs[j], k)] == 1;
            G.hv_direct[j] = alone ? 1 : 0;
        }
    }
    std::vector<char> hskip(M.nvar, 0);
    for (const Group& G : M.groups) {
        const int64_t bs = (G.ndata + 15) & ~(int64_t)15;
        // weight entries (Pattern::wread) by reference: ~(2 row + negated)
        std::map<int, int> wr;
        for (int p : G.members)
            if (M.pats[p].wread) wr[M.pats[p].vg[0]] = p;
        std::vector<int> jall(G.jt_refs.begin(), G.jt_refs.end());
        for (auto& x : wr) jall.push_back(x.first);
        std::sort(jall.begin(), jall.end());
        // a variable sums its group entries in (group, data point, reference)
        // order
        for (int64_t k = 0; k < G.ndata; ++k) {
            for (int r : jall) {
                const auto w = wr.find(r);
                if (w != wr.end()) {
                    const Pattern& A = M.pats[w->second];
                    const int64_t row = A.tgt0 + (int64_t)A.icols[A.row_icol][k] + A.row_off;
                    jt.emplace_back(gvar(G, r, k), ~(2 * row + (A.wread < 0 ? 1 : 0)));
                    continue;
                }
                const int64_t j = std::find(G.jt_refs.begin(), G.jt_refs.end(), r) - G.jt_refs.begin();
                jt.emplace_back(gvar(G, r, k), M.fo_obj_len + G.ob + j * bs + k);
            }
            for (size_t j = 0; j < G.hv_refs.size(); ++j) {
                const int64_t v = gvar(G, G.hv_refs[j], k);
                if (G.hv_direct[j])
                    hskip[v] = 1;
                else
                    h.emplace_back(v, G.oh + (int64_t)j * bs + k);
            }
        }
    }
    for (auto& P : M.pats) {
        const int st = P.o1step();
        const int64_t bs = P.bstride();
        if (P.kind == EXA_OBJ)
            for (int64_t k = 0; k < P.ndata; ++k)
                for (int s = 0; s < st; ++s) g.emplace_back(P.var_index(s, k), P.ob + s * bs + k);
        if (P.pstep() > 0 && P.o1step() > 0)
            for (int64_t k = 0; k < P.ndata; ++k)
                for (int t = 0; t < P.pstep(); ++t)
                    pr.emplace_back(P.par_index(t, k), P.op + t * bs + k);
    }
    // every position lies inside its buffer (the kernels store to the same
    // positions: block + slot * bstride() + k, k < ndata)
    auto inside = [](const std::vector<std::pair<int64_t, int64_t>>& e, int64_t len, const char* what) {
        for (auto& x : e)
            if (x.second < 0 || x.second >= len) fail(EXA_EINVAL, std::string("internal: work-buffer position outside the ") + what);
    };
    inside(g, M.fo_obj_len, "objective part of the first-order buffer");
    for (auto& x : jt)  // weight entries name a constraint row
        if (x.second < 0 && (~x.second >> 1) >= M.ncon)
            fail(EXA_EINVAL, "internal: a J^T w weight entry outside the constraint rows");
    {
        std::vector<std::pair<int64_t, int64_t>> jb;
        for (auto& x : jt)
            if (x.second >= 0) jb.push_back(x);
        inside(jb, M.fo_obj_len + M.fo_con_len, "first-order buffer");
    }
    inside(h, M.hv_len, "H v buffer");
    inside(pr, M.par_len, "parameter buffer");
    for (auto& P : M.pats) {
        const int64_t bs = P.bstride();
        if ((P.kind == EXA_OBJ && P.ob + bs * P.o1step() > M.fo_obj_len) ||
            (P.pstep() > 0 && P.o1step() > 0 && P.op + bs * P.pstep() > M.par_len))
            fail(EXA_EINVAL, "internal: a pattern's work-buffer block ends past its buffer");
    }
    for (const Group& G : M.groups) {
        const int64_t bs = (G.ndata + 15) & ~(int64_t)15;
        if (G.ob + bs * (int64_t)G.jt_refs.size() > M.fo_con_len || G.oh + bs * (int64_t)G.hv_refs.size() > M.hv_len)
            fail(EXA_EINVAL, "internal: a group's work-buffer block ends past its buffer");
    }
    build_map(M.grad_map, M.nvar, g);
    M.grad_direct = true;
    for (int64_t v = 0; v < M.nvar; ++v)
        if (M.grad_map.ptr[v + 1] - M.grad_map.ptr[v] > 1) M.grad_direct = false;
    for (int64_t v = 0; v < M.nvar;) {
        if (M.grad_map.ptr[v + 1] > M.grad_map.ptr[v]) { ++v; continue; }
        int64_t e = v;
        while (e < M.nvar && M.grad_map.ptr[e + 1] == M.grad_map.ptr[e]) ++e;
        M.grad_zero.emplace_back(v, e - v);
        v = e;
    }
    build_map(M.jt_map, M.nvar, jt);
    build_map(M.h_map, M.nvar, h);
    if (std::find(hskip.begin(), hskip.end(), 1) != hskip.end()) M.h_map.skip = std::move(hskip);
    build_map(M.par_map, M.ntheta, pr);
    for (auto& P : M.pats) {
        P.ident.assign(P.n_icols, 0);
        if (P.ndata < kIdentMin) continue;
        for (int c = 0; c < P.n_icols; ++c) {
            bool id = true;
            for (int64_t k = 0; k < P.ndata && id; ++k) id = P.icols[c][k] == k;
            P.ident[c] = id ? 1 : 0;
        }
    }
    M.signature = pattern_signature(M);
}

bool same_walk(const Model& M, int a, int b) {
    if (a == b) return true;
    const Pattern& A = M.pats[a];
    const Pattern& B = M.pats[b];
    return A.kind == EXA_AUG && B.kind == EXA_AUG && A.group >= 0 && A.group == B.group &&
           A.row_icol == B.row_icol && A.row_off == B.row_off &&
           M.pats[A.target].ndata == M.pats[B.target].ndata;
}

std::string pattern_signature(const Model& M) {
    std::ostringstream os;
    os.precision(17);
    for (auto& P : M.pats) {
        os << "P" << P.kind << ":" << P.n_icols << "," << P.n_fcols << ":" << P.row_icol << ";";
        // the generated code has no unit for a pattern without data points
        // (of any kind), so instances that share code agree on which
        // patterns are empty
        os << (P.ndata > 0 ? "D;" : "E;");
        // reference offsets are per-instance data (ExaPatDev::roff): left out;
        // which references coincide inside a data-set group is kept
        for (auto& n : P.nodes)
            os << n.op << "," << n.a << "," << n.b << "," << n.col << "," << n.val << "," << n.slot
               << ";";
        os << "G" << P.group << ":";
        // which augmentation pulls share a walk is fixed by the code
        if (P.kind == EXA_AUG) {
            int w = -1;
            for (int q = 0; q < P.index && w < 0; ++q)
                if (same_walk(M, q, P.index)) w = q;
            os << "W" << w << ":";
        }
        for (int r : P.vg) os << r << ",";
        os << "|";
        for (int r : P.pg) os << r << ",";
        os << ";";
    }
    return os.str();
}

}  // namespace exa

// ---------------------------------------------------------------------------
// Host-side structure callbacks (Sec. 5.3.1).
using exa::Model;
using exa::Pattern;

namespace exa {
void jac_structure_host(const Model& M, int32_t* rows, int32_t* cols) {
    for (const Pattern& P : M.pats) {
        if (P.kind == EXA_OBJ) continue;
        const int st = P.o1step();
        for (int64_t k = 0; k < P.ndata; ++k) {
            const int64_t r = P.row(k);
            for (int s = 0; s < st; ++s) {
                rows[P.o1 + k * st + s] = (int32_t)r;
                cols[P.o1 + k * st + s] = (int32_t)P.var_index(s, k);
            }
        }
    }
}

void hess_structure_host(const Model& M, int32_t* rows, int32_t* cols) {
    for (const Pattern& P : M.pats) {
        const int st = P.o2step();
        for (int64_t k = 0; k < P.ndata; ++k)
            for (int s = 0; s < st; ++s) {
                const int64_t ga = P.var_index(P.hslots[s].first, k);
                const int64_t gb = P.var_index(P.hslots[s].second, k);
                rows[P.o2 + k * st + s] = (int32_t)std::max(ga, gb);
                cols[P.o2 + k * st + s] = (int32_t)std::min(ga, gb);
            }
    }
}
}  // namespace exa
