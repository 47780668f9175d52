// Index-notation front-end and leaf generator: statements of tensor index
// notation (Sec. II-A) over the library's level formats (Sec. II-B, III-B)
// are parsed, given a concordant loop order and lowered to HIP leaves in
// which each index variable is a coordinate-value loop or a co-iteration of
// the Compressed levels that index it (Sec. IV-C); sparse outputs are
// assembled in two phases (Sec. V-B).  See tin.hpp.
#include "tin.hpp"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cctype>
#include <cstdint>
#include <cstdio>
#include <set>
#include <sstream>

#include "internal.hpp"

namespace spl {
namespace tin {
namespace {

// ------------------------------------------------------------------ syntax

struct Access {
    std::string name;
    std::vector<int> vars;
    int op = -1;  // binding index (right side)
};

struct Term {
    int sign = 1;
    std::vector<Access> f;
};

// lhs = sum of signed terms, each a product of accesses
struct Stmt {
    Access lhs;
    std::vector<Term> terms;
    std::vector<std::string> vars;
};

class Parser {
  public:
    Parser(const char *s, Stmt &st, std::string &err) : p_(s), st_(st), err_(err) {}

    bool parse() {
        if (!access(st_.lhs)) return false;
        if (!eat('=')) return fail("expected '='");
        int sign = 1;
        if (eat('-'))
            sign = -1;
        else
            eat('+');
        for (;;) {
            Term t;
            t.sign = sign;
            if (!term(t)) return false;
            st_.terms.push_back(t);
            if (eat('+'))
                sign = 1;
            else if (eat('-'))
                sign = -1;
            else
                break;
        }
        ws();
        if (*p_) return fail(std::string("unexpected '") + *p_ + "'");
        return true;
    }

  private:
    const char *p_;
    Stmt &st_;
    std::string &err_;

    bool fail(const std::string &m) {
        err_ = m;
        return false;
    }
    void ws() {
        while (*p_ && std::isspace(static_cast<unsigned char>(*p_))) ++p_;
    }
    bool eat(char c) {
        ws();
        if (*p_ != c) return false;
        ++p_;
        return true;
    }
    bool ident(std::string &s) {
        ws();
        if (!(std::isalpha(static_cast<unsigned char>(*p_)) || *p_ == '_')) return false;
        const char *b = p_;
        while (std::isalnum(static_cast<unsigned char>(*p_)) || *p_ == '_') ++p_;
        s.assign(b, p_);
        return true;
    }
    int var(const std::string &n) {
        for (size_t k = 0; k < st_.vars.size(); ++k)
            if (st_.vars[k] == n) return static_cast<int>(k);
        st_.vars.push_back(n);
        return static_cast<int>(st_.vars.size()) - 1;
    }
    bool access(Access &a) {
        if (!ident(a.name)) return fail("expected a tensor name");
        if (eat('(') && !eat(')')) {
            do {
                std::string v;
                if (!ident(v)) return fail("expected an index variable");
                a.vars.push_back(var(v));
            } while (eat(','));
            if (!eat(')')) return fail("expected ')'");
        }
        return true;
    }
    bool term(Term &t) {
        do {
            Access a;
            if (!access(a)) return false;
            t.f.push_back(a);
        } while (eat('*'));
        return true;
    }
};

// ------------------------------------------------------------- operands

struct OpInfo {
    bool sparse = false;
    int order = 0;
    int level[3] = {0, 0, 0};
    int dtype = 0;
    int64_t dims[3] = {0, 0, 0};
};

bool op_info(const Binding &b, OpInfo &o, std::string &err) {
    if ((b.sparse != nullptr) == (b.dense != nullptr)) {
        err = "operand " + b.name + ": bind exactly one of a sparse and a dense tensor";
        return false;
    }
    if (b.sparse) {
        const spl_sparse *s = b.sparse;
        o.sparse = true;
        o.order = s->order;
        o.dtype = s->vtype;
        for (int l = 0; l < s->order && l < 3; ++l) {
            o.level[l] = s->level[l];
            o.dims[l] = s->dims[l];
        }
        if (s->order < 2 || s->order > 3 || s->level[0] != SPL_DENSE ||
            s->level[s->order - 1] != SPL_COMPRESSED) {
            err = "operand " + b.name + ": formats (Dense, Compressed), (Dense, Compressed, "
                  "Compressed) or (Dense, Dense, Compressed)";
            return false;
        }
        if (s->pos_type != SPL_I32) {
            err = "operand " + b.name + ": int32 positions only";
            return false;
        }
    } else {
        const spl_dense *d = b.dense;
        o.order = d->ndim;
        o.dtype = d->dtype;
        o.dims[0] = d->dims[0];
        o.dims[1] = d->ndim == 2 ? d->dims[1] : 0;
        if (d->ndim != 1 && d->ndim != 2) {
            err = "operand " + b.name + ": dense operands are vectors or matrices";
            return false;
        }
    }
    return true;
}

// ------------------------------------------------------------- emission

struct Emitter {
    std::ostringstream s;
    int ind = 0;
    void line(const std::string &t) {
        for (int k = 0; k < ind; ++k) s << "    ";
        s << t << "\n";
    }
    void open(const std::string &t) {
        line(t);
        ++ind;
    }
    void close(const std::string &t = "}") {
        --ind;
        line(t);
    }
};

std::string join(const std::vector<std::string> &v, const std::string &sep) {
    std::string r;
    for (size_t k = 0; k < v.size(); ++k) r += (k ? sep : "") + v[k];
    return r;
}

std::string num(int64_t v) { return std::to_string(v); }

// Everything the code generator needs about one planned statement.
struct Gen {
    const Stmt &st;
    const std::vector<OpInfo> &oi;
    const OpInfo &out;
    int out_kind;
    std::vector<int> order;
    std::vector<int> slot_of_extent;  // per variable
    // per flattened access (terms in order, factors in order)
    std::vector<const Access *> acc;
    std::vector<int> acc_term;
    std::vector<int> acc_slot;        // first slot of the access
    std::string T;                    // value type
    int w = -1;                       // second output variable (dense 2-D, CSR)
    enum Mode { kEval, kCount, kFill } mode = kEval;

    std::string coord(int v) const { return "c" + num(v); }

    bool sparse(int a) const { return oi[acc[a]->op].sparse; }
    int last_level(int a) const { return oi[acc[a]->op].order - 1; }

    void emit_terms(Emitter &e, const std::string &target) const {
        for (size_t t = 0; t < st.terms.size(); ++t) {
            std::vector<std::string> guard, fac;
            for (size_t a = 0; a < acc.size(); ++a) {
                if (acc_term[a] != static_cast<int>(t)) continue;
                const Access &x = *acc[a];
                if (sparse(a)) {
                    const int L = last_level(a);
                    guard.push_back("h" + num(a) + "_" + num(L));
                    fac.push_back("(double)V" + num(a) + "[p" + num(a) + "_" + num(L) + "]");
                } else if (x.vars.size() == 1) {
                    fac.push_back("(double)D" + num(a) + "[" + coord(x.vars[0]) + "]");
                } else {
                    fac.push_back("(double)D" + num(a) + "[" + coord(x.vars[0]) + " * L" + num(a) +
                                  " + " + coord(x.vars[1]) + "]");
                }
            }
            const std::string val = (st.terms[t].sign < 0 ? "-(" : "(") + join(fac, " * ") + ")";
            if (guard.empty())
                e.line(target + " += " + val + ";");
            else
                e.line("if (" + join(guard, " && ") + ") " + target + " += " + val + ";");
        }
    }

    std::string body_target() const {
        if (out_kind == kOutScalar) return "tot";
        if (out_kind == kOutCsr) return "acc";
        if (w < 0) return "acc0";
        // dense 2-D: F64 outputs accumulate in place, F32 ones in F64 scratch
        if (T == "double") return "O[i0 * OL + " + coord(w) + "]";
        return "W[i0 * E" + num(w) + " + " + coord(w) + "]";
    }

    void emit_level(Emitter &e, size_t depth) const {
        if (depth == order.size()) {
            emit_terms(e, body_target());
            return;
        }
        const int v = order[depth];
        struct Part {
            int a, l;
        };
        std::vector<Part> parts, dlev;
        for (size_t a = 0; a < acc.size(); ++a) {
            if (!sparse(a)) continue;
            const OpInfo &o = oi[acc[a]->op];
            for (int l = 1; l < o.order; ++l)
                if (acc[a]->vars[l] == v)
                    (o.level[l] == SPL_COMPRESSED ? parts : dlev).push_back({static_cast<int>(a), l});
        }
        // a point of v counts when, for some term, every Compressed level of
        // that term's operands indexed by v stores it (union over terms,
        // intersection within a term); a term with no such level counts
        // every coordinate, so v is then iterated densely
        bool always = false;
        std::vector<std::vector<int>> conj(st.terms.size());
        for (size_t t = 0; t < st.terms.size(); ++t) {
            for (size_t k = 0; k < parts.size(); ++k)
                if (acc_term[parts[k].a] == static_cast<int>(t)) conj[t].push_back(static_cast<int>(k));
            if (conj[t].empty()) always = true;
        }
        auto P = [&](const Part &x) { return num(x.a) + "_" + num(x.l); };
        // the merge state of access a at level l: q, e, m suffixed a_l
        auto A = [&](const Part &x) { return num(x.a) + "_" + num(x.l); };
        for (const Part &x : parts) {
            const std::string par = num(x.a) + "_" + num(x.l - 1);
            e.line("i64 q" + A(x) + " = h" + par + " ? (i64)P" + P(x) + "[p" + par + "] : 0, e" +
                   A(x) + " = h" + par + " ? (i64)P" + P(x) + "[p" + par + " + 1] : 0;");
        }
        const std::string c = coord(v);
        std::vector<std::string> cond_terms;
        for (const auto &cj : conj) {
            std::vector<std::string> m;
            for (int k : cj) m.push_back("m" + A(parts[k]));
            cond_terms.push_back("(" + join(m, " && ") + ")");
        }
        if (always) {
            e.open("for (i64 " + c + " = 0; " + c + " < E" + num(v) + "; ++" + c + ") {");
            for (const Part &x : parts)
                e.line("const bool m" + A(x) + " = q" + A(x) + " < e" + A(x) + " && (i64)C" + P(x) +
                       "[q" + A(x) + "] == " + c + ";");
            descend(e, depth, parts, dlev);
            for (const Part &x : parts) e.line("if (m" + A(x) + ") ++q" + A(x) + ";");
            e.close();
            return;
        }
        std::vector<std::string> live;
        for (const Part &x : parts) live.push_back("q" + A(x) + " < e" + A(x));
        // one term: every level must store the point, so stop at the first
        // exhausted one; several: walk until all are exhausted
        e.open("while (" + join(live, st.terms.size() == 1 ? " && " : " || ") + ") {");
        e.line("i64 " + c + " = 0x7fffffffffffffffLL;");
        for (const Part &x : parts)
            e.line("if (q" + A(x) + " < e" + A(x) + " && (i64)C" + P(x) + "[q" + A(x) + "] < " + c +
                   ") " + c + " = C" + P(x) + "[q" + A(x) + "];");
        for (const Part &x : parts)
            e.line("const bool m" + A(x) + " = q" + A(x) + " < e" + A(x) + " && (i64)C" + P(x) +
                   "[q" + A(x) + "] == " + c + ";");
        e.open("if (" + join(cond_terms, " || ") + ") {");
        descend(e, depth, parts, dlev);
        e.close();
        for (const Part &x : parts) e.line("if (m" + A(x) + ") ++q" + A(x) + ";");
        e.close();
    }

    template <typename PartT>
    void descend(Emitter &e, size_t depth, const std::vector<PartT> &parts,
                 const std::vector<PartT> &dlev) const {
        const int v = order[depth];
        for (const auto &x : parts) {
            const std::string n = num(x.a) + "_" + num(x.l);
            e.line("const i64 p" + n + " = q" + n + "; const bool h" + n + " = m" + n + ";");
        }
        for (const auto &x : dlev) {
            const std::string n = num(x.a) + "_" + num(x.l), par = num(x.a) + "_" + num(x.l - 1);
            e.line("const i64 p" + n + " = p" + par + " * N" + n + " + " + coord(v) +
                   "; const bool h" + n + " = h" + par + ";");
        }
        if (out_kind == kOutCsr && depth == 1) {
            // the second output coordinate is emitted here
            if (mode == kCount) {
                e.line("++cnt;");
                return;
            }
            e.line("double acc = 0.0;");
            emit_level(e, depth + 1);
            e.line("OC[q] = (int)" + coord(v) + "; OV[q] = (" + T + ")acc; ++q;");
            return;
        }
        emit_level(e, depth + 1);
    }

    std::string kernel(const std::string &name) const {
        Emitter e;
        e.open("extern \"C\" __global__ void __launch_bounds__(256) " + name + "(TinArgs a) {");
        e.line("const i64 i0 = (i64)blockIdx.x * 256 + threadIdx.x;");
        e.line("const i64 n0 = (i64)a.s[0];");
        e.line("if (i0 >= n0) return;");
        for (size_t v = 0; v < st.vars.size(); ++v)
            e.line("const i64 E" + num(v) + " = (i64)a.s[" + num(slot_of_extent[v]) + "];");
        for (size_t a = 0; a < acc.size(); ++a) {
            int k = acc_slot[a];
            const OpInfo &o = oi[acc[a]->op];
            if (o.sparse) {
                for (int l = 1; l < o.order; ++l) {
                    const std::string n = num(a) + "_" + num(l);
                    if (o.level[l] == SPL_COMPRESSED) {
                        e.line("const int *__restrict__ P" + n + " = (const int *)a.s[" + num(k++) + "];");
                        e.line("const int *__restrict__ C" + n + " = (const int *)a.s[" + num(k++) + "];");
                    } else {
                        e.line("const i64 N" + n + " = (i64)a.s[" + num(k++) + "];");
                    }
                }
                e.line("const " + T + " *__restrict__ V" + num(a) + " = (const " + T + " *)a.s[" + num(k++) + "];");
            } else {
                e.line("const " + T + " *__restrict__ D" + num(a) + " = (const " + T + " *)a.s[" + num(k++) + "];");
                e.line("const i64 L" + num(a) + " = (i64)a.s[" + num(k++) + "];");
            }
        }
        const int os = out_slot;
        const std::string c0 = coord(order[0]);
        e.line("const i64 " + c0 + " = i0;");
        for (size_t a = 0; a < acc.size(); ++a)
            if (sparse(a)) e.line("const i64 p" + num(a) + "_0 = i0; const bool h" + num(a) + "_0 = true;");
        if (out_kind == kOutScalar) {
            e.line("double *__restrict__ PART = (double *)a.s[" + num(os) + "];");
            e.line("double tot = 0.0;");
            emit_level(e, 1);
            e.line("PART[i0] = tot;");
        } else if (out_kind == kOutCsr) {
            e.line("int *__restrict__ OP = (int *)a.s[" + num(os) + "];");
            if (mode == kCount) {
                e.line("i64 cnt = 0;");
                emit_level(e, 1);
                e.line("OP[i0 + 1] = (int)cnt;");
            } else {
                e.line("int *__restrict__ OC = (int *)a.s[" + num(os + 1) + "];");
                e.line(T + " *__restrict__ OV = (" + T + " *)a.s[" + num(os + 2) + "];");
                e.line("i64 q = OP[i0];");
                emit_level(e, 1);
            }
        } else {
            e.line(T + " *__restrict__ O = (" + T + " *)a.s[" + num(os) + "];");
            e.line("const i64 OL = (i64)a.s[" + num(os + 1) + "];");
            if (w < 0) {
                e.line("double acc0 = 0.0;");
                emit_level(e, 1);
                e.line("O[i0] = (" + T + ")acc0;");
            } else if (T == "double") {
                e.line("for (i64 z = 0; z < E" + num(w) + "; ++z) O[i0 * OL + z] = 0.0;");
                emit_level(e, 1);
            } else {
                e.line("double *__restrict__ W = (double *)a.s[" + num(os + 2) + "];");
                e.line("for (i64 z = 0; z < E" + num(w) + "; ++z) W[i0 * E" + num(w) + " + z] = 0.0;");
                emit_level(e, 1);
                e.line("for (i64 z = 0; z < E" + num(w) + "; ++z) O[i0 * OL + z] = (float)W[i0 * E" +
                       num(w) + " + z];");
            }
        }
        e.close();
        return e.s.str();
    }

    int out_slot = 0;
};

}  // namespace

Program::~Program() {
    if (module) (void)hipModuleUnload(module);
}

spl_status plan(const char *stmt, const std::vector<Binding> &ops, const Binding &out,
                Program &prog, std::string &err) {
    if (!stmt) {
        err = "statement is NULL";
        return SPL_ERR_ARG;
    }
    Stmt st;
    Parser ps(stmt, st, err);
    if (!ps.parse()) {
        err = "index notation: " + err;
        return SPL_ERR_ARG;
    }
    // bind names
    std::vector<OpInfo> oi(ops.size());
    for (size_t k = 0; k < ops.size(); ++k) {
        if (!op_info(ops[k], oi[k], err)) return SPL_ERR_FORMAT;
        for (size_t m = 0; m < k; ++m)
            if (ops[m].name == ops[k].name) {
                err = "operand " + ops[k].name + " bound twice";
                return SPL_ERR_ARG;
            }
    }
    if (out.name != st.lhs.name) {
        err = "the output is bound as " + out.name + " but the statement assigns " + st.lhs.name;
        return SPL_ERR_ARG;
    }
    OpInfo oo;
    if (!op_info(out, oo, err)) return SPL_ERR_FORMAT;
    std::set<int> first_set;
    bool first = true;
    for (Term &t : st.terms) {
        std::set<int> vs;
        for (Access &a : t.f) {
            if (a.name == st.lhs.name) {
                err = "the output " + a.name + " appears on the right side";
                return SPL_ERR_ARG;
            }
            for (size_t k = 0; k < ops.size(); ++k)
                if (ops[k].name == a.name) a.op = static_cast<int>(k);
            if (a.op < 0) {
                err = "operand " + a.name + " is not bound";
                return SPL_ERR_ARG;
            }
            if (static_cast<int>(a.vars.size()) != oi[a.op].order) {
                err = "operand " + a.name + " has order " + std::to_string(oi[a.op].order) +
                      " but is indexed by " + std::to_string(a.vars.size()) + " variables";
                return SPL_ERR_SHAPE;
            }
            std::set<int> own(a.vars.begin(), a.vars.end());
            if (own.size() != a.vars.size()) {
                err = "operand " + a.name + " repeats an index variable";
                return SPL_ERR_UNSUPPORTED;
            }
            vs.insert(a.vars.begin(), a.vars.end());
        }
        if (!first && vs != first_set) {
            err = "every term of a sum must use the same index variables";
            return SPL_ERR_UNSUPPORTED;
        }
        first_set = vs;
        first = false;
    }
    {
        std::set<int> own(st.lhs.vars.begin(), st.lhs.vars.end());
        if (own.size() != st.lhs.vars.size()) {
            err = "the output repeats an index variable";
            return SPL_ERR_UNSUPPORTED;
        }
        for (int v : st.lhs.vars)
            if (!first_set.count(v)) {
                err = "output variable " + st.vars[v] + " does not appear on the right side";
                return SPL_ERR_ARG;
            }
    }
    // value types
    const int vt = oi.empty() ? SPL_F64 : oi[0].dtype;
    if (vt != SPL_F64 && vt != SPL_F32) {
        err = "generated leaves take F64 or F32 values";
        return SPL_ERR_DTYPE;
    }
    for (const OpInfo &o : oi)
        if (o.dtype != vt) {
            err = "every operand must have the same value type";
            return SPL_ERR_DTYPE;
        }
    // output kind
    int kind;
    if (st.lhs.vars.empty()) {
        kind = kOutScalar;
        if (oo.sparse || oo.order != 1 || oo.dims[0] != 1 || oo.dtype != SPL_F64) {
            err = "a scalar output is a dense F64 vector of one entry";
            return SPL_ERR_SHAPE;
        }
    } else if (oo.sparse) {
        kind = kOutCsr;
        if (oo.order != 2 || oo.level[1] != SPL_COMPRESSED || st.lhs.vars.size() != 2) {
            err = "a sparse output is a CSR matrix (Dense, Compressed)";
            return SPL_ERR_FORMAT;
        }
        if (oo.dtype != vt) {
            err = "the output's value type must match the operands'";
            return SPL_ERR_DTYPE;
        }
    } else {
        kind = kOutDense;
        if (oo.order != static_cast<int>(st.lhs.vars.size())) {
            err = "the dense output's order does not match the statement";
            return SPL_ERR_SHAPE;
        }
        if (oo.dtype != vt) {
            err = "the output's value type must match the operands'";
            return SPL_ERR_DTYPE;
        }
    }
    // extents
    const int nv = static_cast<int>(st.vars.size());
    std::vector<int64_t> ext(nv, -1);
    auto set_ext = [&](int v, int64_t d, const std::string &who) {
        if (ext[v] < 0) ext[v] = d;
        if (ext[v] != d) {
            err = "index " + st.vars[v] + " has extent " + std::to_string(ext[v]) + " but " + who +
                  " gives " + std::to_string(d);
            return false;
        }
        return true;
    };
    for (const Term &t : st.terms)
        for (const Access &a : t.f)
            for (size_t l = 0; l < a.vars.size(); ++l)
                if (!set_ext(a.vars[l], oi[a.op].dims[l], a.name)) return SPL_ERR_SHAPE;
    for (size_t l = 0; l < st.lhs.vars.size(); ++l)
        if (!set_ext(st.lhs.vars[l], oo.dims[l], st.lhs.name)) return SPL_ERR_SHAPE;
    for (int v = 0; v < nv; ++v)
        if (ext[v] < 0 || ext[v] > 2147483647LL) {
            err = "index " + st.vars[v] + " has no usable extent";
            return SPL_ERR_SHAPE;
        }
    // the outermost index: the first of every sparse operand (their Dense
    // first level), one thread per coordinate
    int i0 = -1;
    for (const Term &t : st.terms)
        for (const Access &a : t.f)
            if (oi[a.op].sparse) {
                if (i0 < 0) i0 = a.vars[0];
                if (a.vars[0] != i0) {
                    err = "every sparse operand must be indexed first by the same variable";
                    return SPL_ERR_UNSUPPORTED;
                }
            }
    if (i0 < 0) i0 = st.lhs.vars.empty() ? st.terms[0].f[0].vars[0] : st.lhs.vars[0];
    if (!st.lhs.vars.empty() && st.lhs.vars[0] != i0) {
        err = "the output's first index must be the sparse operands' first (each thread owns "
              "one output row)";
        return SPL_ERR_UNSUPPORTED;
    }
    // concordant loop order: a sparse operand's level l needs its levels
    // before l outside it
    std::vector<std::set<int>> need(nv);
    bool uses_sparse[64] = {};
    if (nv > 64) {
        err = "too many index variables";
        return SPL_ERR_UNSUPPORTED;
    }
    for (const Term &t : st.terms)
        for (const Access &a : t.f)
            if (oi[a.op].sparse)
                for (size_t l = 0; l < a.vars.size(); ++l) {
                    uses_sparse[a.vars[l]] = true;
                    for (size_t m = 0; m < l; ++m) need[a.vars[l]].insert(a.vars[m]);
                }
    std::vector<int> order{i0};
    std::vector<bool> placed(nv, false);
    placed[i0] = true;
    const int w = st.lhs.vars.size() == 2 ? st.lhs.vars[1] : -1;
    while (static_cast<int>(order.size()) < nv) {
        int best = -1, best_rank = 1 << 30;
        for (int v = 0; v < nv; ++v) {
            if (placed[v]) continue;
            bool ready = true;
            for (int u : need[v]) ready = ready && placed[u];
            if (!ready) continue;
            // sparse output: its second index next; then the variables of
            // sparse levels; dense-only variables innermost
            int rank = (kind == kOutCsr && v == w) ? 0 : uses_sparse[v] ? 1 : 2;
            if (rank < best_rank) {
                best = v;
                best_rank = rank;
            }
        }
        if (best < 0) {
            err = "the sparse operands' level orders admit no common loop order";
            return SPL_ERR_UNSUPPORTED;
        }
        order.push_back(best);
        placed[best] = true;
    }
    if (kind == kOutCsr && order[1] != w) {
        err = "a sparse output's second index must be iterated right after its first";
        return SPL_ERR_UNSUPPORTED;
    }
    // slots and code
    Gen g{st, oi, oo, kind};
    g.order = order;
    g.T = vt == SPL_F64 ? "double" : "float";
    g.w = w;
    prog.slots.clear();
    prog.slots.push_back({Slot::kRows, -1, i0});
    g.slot_of_extent.resize(nv);
    for (int v = 0; v < nv; ++v) {
        g.slot_of_extent[v] = static_cast<int>(prog.slots.size());
        prog.slots.push_back({Slot::kExtent, -1, v});
    }
    for (size_t t = 0; t < st.terms.size(); ++t)
        for (const Access &a : st.terms[t].f) {
            g.acc.push_back(&a);
            g.acc_term.push_back(static_cast<int>(t));
            g.acc_slot.push_back(static_cast<int>(prog.slots.size()));
            const OpInfo &o = oi[a.op];
            if (o.sparse) {
                for (int l = 1; l < o.order; ++l) {
                    if (o.level[l] == SPL_COMPRESSED) {
                        prog.slots.push_back({Slot::kPos, a.op, l});
                        prog.slots.push_back({Slot::kCrd, a.op, l});
                    } else {
                        prog.slots.push_back({Slot::kLevelDim, a.op, l});
                    }
                }
                prog.slots.push_back({Slot::kVals, a.op, 0});
            } else {
                prog.slots.push_back({Slot::kDenseData, a.op, 0});
                prog.slots.push_back({Slot::kDenseLd, a.op, 0});
            }
        }
    g.out_slot = static_cast<int>(prog.slots.size());
    if (kind == kOutScalar) {
        prog.slots.push_back({Slot::kPartials, -1, 0});
    } else if (kind == kOutCsr) {
        prog.slots.push_back({Slot::kOutPos, -1, 0});
        prog.slots.push_back({Slot::kOutCrd, -1, 0});
        prog.slots.push_back({Slot::kOutVals, -1, 0});
    } else {
        prog.slots.push_back({Slot::kOutData, -1, 0});
        prog.slots.push_back({Slot::kOutLd, -1, 0});
        if (w >= 0 && vt == SPL_F32) prog.slots.push_back({Slot::kScratch, -1, 0});
    }
    if (prog.slots.size() > 120) {
        err = "statement too large";
        return SPL_ERR_UNSUPPORTED;
    }

    std::ostringstream src;
    src << "// generated from: " << stmt << "\n";
    src << "typedef long long i64;\n";
    src << "struct TinArgs { unsigned long long s[" << prog.slots.size() << "]; };\n";
    if (kind == kOutCsr) {
        g.mode = Gen::kCount;
        src << g.kernel("tin_count");
        g.mode = Gen::kFill;
        src << g.kernel("tin_fill");
    } else {
        g.mode = Gen::kEval;
        src << g.kernel("tin_eval");
    }
    prog.source = src.str();
    prog.out_kind = kind;
    prog.vtype = vt;
    prog.rows = ext[i0];
    prog.extents = ext;
    prog.out_cols = w >= 0 ? ext[w] : 1;
    prog.scratch_rows = kind == kOutDense && w >= 0 && vt == SPL_F32;
    // the cache key: the statement and every operand's format, dtype and
    // shape (the shapes are runtime slots, but they are checked above)
    std::ostringstream key;
    key << stmt << "|" << out.name << ":" << oo.sparse << oo.order << oo.level[1] << oo.dtype;
    for (size_t k = 0; k < ops.size(); ++k)
        key << "|" << ops[k].name << ":" << oi[k].sparse << oi[k].order << oi[k].level[0]
            << oi[k].level[1] << oi[k].level[2] << oi[k].dtype;
    prog.key = key.str();
    return SPL_OK;
}

spl_status compile(Program &prog, std::string &err) {
    hiprtcProgram p = nullptr;
    if (hiprtcCreateProgram(&p, prog.source.c_str(), "tin.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return SPL_ERR_HIP;
    }
    // no packed FP32 instructions in generated code either
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(p, 6, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(p, &n);
        std::string log(n + 1, '\0');
        if (n) hiprtcGetProgramLog(p, &log[0]);
        err = "generated leaf did not compile: " + log;
        hiprtcDestroyProgram(&p);
        return SPL_ERR_HIP;
    }
    size_t n = 0;
    hiprtcGetCodeSize(p, &n);
    std::vector<char> code(n);
    hiprtcGetCode(p, code.data());
    hiprtcDestroyProgram(&p);
    hipError_t e = hipModuleLoadData(&prog.module, code.data());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        prog.module = nullptr;
        err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        return SPL_ERR_HIP;
    }
    auto get = [&](const char *name, hipFunction_t &f) {
        hipError_t x = hipModuleGetFunction(&f, prog.module, name);
        if (x != hipSuccess) {
            (void)hipGetLastError();
            err = std::string("hipModuleGetFunction(") + name + "): " + hipGetErrorString(x);
            return false;
        }
        return true;
    };
    if (prog.out_kind == kOutCsr) {
        if (!get("tin_count", prog.f_count) || !get("tin_fill", prog.f_fill)) return SPL_ERR_HIP;
    } else if (!get("tin_eval", prog.f_eval)) {
        return SPL_ERR_HIP;
    }
    return SPL_OK;
}

void fill_slots(const Program &prog, const std::vector<Binding> &ops, const Binding &out,
                const int32_t *out_pos, void *partials, void *scratch,
                std::vector<unsigned long long> &slots) {
    auto u = [](const void *p) { return static_cast<unsigned long long>(reinterpret_cast<uintptr_t>(p)); };
    slots.assign(prog.slots.size(), 0);
    for (size_t k = 0; k < prog.slots.size(); ++k) {
        const Slot &s = prog.slots[k];
        const Binding *b = s.operand >= 0 ? &ops[s.operand] : &out;
        switch (s.kind) {
        case Slot::kRows: slots[k] = static_cast<unsigned long long>(prog.rows); break;
        case Slot::kExtent: slots[k] = static_cast<unsigned long long>(prog.extents[s.level]); break;
        case Slot::kPos: slots[k] = u(b->sparse->pos[s.level]); break;
        case Slot::kCrd: slots[k] = u(b->sparse->crd[s.level]); break;
        case Slot::kVals: slots[k] = u(b->sparse->vals); break;
        case Slot::kLevelDim:
            slots[k] = static_cast<unsigned long long>(b->sparse->dims[s.level]);
            break;
        case Slot::kDenseData: slots[k] = u(b->dense->data); break;
        case Slot::kDenseLd: slots[k] = static_cast<unsigned long long>(b->dense->ld); break;
        case Slot::kOutData: slots[k] = u(out.dense->data); break;
        case Slot::kOutLd: slots[k] = static_cast<unsigned long long>(out.dense->ld); break;
        case Slot::kOutPos: slots[k] = u(out_pos); break;
        case Slot::kOutCrd: slots[k] = out.sparse ? u(out.sparse->crd[1]) : 0; break;
        case Slot::kOutVals: slots[k] = out.sparse ? u(out.sparse->vals) : 0; break;
        case Slot::kPartials: slots[k] = u(partials); break;
        case Slot::kScratch: slots[k] = u(scratch); break;
        }
    }
}

size_t workspace_bytes(const Program &prog, bool symbolic) {
    auto up = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    const size_t rows = static_cast<size_t>(prog.rows);
    size_t b = 0;
    if (prog.out_kind == kOutScalar) b += up(rows * 8);
    if (prog.scratch_rows) b += up(rows * static_cast<size_t>(prog.out_cols) * 8);
    if (symbolic) b += up(static_cast<size_t>(spadd3_scan_tiles(prog.rows)) * 8) + up(8);
    return b;
}

}  // namespace tin
}  // namespace spl
