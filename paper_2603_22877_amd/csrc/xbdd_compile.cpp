// Host compiler: constraint -> xBDD (paper, Supplementary Note 3, Def. "xBDD").
//
// Each constraint's formula is built as a reduced ordered BDD over its distinct variables
// (Booleans by id, then atoms by id; atoms are propositional variables and no LP pruning
// is done, as the paper prescribes for xBDDs). The paper uses the CUDD package for this
// step; here a small ROBDD package (unique table + computed table + ITE) is written for
// the purpose. Constraints whose formula has the same structure over the same pattern of
// support slots share one compiled diagram ("template"), so a 720,000-constraint placement
// instance compiles a handful of diagrams. Nodes are emitted in topological order
// (ascending variable level, root first), the order in which the forward traversal visits
// them (Alg. "Forward Traversal of XBDDs").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "fsmt_internal.hpp"

namespace fsmt {

// ------------------------------------------------------------------ error state
static thread_local char g_err[512] = "";

fsmt_status set_error(fsmt_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}
void clear_error() { g_err[0] = 0; }
const char *last_error() { return g_err; }

// ------------------------------------------------------------------ ROBDD package
class Robdd {
  public:
    static constexpr uint32_t kFalse = 0, kTrue = 1;
    static constexpr uint32_t kTermVar = 0xFFFFFFFFu;

    Robdd() {
        var_ = {kTermVar, kTermVar};
        hi_ = {kFalse, kTrue};
        lo_ = {kFalse, kTrue};
    }
    uint32_t var(uint32_t f) const { return var_[f]; }
    uint32_t hi(uint32_t f) const { return hi_[f]; }
    uint32_t lo(uint32_t f) const { return lo_[f]; }
    size_t size() const { return var_.size(); }

    uint32_t literal(uint32_t v, bool neg) { return neg ? mk(v, kFalse, kTrue) : mk(v, kTrue, kFalse); }

    uint32_t ite(uint32_t f, uint32_t g, uint32_t h) {
        if (f == kTrue) return g;
        if (f == kFalse) return h;
        if (g == h) return g;
        if (g == kTrue && h == kFalse) return f;
        Key k{f, g, h};
        auto it = computed_.find(k);
        if (it != computed_.end()) return it->second;
        uint32_t v = std::min(var_[f], std::min(var_[g], var_[h]));
        uint32_t r = mk(v, ite(cof(f, v, true), cof(g, v, true), cof(h, v, true)),
                        ite(cof(f, v, false), cof(g, v, false), cof(h, v, false)));
        computed_.emplace(k, r);
        return r;
    }
    uint32_t NOT(uint32_t f) { return ite(f, kFalse, kTrue); }
    uint32_t AND(uint32_t f, uint32_t g) { return ite(f, g, kFalse); }
    uint32_t OR(uint32_t f, uint32_t g) { return ite(f, kTrue, g); }
    uint32_t XOR(uint32_t f, uint32_t g) { return ite(f, NOT(g), g); }

  private:
    struct Key {
        uint32_t a, b, c;
        bool operator==(const Key &o) const { return a == o.a && b == o.b && c == o.c; }
    };
    struct KeyHash {
        size_t operator()(const Key &k) const {
            uint64_t x = (uint64_t)k.a * 0x9E3779B97F4A7C15ull ^ (uint64_t)k.b * 0xC2B2AE3D27D4EB4Full ^
                         (uint64_t)k.c * 0x165667B19E3779F9ull;
            return (size_t)(x ^ (x >> 29));
        }
    };
    uint32_t cof(uint32_t f, uint32_t v, bool high) const {
        if (var_[f] != v) return f;
        return high ? hi_[f] : lo_[f];
    }
    uint32_t mk(uint32_t v, uint32_t h, uint32_t l) {
        if (h == l) return h;
        Key k{v, h, l};
        auto it = unique_.find(k);
        if (it != unique_.end()) return it->second;
        uint32_t id = (uint32_t)var_.size();
        var_.push_back(v);
        hi_.push_back(h);
        lo_.push_back(l);
        unique_.emplace(k, id);
        return id;
    }
    std::vector<uint32_t> var_, hi_, lo_;
    std::unordered_map<Key, uint32_t, KeyHash> unique_, computed_;
};

// ------------------------------------------------------------------ constraint structure

struct ConView {
    int kind = 0, param = 0;
    std::vector<int32_t> ids;        // sorted distinct variable ids (the support)
    std::vector<int32_t> lit_slot;   // literal position -> slot
    std::vector<uint8_t> lit_neg;
    const int32_t *ops = nullptr;
    int64_t n_ops = 0;
    int n_bslots = 0;
};

static bool symmetric_value(int kind, int param, int L, int t) {
    switch (kind) {
    case FSMT_CLAUSE: return t >= 1;
    case FSMT_AND: return t == L;
    case FSMT_XOR: return (t & 1) != 0;
    case FSMT_NAE: return t > 0 && t < L;
    case FSMT_CARD_LE: return t <= param;
    case FSMT_CARD_GE: return t >= param;
    }
    return false;
}

// Builds the constraint's BDD over slot variables; returns the root.
static uint32_t build_formula(Robdd &B, const ConView &cv) {
    const int L = (int)cv.lit_slot.size();
    std::vector<uint32_t> lits(L);
    for (int t = 0; t < L; ++t) lits[t] = B.literal((uint32_t)cv.lit_slot[t], cv.lit_neg[t] != 0);
    if (cv.kind == FSMT_EXPR) {
        std::vector<uint32_t> st;
        for (int64_t i = 0; i < cv.n_ops; ++i) {
            int op = cv.ops[i];
            if (op >= 0) { st.push_back(lits[op]); continue; }
            if (op == FSMT_X_TRUE) { st.push_back(Robdd::kTrue); continue; }
            if (op == FSMT_X_FALSE) { st.push_back(Robdd::kFalse); continue; }
            if (op == FSMT_X_NOT) { st.back() = B.NOT(st.back()); continue; }
            if (op == FSMT_X_ITE) {
                uint32_t e = st.back(); st.pop_back();
                uint32_t th = st.back(); st.pop_back();
                uint32_t c = st.back(); st.pop_back();
                st.push_back(B.ite(c, th, e));
                continue;
            }
            uint32_t y = st.back(); st.pop_back();
            uint32_t x = st.back(); st.pop_back();
            st.push_back(op == FSMT_X_AND ? B.AND(x, y) : op == FSMT_X_OR ? B.OR(x, y) : B.XOR(x, y));
        }
        return st.back();
    }
    if (cv.kind == FSMT_CLAUSE) {
        uint32_t r = Robdd::kFalse;
        for (int t = L - 1; t >= 0; --t) r = B.OR(lits[t], r);
        return r;
    }
    if (cv.kind == FSMT_AND) {
        uint32_t r = Robdd::kTrue;
        for (int t = L - 1; t >= 0; --t) r = B.AND(lits[t], r);
        return r;
    }
    // symmetric kinds: F(i, t) = function of literals i..L-1 given t true literals so far
    std::vector<uint32_t> next(L + 1), cur(L + 1);
    for (int t = 0; t <= L; ++t) next[t] = symmetric_value(cv.kind, cv.param, L, t) ? Robdd::kTrue : Robdd::kFalse;
    for (int i = L - 1; i >= 0; --i) {
        for (int t = 0; t <= i; ++t) cur[t] = B.ite(lits[i], next[t + 1], next[t]);
        std::swap(cur, next);
    }
    return next[0];
}

static fsmt_status check_expr(const ConView &cv, int n_lits, int c) {
    int sp = 0;
    for (int64_t i = 0; i < cv.n_ops; ++i) {
        int op = cv.ops[i];
        if (op >= 0) {
            if (op >= n_lits) return set_error(FSMT_EINVAL, "constraint %d: EXPR pushes literal %d of %d", c, op, n_lits);
            ++sp;
        } else if (op == FSMT_X_TRUE || op == FSMT_X_FALSE) {
            ++sp;
        } else if (op == FSMT_X_NOT) {
            if (sp < 1) return set_error(FSMT_EINVAL, "constraint %d: EXPR stack underflow", c);
        } else if (op == FSMT_X_ITE) {
            if (sp < 3) return set_error(FSMT_EINVAL, "constraint %d: EXPR stack underflow", c);
            sp -= 2;
        } else if (op == FSMT_X_AND || op == FSMT_X_OR || op == FSMT_X_XOR) {
            if (sp < 2) return set_error(FSMT_EINVAL, "constraint %d: EXPR stack underflow", c);
            --sp;
        } else {
            return set_error(FSMT_EINVAL, "constraint %d: unknown EXPR op %d", c, op);
        }
    }
    if (sp != 1) return set_error(FSMT_EINVAL, "constraint %d: EXPR leaves %d values", c, sp);
    return FSMT_OK;
}

struct Template {
    int n_nodes = 0, n_slots = 0, n_bslots = 0, root = 0;
    int pair_l = 0;   // > 0: pair disjunction with this many XOR pairs (closed-form evaluation)
    GdInfo gd{};      // guarded disjunction when gd.k >= 0 (closed-form evaluation)
    std::vector<Node> nodes;
};

// Guarded disjunction, read off the levelized diagram itself: for the smallest k <= kGdMaxSel
// such that, for every assignment g of slots 0..k-1, the path that takes g's branches at
// those slots reaches a terminal or a chain whose every node has one edge to the True
// terminal (the literal of that node: positive when its true edge is that edge) and its
// other edge to the next node of the chain or to the False terminal. A slot must keep its
// polarity in every chain. The false-terminal mass of such a diagram is the sum over g of
// P[g] times the product of the chain's literal-false probabilities, which is what the
// forward pass accumulates (chains that share their tails add their masses into the shared
// nodes, and a selector the path skips contributes both of its branches).
// Separable guarded disjunction (GdInfo::sep): two selectors and no other Boolean, every
// assignment reaches a disjunction of atoms, and the disjunction of assignment (v0, v1) is
// the union of a set picked by v0 alone and one picked by v1 alone: S_{0,v0} = the atoms
// common to (v0, F) and (v0, T), S_{1,v1} likewise. The four sets must be disjoint and hold at
// most two atoms each (a rectangle pair's rotation ITE: each rotation bit picks the two atoms
// that use that rectangle's sides).
static void gd_separable(GdInfo &g, int nb, int na) {
    g.sep = 0;
    g.sep_slots = 0;
    if (g.k != 2 || nb != 2 || na > kGdMaxAtoms) return;
    uint32_t mA[4];
    for (int c = 0; c < 4; ++c) {
        if ((g.mask[c] >> 31) || (g.mask[c] & 3u)) return;
        mA[c] = g.mask[c] >> 2;
    }
    // assignment c: bit 0 = selector 0 True, bit 1 = selector 1 True
    const uint32_t S[4] = {mA[0] & mA[2], mA[1] & mA[3], mA[0] & mA[1], mA[2] & mA[3]};
    for (int c = 0; c < 4; ++c)
        if (mA[c] != (S[c & 1] | S[2 + (c >> 1)])) return;
    int total = 0;
    uint32_t all = 0;
    for (int q = 0; q < 4; ++q) {
        const int cnt = __builtin_popcount(S[q]);
        if (cnt > 2) return;
        total += cnt;
        all |= S[q];
    }
    if (__builtin_popcount(all) != total) return;   // not disjoint
    uint32_t slots = 0;
    for (int q = 0; q < 4; ++q) {
        int f = 0;
        for (int j = 0; j < na; ++j)
            if ((S[q] >> j) & 1u) slots |= (uint32_t)j << (4 * (2 * q + f++));
        for (; f < 2; ++f) slots |= (uint32_t)kGdMaxAtoms << (4 * (2 * q + f));
    }
    g.sep = 1;
    g.sep_slots = slots;
}

static GdInfo gd_family(const Template &T) {
    GdInfo g{};
    g.k = -1;
    const int N = T.n_nodes;
    if (N == 0 || T.n_bslots > kGdMaxBool || T.n_slots - T.n_bslots > kGdMaxAtoms) return g;
    for (int k = 0; k <= std::min(kGdMaxSel, T.n_bslots); ++k) {   // selectors are Booleans
        bool ok = true;
        uint32_t neg = 0, seen = 0, mask[4] = {0, 0, 0, 0};
        for (int c = 0; c < (1 << k) && ok; ++c) {
            int v = 0;
            while (v < N && T.nodes[v].slot < k) v = ((c >> T.nodes[v].slot) & 1) ? T.nodes[v].hi : T.nodes[v].lo;
            if (v == N) { mask[c] = 1u << 31; continue; }   // True: no false mass
            uint32_t m = 0;
            while (v < N && ok) {
                const Node &x = T.nodes[v];
                uint32_t pol;
                int next;
                if (x.hi == N) { pol = 0; next = x.lo; }
                else if (x.lo == N) { pol = 1; next = x.hi; }
                else { ok = false; break; }
                const uint32_t bit = 1u << x.slot;
                if ((seen & bit) && ((neg & bit) != 0) != (pol != 0)) { ok = false; break; }
                seen |= bit;
                if (pol) neg |= bit;
                m |= bit;
                v = next;
            }
            if (ok && v != N + 1) ok = false;   // a chain ends at the False terminal
            mask[c] = m;
        }
        if (ok) {
            for (int c = 0; c < 4; ++c) g.mask[c] = c < (1 << k) ? mask[c] : 0;
            g.neg = neg;
            g.k = k;
            gd_separable(g, T.n_bslots, T.n_slots - T.n_bslots);
            return g;
        }
    }
    return g;
}

// Pair disjunction: the EXPR program OR_i (l_{2i} XOR l_{2i+1}) OR l_{2L} OR ... OR
// l_{2L+T-1}, written as [0 1 XOR (2i 2i+1 XOR OR)* (t OR)*], every literal positive and on
// its own slot in literal order, the 2L pair literals Booleans and the T others atoms.
// Returns L, or 0 when the constraint is not of this form.
static int pair_family(const ConView &cv, int n_lits) {
    if (cv.kind != FSMT_EXPR || (int)cv.ids.size() != n_lits) return 0;
    for (int t = 0; t < n_lits; ++t)
        if (cv.lit_slot[t] != t || cv.lit_neg[t]) return 0;
    auto op = [&](int64_t i) { return i < cv.n_ops ? cv.ops[i] : INT32_MIN; };
    if (!(op(0) == 0 && op(1) == 1 && op(2) == FSMT_X_XOR)) return 0;
    int64_t q = 3;
    int L = 1, T = 0;
    while (op(q) == 2 * L && op(q + 1) == 2 * L + 1 && op(q + 2) == FSMT_X_XOR && op(q + 3) == FSMT_X_OR) {
        q += 4;
        ++L;
    }
    while (op(q) == 2 * L + T && op(q + 1) == FSMT_X_OR) {
        q += 2;
        ++T;
    }
    if (q != cv.n_ops || 2 * L + T != n_lits || cv.n_bslots != 2 * L) return 0;
    return (L <= kPairMaxL && T <= kPairMaxT) ? L : 0;
}

// Levelize: nodes reachable from the root sorted by (level, id); root first.
static fsmt_status emit_template(const Robdd &B, uint32_t root, const ConView &cv, int max_nodes,
                                 Template &T) {
    T.n_slots = (int)cv.ids.size();
    T.n_bslots = cv.n_bslots;
    if (root == Robdd::kTrue || root == Robdd::kFalse) {
        T.n_nodes = 0;
        T.root = root == Robdd::kTrue ? 0 : 1;
        return FSMT_OK;
    }
    std::vector<uint32_t> stack{root}, order;
    std::unordered_map<uint32_t, int> seen;
    seen.emplace(root, 0);
    while (!stack.empty()) {
        uint32_t f = stack.back();
        stack.pop_back();
        order.push_back(f);
        for (uint32_t ch : {B.hi(f), B.lo(f)})
            if (ch > Robdd::kTrue && seen.emplace(ch, 0).second) stack.push_back(ch);
    }
    if ((int)order.size() > max_nodes)
        return set_error(FSMT_ELIMIT, "diagram with %zu nodes exceeds max_nodes=%d", order.size(), max_nodes);
    std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return B.var(x) != B.var(y) ? B.var(x) < B.var(y) : x < y;
    });
    const int N = (int)order.size();
    for (int i = 0; i < N; ++i) seen[order[i]] = i;
    auto child = [&](uint32_t ch) -> uint16_t {
        if (ch == Robdd::kTrue) return (uint16_t)N;
        if (ch == Robdd::kFalse) return (uint16_t)(N + 1);
        return (uint16_t)seen[ch];
    };
    T.n_nodes = N;
    T.root = 0;
    T.nodes.resize(N);
    for (int i = 0; i < N; ++i) {
        uint32_t f = order[i];
        T.nodes[i] = Node{(uint16_t)B.var(f), child(B.hi(f)), child(B.lo(f)), 0};
    }
    return FSMT_OK;
}

// ------------------------------------------------------------------ device upload helper
struct Uploader {
    fsmt_xbdd *h;
    template <class T>
    fsmt_status put(T **dst, const std::vector<T> &src, const char *what) {
        size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess)
            return set_error(FSMT_ENOMEM, "hipMalloc of %zu bytes for %s failed", bytes, what);
        h->allocations.push_back(p);
        if (!src.empty() && hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return set_error(FSMT_EHIP, "hipMemcpy for %s failed", what);
        h->table_bytes += (int64_t)(src.size() * sizeof(T));
        *dst = (T *)p;
        return FSMT_OK;
    }
};

static void release(fsmt_xbdd *h) {
    if (!h) return;
    if (h->allocations.empty()) {
        delete h;
        return;
    }
    int prev = 0;
    bool sw = hipGetDevice(&prev) == hipSuccess && prev != h->device;
    if (sw) (void)hipSetDevice(h->device);
    for (void *p : h->allocations) (void)hipFree(p);
    if (sw) (void)hipSetDevice(prev);
    delete h;
}

static fsmt_status compile_impl(const fsmt_problem *P, const fsmt_compile_opts *opts, fsmt_xbdd **out) {
    if (!P || !out) return set_error(FSMT_EINVAL, "null problem or output pointer");
    *out = nullptr;
    const int n = P->n_bool, m = P->n_real, A = P->n_atoms, C = P->n_cons;
    if (n < 0 || m < 0 || A < 0 || C < 0) return set_error(FSMT_EINVAL, "negative size");
    if ((A > 0 && (!P->atom_ptr || !P->atom_var || !P->atom_coef || !P->atom_rhs || !P->atom_op)) ||
        (C > 0 && (!P->con_kind || !P->con_ptr || !P->con_lit)) || (m > 0 && (!P->real_lo || !P->real_hi)))
        return set_error(FSMT_EINVAL, "null array in problem");
    const int max_nodes = (opts && opts->max_nodes > 0) ? std::min(opts->max_nodes, 65000) : 1024;
    const bool host_only = opts && opts->device == FSMT_HOST_ONLY;
    if (opts && opts->messages != FSMT_MSG_AUTO && opts->messages != FSMT_MSG_LDS && opts->messages != FSMT_MSG_GENERIC)
        return set_error(FSMT_EINVAL, "messages must be FSMT_MSG_AUTO, FSMT_MSG_LDS or FSMT_MSG_GENERIC");
    const bool closed = !(opts && opts->messages == FSMT_MSG_GENERIC);
    if (opts && opts->projection != FSMT_PROJ_UNIT && opts->projection != FSMT_PROJ_BOX)
        return set_error(FSMT_EINVAL, "projection must be FSMT_PROJ_UNIT or FSMT_PROJ_BOX");
    int h_box_units = 0;
    int device = (opts && opts->device >= 0) ? opts->device : -1;
    if (!host_only && device < 0 && hipGetDevice(&device) != hipSuccess)
        return set_error(FSMT_EHIP, "hipGetDevice failed");
    if ((int64_t)n + A > INT32_MAX / 2) return set_error(FSMT_ELIMIT, "too many variables");

    // ---- atoms: validate and normalize to "<=" form
    std::vector<int32_t> a_ptr(A + 1, 0), a_var;
    std::vector<double> a_coef, a_rhs(A), a_scale(A);
    std::vector<uint8_t> a_strict(A);
    if (A > 0 && P->atom_ptr[0] != 0) return set_error(FSMT_EINVAL, "atom_ptr[0] != 0");
    for (int k = 0; k < A; ++k) {
        int64_t e0 = P->atom_ptr[k], e1 = P->atom_ptr[k + 1];
        if (e1 <= e0) return set_error(FSMT_EINVAL, "atom %d has no coefficient", k);
        int op = P->atom_op[k];
        if (op == FSMT_EQ) return set_error(FSMT_EUNSUPPORTED, "atom %d: '=' atoms are not supported", k);
        if (op < FSMT_LE || op > FSMT_GT) return set_error(FSMT_EINVAL, "atom %d: bad operator %d", k, op);
        double sgn = (op == FSMT_GE || op == FSMT_GT) ? -1.0 : 1.0;
        double nrm = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            int32_t j = P->atom_var[e];
            if (j < 0 || j >= m) return set_error(FSMT_EINVAL, "atom %d: real variable %d out of range", k, j);
            double q = P->atom_coef[e];
            if (!std::isfinite(q)) return set_error(FSMT_EINVAL, "atom %d: non-finite coefficient", k);
            a_var.push_back(j);
            a_coef.push_back(sgn * q);
            nrm += q * q;
        }
        if (!(nrm > 0.0)) return set_error(FSMT_EINVAL, "atom %d: all coefficients are zero", k);
        if (!std::isfinite(P->atom_rhs[k])) return set_error(FSMT_EINVAL, "atom %d: non-finite rhs", k);
        if ((int64_t)a_var.size() > INT32_MAX) return set_error(FSMT_ELIMIT, "too many atom coefficients");
        a_ptr[k + 1] = (int32_t)a_var.size();
        a_rhs[k] = sgn * P->atom_rhs[k];
        a_scale[k] = 1.0 / (std::sqrt(2.0) * std::sqrt(nrm));
        a_strict[k] = (op == FSMT_LT || op == FSMT_GT) ? 1 : 0;
    }
    for (int j = 0; j < m; ++j)
        if (!(P->real_lo[j] <= P->real_hi[j])) return set_error(FSMT_EINVAL, "real %d: lo > hi", j);

    // ---- constraints -> templates
    std::unordered_map<std::string, int> tpl_index;
    std::vector<Template> tpls;
    std::vector<int32_t> con_tpl(C);
    std::vector<int64_t> con_sup_off(C + 1, 0);
    std::vector<int32_t> con_ids;   // concatenated supports in original order
    std::vector<int32_t> key;
    std::vector<std::pair<int32_t, int>> tmp;
    if (C > 0 && P->con_ptr[0] != 0) return set_error(FSMT_EINVAL, "con_ptr[0] != 0");
    for (int c = 0; c < C; ++c) {
        int64_t l0 = P->con_ptr[c], l1 = P->con_ptr[c + 1];
        if (l1 < l0) return set_error(FSMT_EINVAL, "constraint %d: con_ptr not monotone", c);
        const int L = (int)(l1 - l0);
        ConView cv;
        cv.kind = P->con_kind[c];
        cv.param = P->con_param ? P->con_param[c] : 0;
        if (cv.kind < FSMT_CLAUSE || cv.kind > FSMT_EXPR) return set_error(FSMT_EINVAL, "constraint %d: bad kind %d", c, cv.kind);
        tmp.clear();
        for (int t = 0; t < L; ++t) {
            int32_t lit = P->con_lit[l0 + t];
            if (lit < 0 || (lit >> 1) >= n + A) return set_error(FSMT_EINVAL, "constraint %d: literal %d out of range", c, lit);
            tmp.emplace_back(lit >> 1, t);
        }
        std::sort(tmp.begin(), tmp.end());
        cv.lit_slot.assign(L, 0);
        cv.lit_neg.assign(L, 0);
        for (auto &pr : tmp) {
            if (cv.ids.empty() || cv.ids.back() != pr.first) cv.ids.push_back(pr.first);
            cv.lit_slot[pr.second] = (int32_t)cv.ids.size() - 1;
            cv.lit_neg[pr.second] = (uint8_t)(P->con_lit[l0 + pr.second] & 1);
        }
        if (cv.ids.size() > 4096) return set_error(FSMT_ELIMIT, "constraint %d: support of %zu variables", c, cv.ids.size());
        cv.n_bslots = 0;
        while (cv.n_bslots < (int)cv.ids.size() && cv.ids[cv.n_bslots] < n) ++cv.n_bslots;
        if (cv.kind == FSMT_EXPR) {
            if (!P->expr_ptr || !P->expr_ops) return set_error(FSMT_EINVAL, "EXPR constraint %d without expr arrays", c);
            cv.ops = P->expr_ops + P->expr_ptr[c];
            cv.n_ops = P->expr_ptr[c + 1] - P->expr_ptr[c];
            if (cv.n_ops < 0) return set_error(FSMT_EINVAL, "constraint %d: expr_ptr not monotone", c);
            fsmt_status rc = check_expr(cv, L, c);
            if (rc) return rc;
        }
        // structural key: kind, param, slot pattern of literals, slot kinds, program
        key.clear();
        key.push_back(cv.kind);
        key.push_back((cv.kind == FSMT_CARD_LE || cv.kind == FSMT_CARD_GE) ? cv.param : 0);
        key.push_back(L);
        key.push_back((int32_t)cv.ids.size());
        key.push_back(cv.n_bslots);
        for (int t = 0; t < L; ++t) key.push_back(cv.lit_slot[t] * 2 + cv.lit_neg[t]);
        for (int64_t i = 0; i < cv.n_ops; ++i) key.push_back(cv.ops[i]);
        // with the closed forms, small constraints are also keyed by their atoms' forms
        // (terms, strictness, scale, coefficients with the larger first), so the members of a
        // guarded-disjunction template share them slot by slot
        if (closed && cv.n_bslots <= kGdMaxBool && (int)cv.ids.size() - cv.n_bslots <= kGdMaxAtoms) {
            for (size_t s = cv.n_bslots; s < cv.ids.size(); ++s) {
                const int k = cv.ids[s] - n;
                const int64_t e0 = a_ptr[k], nt = a_ptr[k + 1] - e0;
                float c0 = nt >= 1 ? (float)a_coef[e0] : 0.0f, c1 = nt >= 2 ? (float)a_coef[e0 + 1] : 0.0f;
                if (nt == 2 && c1 > c0) std::swap(c0, c1);
                const float sc = (float)a_scale[k];
                int32_t w[3];
                std::memcpy(&w[0], &c0, 4);
                std::memcpy(&w[1], &c1, 4);
                std::memcpy(&w[2], &sc, 4);
                key.push_back((int32_t)(nt * 2 + a_strict[k]));
                key.insert(key.end(), w, w + 3);
            }
        }
        std::string ks((const char *)key.data(), key.size() * sizeof(int32_t));
        auto it = tpl_index.find(ks);
        int t_id;
        if (it == tpl_index.end()) {
            Robdd B;
            uint32_t root = build_formula(B, cv);
            Template T;
            fsmt_status rc = emit_template(B, root, cv, max_nodes, T);
            if (rc) return set_error(rc, "constraint %d: %s", c, last_error());
            if (T.n_nodes > 0 && closed) T.pair_l = pair_family(cv, L);
            T.gd.k = -1;
            if (T.pair_l == 0 && closed) T.gd = gd_family(T);
            if (T.n_slots > 65535) return set_error(FSMT_ELIMIT, "constraint %d: support too large", c);
            t_id = (int)tpls.size();
            tpls.push_back(std::move(T));
            tpl_index.emplace(std::move(ks), t_id);
        } else {
            t_id = it->second;
        }
        con_tpl[c] = t_id;
        con_ids.insert(con_ids.end(), cv.ids.begin(), cv.ids.end());
        con_sup_off[c + 1] = (int64_t)con_ids.size();
    }

    // ---- buckets: template-major, original order inside, padded to 64 positions
    const int T = (int)tpls.size();
    std::vector<std::vector<int32_t>> members(T);
    for (int c = 0; c < C; ++c) members[con_tpl[c]].push_back(c);
    auto *h = new (std::nothrow) fsmt_xbdd();
    if (!h) return set_error(FSMT_ENOMEM, "out of host memory");
    h->device = device;
    h->n_bool = n;
    h->n_real = m;
    h->n_atoms = A;
    h->n_cons = C;
    h->n_tpl = T;
    h->nnz = (int64_t)a_var.size();
    // an atom fits an inline record when it has at most two terms and float32-exact
    // coefficients and right-hand side (the register message stores need every atom so)
    auto atom_inline_ok = [&](int k) {
        const int64_t e0 = a_ptr[k], e1 = a_ptr[k + 1];
        bool ok = (e1 - e0) <= 2 && (double)(float)a_rhs[k] == a_rhs[k] && std::isfinite((float)a_scale[k]);
        for (int64_t e = e0; e < e1 && ok; ++e) ok = (double)(float)a_coef[e] == a_coef[e];
        return ok;
    };
    // guarded disjunctions keep their atoms in inline records (every atom of every member
    // must qualify, else the template takes the generic passes). The template's form holds
    // each atom slot's coefficients, scale and flags, which must be the same in every member
    // (the closed form streams only variables and right-hand sides); a two-variable atom may
    // list its variables in either order to match (q.y is a sum of two exact FP64 products,
    // so the order does not change it). The run flags record which consecutive atom slots
    // share variables (and coefficients) in every member, in that matched order.
    std::vector<GdForm> gd_form(T);
    struct Canon { int32_t v0, v1; float c0, c1, sc; uint32_t fl; };
    auto canon = [&](int k) {
        const int64_t e0 = a_ptr[k];
        const bool two = a_ptr[k + 1] - e0 == 2;
        return Canon{a_var[e0], two ? a_var[e0 + 1] : a_var[e0], (float)a_coef[e0], two ? (float)a_coef[e0 + 1] : 0.0f,
                     (float)a_scale[k], (a_strict[k] ? 1u : 0u) | (two ? 2u : 0u)};
    };
    auto matches = [](const GdForm &F, int j, Canon &a) {   // swaps a's terms if that matches
        const uint32_t fl = ((F.flags >> j) & 1u) | (((F.flags >> (8 + j)) & 1u) << 1);
        if (a.fl != fl || a.sc != F.scale[j]) return false;
        if (a.c0 == F.c0[j] && a.c1 == F.c1[j]) return true;
        if ((a.fl & 2u) && a.c1 == F.c0[j] && a.c0 == F.c1[j]) {
            std::swap(a.v0, a.v1);
            std::swap(a.c0, a.c1);
            return true;
        }
        return false;
    };
    for (int t = 0; t < T; ++t) {
        Template &tp = tpls[t];
        gd_form[t] = GdForm{};
        gd_form[t].srec_base = -1;
        if (tp.gd.k < 0 || members[t].empty()) continue;
        const int nb = tp.n_bslots, na = tp.n_slots - tp.n_bslots;
        GdForm &F = gd_form[t];
        {
            // a two-variable atom on the previous slot's variables in the other order takes
            // that order (its coefficients swapped with them), so the two slots form one run
            // of the closed form's reads and scatter (a rectangle pair's x_i + w <= x_j and
            // x_j + w' <= x_i); the other members are matched to these forms term by term
            const int32_t *ids0 = con_ids.data() + con_sup_off[members[t][0]];
            Canon prev{};
            for (int j = 0; j < na; ++j) {
                Canon a = canon(ids0[nb + j] - n);
                if (j > 0 && (a.fl & 2u) && (prev.fl & 2u) && a.v0 != a.v1 && a.v0 == prev.v1 && a.v1 == prev.v0) {
                    std::swap(a.v0, a.v1);
                    std::swap(a.c0, a.c1);
                }
                prev = a;
                F.c0[j] = a.c0;
                F.c1[j] = a.c1;
                F.scale[j] = a.sc;
                F.flags |= ((a.fl & 1u) << j) | (((a.fl >> 1) & 1u) << (8 + j));
            }
        }
        bool ok = true;
        uint32_t same_vars = 0;
        for (int j = 1; j < na; ++j) same_vars |= 1u << j;
        for (int c : members[t]) {
            const int32_t *ids = con_ids.data() + con_sup_off[c];
            Canon prev{};
            for (int j = 0; j < na && ok; ++j) {
                const int kj = ids[nb + j] - n;
                Canon a = canon(kj);
                ok = atom_inline_ok(kj) && matches(F, j, a);
                if (ok && j > 0 && !(a.v0 == prev.v0 && a.v1 == prev.v1 && (a.fl & 2u) == (prev.fl & 2u)))
                    same_vars &= ~(1u << j);
                prev = a;
            }
            if (!ok) break;
        }
        if (!ok) {
            tp.gd.k = -1;
            continue;
        }
        uint32_t same_lin = same_vars;
        for (int j = 1; j < na; ++j)
            if (F.c0[j] != F.c0[j - 1] || F.c1[j] != F.c1[j - 1]) same_lin &= ~(1u << j);
        tp.gd.same_vars = same_vars;
        tp.gd.same_lin = same_lin;
    }
    std::vector<TplInfo> tinfo(T);
    std::vector<GdInfo> gd_rec(T);
    std::vector<Node> nodes;
    std::vector<int32_t> lev;   // level starts: nodes are sorted by slot, so each level is a range
    for (int t = 0; t < T; ++t) {
        const Template &tp = tpls[t];
        tinfo[t] = TplInfo{(int32_t)nodes.size(), tp.n_nodes, tp.n_slots, tp.n_bslots, tp.root, (int32_t)lev.size(),
                           {tp.pair_l > 0 ? tp.pair_l : (tp.gd.k >= 0 ? -1 : 0), 0}};
        gd_rec[t] = tp.gd;
        int v = 0;
        for (int sl = 0; sl <= tp.n_slots; ++sl) {
            while (v < tp.n_nodes && tp.nodes[v].slot < sl) ++v;
            lev.push_back(v);
        }
        nodes.insert(nodes.end(), tp.nodes.begin(), tp.nodes.end());
        h->max_nodes = std::max(h->max_nodes, tp.n_nodes);
        h->max_slots = std::max(h->max_slots, tp.n_slots);
        if (members[t].empty()) continue;
        if (tp.pair_l > 0) {
            h->n_pair += (int64_t)members[t].size();   // closed form: no message store, never big
        } else if (tp.gd.k >= 0) {
            h->n_gd += (int64_t)members[t].size();     // likewise
            if (tp.gd.sep) h->n_gd_sep += (int64_t)members[t].size();
            h->gd_level = std::max(h->gd_level, gd_level_of(tp.n_bslots, tp.n_slots - tp.n_bslots));
        } else if (big_diagram(tp.n_nodes, tp.n_slots)) {
            h->big_max_nodes = std::max(h->big_max_nodes, tp.n_nodes);
            h->big_max_slots = std::max(h->big_max_slots, tp.n_slots);
        } else {
            h->small_max_nodes = std::max(h->small_max_nodes, tp.n_nodes);
            h->small_max_slots = std::max(h->small_max_slots, tp.n_slots);
        }
    }
    std::vector<BucketInfo> buckets;
    std::vector<int32_t> bstart{0}, pos_con, con_bucket(C), con_local(C), sup, big_pos;
    for (int t = 0; t < T; ++t) {
        if (members[t].empty()) continue;
        const int nc = (int)members[t].size();
        const int npos = (nc + 63) / 64 * 64;
        const int ns = tpls[t].n_slots;
        const TplInfo &ti = tinfo[t];
        const int big = (ti.pad[0] == 0 && big_diagram(ti.n_nodes, ti.n_slots)) ? 1 : 0;
        BucketInfo bi{t, bstart.back(), npos, nc, (int64_t)sup.size(), -1, ti.node_off, ti.n_nodes, ti.n_slots,
                      ti.n_bslots, ti.root, ti.lev_off, big, ti.pad[0]};
        const int b_id = (int)buckets.size();
        sup.resize(sup.size() + (size_t)ns * npos, 0);
        for (int i = 0; i < npos; ++i) {
            int c = i < nc ? members[t][i] : -1;
            pos_con.push_back(c);
            if (c < 0) continue;
            con_bucket[c] = b_id;
            con_local[c] = i;
            if (big) big_pos.push_back(bstart.back() + i);
            for (int s = 0; s < ns; ++s) sup[bi.sup_base + (int64_t)s * npos + i] = con_ids[con_sup_off[c] + s];
            h->total_nodes += tpls[t].n_nodes;
        }
        if ((int64_t)bstart.back() + npos > INT32_MAX) { release(h); return set_error(FSMT_ELIMIT, "too many constraints"); }
        bstart.push_back(bstart.back() + npos);
        buckets.push_back(bi);
    }
    // inline atom records for buckets whose atoms all qualify
    std::vector<AtomRec> arec;
    std::vector<SlimRec> srec;
    bool all_inline = true;
    for (BucketInfo &bi : buckets) {
        const int na = bi.n_slots - bi.n_bslots;
        if (na == 0) continue;
        bool ok = true;
        for (int i = 0; i < bi.n_con && ok; ++i)
            for (int s = bi.n_bslots; s < bi.n_slots && ok; ++s) {
                ok = atom_inline_ok(sup[bi.sup_base + (int64_t)s * bi.n_pos + i] - n);
            }
        if (!ok) {
            all_inline = false;
            continue;
        }
        bi.arec_base = (int64_t)arec.size();
        arec.resize(arec.size() + (size_t)na * bi.n_pos, AtomRec{0, 0, 0.0f, 0.0f, 0.0f, 0.0f, 0, 0u});
        for (int i = 0; i < bi.n_con; ++i)
            for (int s = bi.n_bslots; s < bi.n_slots; ++s) {
                const int k = sup[bi.sup_base + (int64_t)s * bi.n_pos + i] - n;
                const int e0 = a_ptr[k], e1 = a_ptr[k + 1];
                AtomRec &rr = arec[bi.arec_base + (int64_t)(s - bi.n_bslots) * bi.n_pos + i];
                rr.v0 = a_var[e0];
                rr.c0 = (float)a_coef[e0];
                rr.v1 = (e1 - e0 == 2) ? a_var[e0 + 1] : a_var[e0];
                rr.c1 = (e1 - e0 == 2) ? (float)a_coef[e0 + 1] : 0.0f;
                rr.rhs = (float)a_rhs[k];
                rr.scale = (float)a_scale[k];
                rr.atom = k;
                rr.flags = (a_strict[k] ? 1u : 0u) | ((e1 - e0 == 2) ? 2u : 0u);
            }
        if (bi.pad < 0) {
            // guarded disjunction: both record kinds list a two-variable atom's terms in the
            // order that matches the template's form (the run flags were found in that
            // order), plus the slim copies (padding positions name variable 0)
            GdForm &F = gd_form[bi.tpl];
            F.srec_base = (int64_t)srec.size();
            srec.resize(srec.size() + (size_t)na * bi.n_pos, SlimRec{0, 0, 0.0f});
            for (int s = 0; s < na; ++s)
                for (int i = 0; i < bi.n_con; ++i) {
                    const int k = sup[bi.sup_base + (int64_t)(bi.n_bslots + s) * bi.n_pos + i] - n;
                    Canon a = canon(k);
                    (void)matches(F, s, a);   // holds for every member (checked above)
                    AtomRec &rr = arec[bi.arec_base + (int64_t)s * bi.n_pos + i];
                    rr.v0 = a.v0;
                    rr.v1 = a.v1;
                    rr.c0 = a.c0;
                    rr.c1 = a.c1;
                    srec[F.srec_base + (int64_t)s * bi.n_pos + i] = SlimRec{a.v0, a.v1, (float)a_rhs[k]};
                }
        }
    }
    std::vector<int32_t> task_bucket((size_t)bstart.back() / 64);
    for (size_t b = 0; b < buckets.size(); ++b)
        for (int q = bstart[b] / 64; q < bstart[b + 1] / 64; ++q) task_bucket[q] = (int32_t)b;
    h->n_buckets = (int)buckets.size();
    h->n_pos = bstart.back();
    h->h_tpl = tinfo;
    h->h_bucket = buckets;
    h->h_bucket_start = bstart;
    h->h_nodes = nodes;
    h->h_sup = sup;
    h->h_con_bucket = con_bucket;
    h->h_con_local = con_local;
    h->host_only = host_only;
    h->lds_messages = opts && opts->messages == FSMT_MSG_LDS;

    // ---- feasible set of the projection (Def. "Projection", Prop. "qp"): the box, plus
    // unit atomic constraints (one atom literal, no Boolean) when requested.
    std::vector<float> lo(m), hi(m);
    for (int j = 0; j < m; ++j) {
        lo[j] = (float)P->real_lo[j];
        hi[j] = (float)P->real_hi[j];
    }
    std::vector<int32_t> hs_ptr{0}, hs_var;
    std::vector<float> hs_coef, hs_rhs, hs_inv;
    const bool unit_proj = !(opts && opts->projection == FSMT_PROJ_BOX);
    for (int c = 0; c < C && unit_proj; ++c) {
        if (P->con_kind[c] != FSMT_CLAUSE && P->con_kind[c] != FSMT_AND) continue;
        if (P->con_ptr[c + 1] - P->con_ptr[c] != 1) continue;
        const int32_t lit = P->con_lit[P->con_ptr[c]];
        if ((lit >> 1) < n) continue;
        const int k = (lit >> 1) - n;
        const bool want = (lit & 1) == 0;                 // the atom must hold (else its negation)
        const int e0 = a_ptr[k], e1 = a_ptr[k + 1];
        const bool strict = a_strict[k] != 0;
        auto holds = [&](float f) {                        // the exact test of the check
            const double z = (0.0 + a_coef[e0] * (double)f) - a_rhs[k];
            const bool t = strict ? (z < 0.0) : (z <= 0.0);
            return t == want;
        };
        if (e1 - e0 == 1) {
            const int j = a_var[e0];
            const double q = a_coef[e0];
            // the atom holds for y <= q0/q (q > 0, want) or y >= q0/q, flipped by negation
            const bool upper = (q > 0.0) == want;
            float f = (float)(a_rhs[k] / q);
            for (int it = 0; it < 8 && !holds(f); ++it) f = nextafterf(f, upper ? -INFINITY : INFINITY);
            if (!holds(f)) continue;
            const float nlo = upper ? lo[j] : std::max(lo[j], f);
            const float nhi = upper ? std::min(hi[j], f) : hi[j];
            if (!(nlo <= nhi)) continue;                   // empty: leave the atom soft
            lo[j] = nlo;
            hi[j] = nhi;
            ++h_box_units;
        } else {
            const double sg = want ? 1.0 : -1.0;
            double scale = std::fabs(a_rhs[k]), q2 = 0.0;
            for (int e = e0; e < e1; ++e) {
                const int j = a_var[e];
                scale += std::fabs(a_coef[e]) * std::max(std::fabs(P->real_lo[j]), std::fabs(P->real_hi[j]));
                hs_var.push_back(j);
                hs_coef.push_back((float)(sg * a_coef[e]));
                q2 += a_coef[e] * a_coef[e];
            }
            hs_rhs.push_back((float)(sg * a_rhs[k] - 1e-6 * scale));
            hs_inv.push_back((float)(1.0 / q2));
            hs_ptr.push_back((int32_t)hs_var.size());
        }
    }

    // colour classes of the half-spaces (greedy, in order): no two half-spaces of a class
    // share a variable, so projecting onto a class is projecting onto each of its members
    // independently, and Dykstra's method runs over the classes with the members of a class
    // on parallel lanes. Half-spaces are stored class by class; hs_cstart[k] is the first
    // of class k.
    std::vector<int32_t> hs_cstart{0};
    {
        const int H = (int)hs_rhs.size();
        std::vector<int32_t> color(H, 0);
        std::vector<std::vector<int32_t>> var_colors(m);
        int n_colors = 0;
        std::vector<char> used;
        for (int t = 0; t < H; ++t) {
            used.assign((size_t)n_colors + 1, 0);
            for (int e = hs_ptr[t]; e < hs_ptr[t + 1]; ++e)
                for (int32_t k : var_colors[hs_var[e]]) used[k] = 1;
            int k = 0;
            while (used[k]) ++k;
            color[t] = k;
            n_colors = std::max(n_colors, k + 1);
            for (int e = hs_ptr[t]; e < hs_ptr[t + 1]; ++e) var_colors[hs_var[e]].push_back(k);
        }
        std::vector<int32_t> order(H);
        for (int t = 0; t < H; ++t) order[t] = t;
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return color[x] < color[y]; });
        std::vector<int32_t> p2{0}, v2;
        std::vector<float> c2, r2, i2;
        for (int q = 0; q < H; ++q) {
            const int t = order[q];
            for (int e = hs_ptr[t]; e < hs_ptr[t + 1]; ++e) {
                v2.push_back(hs_var[e]);
                c2.push_back(hs_coef[e]);
            }
            p2.push_back((int32_t)v2.size());
            r2.push_back(hs_rhs[t]);
            i2.push_back(hs_inv[t]);
            if (q + 1 == H || color[order[q + 1]] != color[t]) hs_cstart.push_back(q + 1);
        }
        hs_ptr.swap(p2);
        hs_var.swap(v2);
        hs_coef.swap(c2);
        hs_rhs.swap(r2);
        hs_inv.swap(i2);
    }

    h->n_box_units = h_box_units;
    h->n_hs_colors = (int)hs_cstart.size() - 1;
    // half-spaces on disjoint variables, each over a few distinct variables: the projection
    // separates into one exact problem per half-space (the kernels' closed form)
    h->hs_separable = h->n_hs_colors == 1;
    for (size_t t = 0; h->hs_separable && t + 1 < hs_ptr.size(); ++t) {
        const int e0 = hs_ptr[t], e1 = hs_ptr[t + 1];
        if (e1 - e0 > kSeparableRowMax) h->hs_separable = 0;
        for (int e = e0; e < e1 && h->hs_separable; ++e)
            for (int f = e0; f < e; ++f)
                if (hs_var[f] == hs_var[e]) h->hs_separable = 0;
    }
    h->n_big = (int)big_pos.size();
    h->n_hs = (int)hs_rhs.size();
    h->hs_nnz = (int)hs_var.size();
    if (host_only) {
        *out = h;
        return FSMT_OK;
    }

    // ---- upload
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
        release(h);
        return set_error(FSMT_EHIP, "cannot select device %d", device);
    }
    Uploader U{h};
    fsmt_status rc = FSMT_OK;
    if (!rc) rc = U.put(&h->d.tpl, tinfo, "templates");
    if (!rc) rc = U.put(&h->d.nodes, nodes, "nodes");
    if (!rc) rc = U.put(&h->d.bucket, buckets, "buckets");
    if (!rc) rc = U.put(&h->d.bucket_start, bstart, "bucket starts");
    if (!rc) rc = U.put(&h->d.task_bucket, task_bucket, "task buckets");
    if (!rc) rc = U.put(&h->d.arec, arec, "inline atom records");
    if (!rc) rc = U.put(&h->d.pos_con, pos_con, "positions");
    if (!rc) rc = U.put(&h->d.sup, sup, "supports");
    if (!rc) rc = U.put(&h->d.con_bucket, con_bucket, "constraint buckets");
    if (!rc) rc = U.put(&h->d.con_local, con_local, "constraint positions");
    if (!rc) rc = U.put(&h->d.lev, lev, "level starts");
    if (!rc) rc = U.put(&h->d.big_pos, big_pos, "big-diagram positions");
    if (!rc) rc = U.put(&h->d.gd, gd_rec, "guarded disjunctions");
    if (!rc) rc = U.put(&h->d.gdf, gd_form, "guarded-disjunction forms");
    if (!rc) rc = U.put(&h->d.srec, srec, "slim atom records");
    h->all_inline = all_inline;
    if (all_inline) {   // every atom is reached through its inline record
        a_ptr.assign(1, 0);
        a_var.clear();
        a_coef.clear();
        a_rhs.clear();
        a_scale.clear();
        a_strict.clear();
    }
    if (!rc) rc = U.put(&h->d.atom_ptr, a_ptr, "atom offsets");
    if (!rc) rc = U.put(&h->d.atom_var, a_var, "atom variables");
    if (!rc) rc = U.put(&h->d.atom_coef, a_coef, "atom coefficients");
    if (!rc) rc = U.put(&h->d.atom_rhs, a_rhs, "atom rhs");
    if (!rc) rc = U.put(&h->d.atom_scale, a_scale, "atom scales");
    if (!rc) rc = U.put(&h->d.atom_strict, a_strict, "atom flags");
    if (!rc) rc = U.put(&h->d.real_lo, lo, "box lo");
    if (!rc) rc = U.put(&h->d.real_hi, hi, "box hi");
    if (!rc) rc = U.put(&h->d.hs_ptr, hs_ptr, "half-space offsets");
    if (!rc) rc = U.put(&h->d.hs_var, hs_var, "half-space variables");
    if (!rc) rc = U.put(&h->d.hs_coef, hs_coef, "half-space coefficients");
    if (!rc) rc = U.put(&h->d.hs_rhs, hs_rhs, "half-space rhs");
    if (!rc) rc = U.put(&h->d.hs_inv, hs_inv, "half-space norms");
    if (!rc) rc = U.put(&h->d.hs_cstart, hs_cstart, "half-space colour classes");
    (void)hipSetDevice(prev);
    if (rc) {
        release(h);
        return rc;
    }
    *out = h;
    return FSMT_OK;
}

}  // namespace fsmt

extern "C" {

const char *fsmt_last_error(void) { return fsmt::last_error(); }

fsmt_status xbdd_compile(const fsmt_problem *problem, const fsmt_compile_opts *opts, fsmt_xbdd **out) {
    fsmt::clear_error();
    try {
        return fsmt::compile_impl(problem, opts, out);
    } catch (const std::bad_alloc &) {
        return fsmt::set_error(FSMT_ENOMEM, "out of host memory during compile");
    } catch (...) {
        return fsmt::set_error(FSMT_EINVAL, "unexpected exception during compile");
    }
}

void xbdd_free(fsmt_xbdd *h) { fsmt::release(h); }

fsmt_status xbdd_info(const fsmt_xbdd *h, fsmt_xbdd_stats *s) {
    fsmt::clear_error();
    if (!h || !s) return fsmt::set_error(FSMT_EINVAL, "null handle or stats");
    s->n_bool = h->n_bool;
    s->n_real = h->n_real;
    s->n_atoms = h->n_atoms;
    s->n_cons = h->n_cons;
    s->total_nodes = h->total_nodes;
    s->n_templates = h->n_tpl;
    s->max_nodes = h->max_nodes;
    s->max_slots = h->max_slots;
    s->n_big = h->n_big;
    s->n_hs_colors = h->n_hs_colors;
    s->n_pair = (int32_t)h->n_pair;
    s->hs_separable = h->hs_separable;
    s->n_gd = (int32_t)h->n_gd;
    s->n_gd_sep = (int32_t)h->n_gd_sep;
    s->n_positions = h->n_pos;
    s->table_bytes = h->table_bytes;
    s->atom_nnz = h->nnz;
    s->n_box_units = h->n_box_units;
    s->n_halfspaces = h->n_hs;
    return FSMT_OK;
}

fsmt_status xbdd_export_diagram(const fsmt_xbdd *h, int32_t c, int32_t max_nodes, int32_t max_slots,
                                int32_t *n_nodes, int32_t *n_slots, int32_t *n_bslots, int32_t *root,
                                int32_t *nodes, int32_t *support) {
    fsmt::clear_error();
    if (!h || !n_nodes || !n_slots || !n_bslots || !root || !nodes || !support)
        return fsmt::set_error(FSMT_EINVAL, "null argument");
    if (c < 0 || c >= h->n_cons) return fsmt::set_error(FSMT_EINVAL, "constraint %d out of range", c);
    const fsmt::BucketInfo &B = h->h_bucket[h->h_con_bucket[c]];
    const fsmt::TplInfo &T = h->h_tpl[B.tpl];
    if (T.n_nodes > max_nodes || T.n_slots > max_slots)
        return fsmt::set_error(FSMT_ELIMIT, "diagram has %d nodes and %d slots", T.n_nodes, T.n_slots);
    *n_nodes = T.n_nodes;
    *n_slots = T.n_slots;
    *n_bslots = T.n_bslots;
    *root = T.root;
    for (int v = 0; v < T.n_nodes; ++v) {
        const fsmt::Node &x = h->h_nodes[T.node_off + v];
        nodes[3 * v] = x.slot;
        nodes[3 * v + 1] = x.hi;
        nodes[3 * v + 2] = x.lo;
    }
    const int local = h->h_con_local[c];
    for (int s = 0; s < T.n_slots; ++s) support[s] = h->h_sup[B.sup_base + (int64_t)s * B.n_pos + local];
    return FSMT_OK;
}

}  // extern "C"
